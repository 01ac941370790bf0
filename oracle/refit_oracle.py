"""Float64 CPU oracle of the helix refit -- TEST INFRASTRUCTURE ONLY.

The refit takes one track candidate's hits (r, z on vane k, the radial plane
at azimuth 2 pi k / n_vanes) and fits a helix in a uniform axial field. The
paper fits its seeds with a Kalman filter (Genfit2, Sec. 3) and names a GPU
fit as future work (Sec. 8); the fit here is the one the benchmark workload
asks for: the float32 chi^2 of the hit residuals (sigma 0.055 mm in r and z,
the strip pitch over sqrt(12)) minimised by Gauss-Newton steps.

Parameters p = (kappa, phi0, d0, z0, tan_lambda) in the perigee form:

* the circle has signed radius rs = 1 / kappa (kappa > 0: clockwise seen from
  +z, the turning of a positive charge in a field along +z);
* n = (sin phi0, -cos phi0) is the right-hand normal of the direction of
  motion (cos phi0, sin phi0) at the perigee P0 = d0 n (the circle's point
  nearest the z axis), and the centre is c = (d0 + rs) n;
* a point at turning angle a (clockwise for kappa > 0) past the perigee has
  z = z0 + R a tan_lambda, R = |rs|.

Prediction of hit i on vane k (unit ray u_k): the crossing of the circle with
the ray, t = b + s_i sqrt(b^2 - d0 (d0 + 2 rs)), b = u_k . c, where the root
s_i = +-1 is fixed at the initial parameters (the one nearest the measured r);
r_hat = t, and z_hat from the turning angle of the crossing, unwrapped against
its value at the initial parameters (so the turn is fixed too). When the ray
misses the circle (negative discriminant) the square root is taken as 0.

Initial parameters: an algebraic circle fit (the Kasa fit: linear least squares
of x^2 + y^2 + D x + E y + F = 0 over the measured points), kappa > 0; the
measured points' turning angles unwrapped along the track (unwrap_turning);
a straight-line fit of z against the arc length R a.

Gauss-Newton step: J the Jacobian of the residual vector e (2 per hit), H =
J^T J, g = J^T e; with D = diag(H), p += -D^-1/2 (D^-1/2 H D^-1/2 + mu I)^-1
D^-1/2 g, mu = 1e-3 (a fixed Levenberg-Marquardt damping, no step control).

The Jacobian and the gradient here come from torch's float64 autograd of the
residual function written out above; the library's kernels use hand-derived
derivatives, so the two are independent.
"""
from __future__ import annotations

import math

import numpy as np
import torch

SIGMA_MM = 0.055
N_VANES = 40
B_TESLA = 3.0
MEV_PER_T_MM = 0.299792458      # pT[MeV/c] = 0.299792458 * B[T] * R[mm]
GN_STEPS = 20
GN_DAMPING = 1e-3
Z_ORDER_MM = 1.0                 # z spread above which the hits are unwrapped in z order
R_MAX_MM = 1.0e4                 # larger initial circles are lines, not helices (p > 9 GeV/c at 3 T)


def vane_dirs(vane, n_vanes: int = N_VANES):
    phi = 2.0 * math.pi * np.asarray(vane, np.float64) / n_vanes
    return np.cos(phi), np.sin(phi)


def unwrap_turning(alpha, z):
    """Turning angles along the track from their values in (-pi, pi].

    z is monotone in the turning angle along a helix, so when the hits' z
    spread is at least Z_ORDER_MM the hits are walked in z order (ascending,
    or descending: whichever turns less in total; ties in z by hit order) and
    each step adds the angle advanced, in [0, 2 pi). Flatter tracks take the
    arc between the two sides of the largest angular gap (at most one turn).
    Either way the smallest unwrapped angle is the hit's own value."""
    alpha = np.asarray(alpha, np.float64)
    z = np.asarray(z, np.float64)
    n = len(alpha)
    if z.max() - z.min() >= Z_ORDER_MM:
        best = None
        for order in (np.argsort(z, kind="stable"), np.argsort(-z, kind="stable")):
            steps = np.mod(np.diff(alpha[order]), 2.0 * math.pi)
            a = np.empty(n)
            a[order] = alpha[order[0]] + np.concatenate([[0.0], np.cumsum(steps)])
            if best is None or steps.sum() < best[0]:
                best = (steps.sum(), a)
        return best[1]
    srt = np.sort(alpha, kind="stable")
    gaps = np.append(np.diff(srt), srt[0] + 2.0 * math.pi - srt[-1])
    g = int(np.argmax(gaps))
    a_start = srt[(g + 1) % n]
    return a_start + np.mod(alpha - a_start, 2.0 * math.pi)


def refit_init(r, z, vane, n_vanes: int = N_VANES):
    """(params (5,), root sign s (n,), reference turning angle a_ref (n,))
    from the measured hits of one candidate, in float64; params is None for a
    candidate no helix is fitted to (fewer than 3 hits or 3 distinct vanes,
    a singular circle system (exactly collinear points), or a circle of
    radius above R_MAX_MM: hits along a line, not a helix)."""
    if len(r) < 3 or len(set(np.asarray(vane).tolist())) < 3:
        return None, np.ones(len(r)), np.zeros(len(r))
    r = np.asarray(r, np.float64)
    z = np.asarray(z, np.float64)
    ux, uy = vane_dirs(vane, n_vanes)
    x, y = r * ux, r * uy
    xm, ym = x.mean(), y.mean()
    u, v = x - xm, y - ym
    w = u * u + v * v
    A = np.array([[np.dot(u, u), np.dot(u, v), u.sum()],
                  [np.dot(u, v), np.dot(v, v), v.sum()],
                  [u.sum(), v.sum(), float(len(u))]])
    rhs = -np.array([np.dot(u, w), np.dot(v, w), w.sum()])
    try:
        D, E, F = np.linalg.solve(A, rhs)
    except np.linalg.LinAlgError:      # exactly collinear points: no circle at all
        return None, np.ones(len(r)), np.zeros(len(r))
    cx, cy = xm - D / 2.0, ym - E / 2.0
    R2 = D * D / 4.0 + E * E / 4.0 - F
    cn = math.hypot(cx, cy)
    if not (R2 > 0.0) or not (cn > 0.0) or math.sqrt(R2) > R_MAX_MM:
        return None, np.ones(len(r)), np.zeros(len(r))
    R = math.sqrt(R2)
    kappa = 1.0 / R
    nx, ny = cx / cn, cy / cn
    d0 = cn - R
    phi0 = math.atan2(nx, -ny)
    # turning angles of the measured points past the perigee (clockwise)
    v0x, v0y = -R * nx, -R * ny
    vx, vy = x - cx, y - cy
    alpha = -np.arctan2(v0x * vy - v0y * vx, v0x * vx + v0y * vy)
    a = unwrap_turning(alpha, z)
    s = R * a
    sm, zm = s.mean(), z.mean()
    den = np.dot(s - sm, s - sm)
    tl = np.dot(s - sm, z - zm) / den if den > 0.0 else 0.0
    z0 = zm - tl * sm
    # root of each hit at the initial circle: the one nearest the measured r
    b = ux * (d0 + R) * nx + uy * (d0 + R) * ny
    disc = b * b - d0 * (d0 + 2.0 * R)
    sq = np.sqrt(np.maximum(disc, 0.0))
    sign = np.where(np.abs(b + sq - r) <= np.abs(b - sq - r), 1.0, -1.0)
    return np.array([kappa, phi0, d0, z0, tl]), sign, a


def refit_residuals(p, r, z, vane, sign, aref, sigma: float = SIGMA_MM, n_vanes: int = N_VANES):
    """Residual vector ((r - r_hat) / sigma, (z - z_hat) / sigma) of one
    candidate (torch float64, differentiable in p)."""
    p = torch.as_tensor(p, dtype=torch.float64)
    kappa, phi0, d0, z0, tl = p[0], p[1], p[2], p[3], p[4]
    ux, uy = (torch.as_tensor(a, dtype=torch.float64) for a in vane_dirs(vane, n_vanes))
    r = torch.as_tensor(np.asarray(r, np.float64))
    z = torch.as_tensor(np.asarray(z, np.float64))
    sign = torch.as_tensor(np.asarray(sign, np.float64))
    aref = torch.as_tensor(np.asarray(aref, np.float64))
    rs = 1.0 / kappa
    nx, ny = torch.sin(phi0), -torch.cos(phi0)
    cx, cy = (d0 + rs) * nx, (d0 + rs) * ny
    b = ux * cx + uy * cy
    disc = b * b - d0 * (d0 + 2.0 * rs)
    sq = torch.where(disc > 0, torch.sqrt(torch.clamp(disc, min=1e-300)), torch.zeros_like(disc))
    t = b + sign * sq
    v0x, v0y = -rs * nx, -rs * ny
    vx, vy = t * ux - cx, t * uy - cy
    alpha = -torch.sign(kappa) * torch.atan2(v0x * vy - v0y * vx, v0x * vx + v0y * vy)
    a = aref + torch.remainder(alpha - aref + math.pi, 2.0 * math.pi) - math.pi
    zhat = z0 + torch.abs(rs) * a * tl
    return torch.cat([(r - t) / sigma, (z - zhat) / sigma])


def refit_chi2(p, r, z, vane, sign, aref, sigma: float = SIGMA_MM) -> float:
    e = refit_residuals(p, r, z, vane, sign, aref, sigma)
    return float(torch.dot(e, e))


def refit_grad(p, r, z, vane, sign, aref, sigma: float = SIGMA_MM) -> np.ndarray:
    """d chi^2 / d p by float64 autograd."""
    pt = torch.tensor(np.asarray(p, np.float64), requires_grad=True)
    e = refit_residuals(pt, r, z, vane, sign, aref, sigma)
    (g,) = torch.autograd.grad(torch.dot(e, e), pt)
    return g.numpy()


def refit_gn(p0, r, z, vane, sign, aref, steps: int = GN_STEPS, mu: float = GN_DAMPING,
             sigma: float = SIGMA_MM) -> np.ndarray:
    """Parameters after `steps` damped, scaled Gauss-Newton steps."""
    p = np.asarray(p0, np.float64).copy()
    for _ in range(steps):
        f = lambda q: refit_residuals(q, r, z, vane, sign, aref, sigma)
        pt = torch.tensor(p)
        e = f(pt).numpy()
        J = torch.autograd.functional.jacobian(f, pt).numpy()
        H = J.T @ J
        g = J.T @ e
        d = np.sqrt(np.diag(H))
        d = np.where(d > 0.0, d, 1.0)
        Hs = H / np.outer(d, d) + mu * np.eye(5)
        y = np.linalg.solve(Hs, -g / d)
        q = p + y / d
        if not np.all(np.isfinite(q)):
            break
        p = q
    return p


def refit_candidate(r, z, vane, steps: int = GN_STEPS):
    """(initial params, fitted params, sign, aref) of one candidate (params
    None when no helix is fitted)."""
    p0, sign, aref = refit_init(r, z, vane)
    if p0 is None:
        return None, None, sign, aref
    return p0, refit_gn(p0, r, z, vane, sign, aref, steps), sign, aref


def momentum_mev(p) -> float:
    """|p| in MeV/c of fitted parameters in the 3 T field."""
    pt = MEV_PER_T_MM * B_TESLA / abs(p[0])
    return pt * math.sqrt(1.0 + p[4] * p[4])


def truth_params(phi_start, z_start, pt, tan_lambda, beta):
    """Perigee parameters of a generated positron (start point on the orbit
    of radius 333 mm at azimuth phi_start, transverse direction beta, clockwise
    turning): the same helix in this parametrisation."""
    R = pt / (MEV_PER_T_MM * B_TESLA)
    x0, y0 = 333.0 * math.cos(phi_start), 333.0 * math.sin(phi_start)
    cx, cy = x0 + R * math.sin(beta), y0 - R * math.cos(beta)
    cn = math.hypot(cx, cy)
    nx, ny = cx / cn, cy / cn
    d0 = cn - R
    phi0 = math.atan2(nx, -ny)
    # turning angle from the perigee to the start point, in (-pi, pi]
    v0x, v0y = -R * nx, -R * ny
    vx, vy = x0 - cx, y0 - cy
    a_start = -math.atan2(v0x * vy - v0y * vx, v0x * vx + v0y * vy)
    z0 = z_start - R * a_start * tan_lambda
    return np.array([1.0 / R, phi0, d0, z0, tan_lambda])
