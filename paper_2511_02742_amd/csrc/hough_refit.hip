// Helix refit of track candidates: initial parameters, the chi^2 of the hit
// residuals, its adjoint (gradient) and damped Gauss-Newton steps.
//
// One thread per candidate (a candidate holds a few to a few tens of hits):
// the work per candidate is small and independent, the hits of a candidate
// are contiguous, and a thread keeps the 5 parameters, the 5 x 5 normal
// matrix and the gradient in registers. The initial fit runs in float64 (it
// takes discrete decisions: the order of the hits along the track and the root
// of each vane crossing); the chi^2, the adjoint and the Gauss-Newton steps run
// in float32.
//
// Model (perigee parameters p = (kappa, phi0, d0, z0, tan_lambda)): signed
// radius rs = 1 / kappa, normal n = (sin phi0, -cos phi0), centre
// c = (d0 + rs) n. Hit i on vane k (unit ray u_k) is predicted at the ray's
// crossing t = b + s_i sqrt(b^2 - d0 (d0 + 2 rs)), b = u_k . c (square root 0
// when the ray misses the circle), and at z = z0 + |rs| a tan_lambda with a the
// crossing's turning angle past the perigee, unwrapped against a_ref_i. The
// residuals (r - t) / sigma and (z - z_hat) / sigma make the chi^2.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "hough_tf.h"

namespace hough {
namespace {

constexpr int kRefitThreads = 256;
constexpr int kMaxRefitHits = 128;   // hits per candidate the initial fit orders
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kZOrderMM = 1.0;    // z spread above which hits are ordered by z
constexpr double kRMaxMM = 1.0e4;    // larger initial circles are lines, not helices

struct RefitHits {
    int32_t n_cand;
    const int64_t *off;   // [n_cand + 1]
    const float *r, *z;
    const int16_t *vane;
    int32_t n_vanes;
};

// ---------------------------------------------------------------------------
// initial parameters (float64)
// ---------------------------------------------------------------------------

__device__ double wrap_2pi(double x) {   // into [0, 2 pi)
    double y = fmod(x, kTwoPi);
    return y < 0.0 ? y + kTwoPi : y;
}

// Parameters and per-hit state of a candidate no helix is fitted to.
__device__ void no_helix(float *P, float *sign, float *aref, int64_t b0, int n) {
    for (int q = 0; q < 5; ++q) P[q] = 0.0f;
    for (int i = 0; i < n; ++i) {
        sign[b0 + i] = 1.0f;
        aref[b0 + i] = 0.0f;
    }
}

__global__ __launch_bounds__(kRefitThreads) void k_refit_init(RefitHits H, float *params, float *sign, float *aref,
                                                             int32_t *status) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= H.n_cand) return;
    const int64_t b0 = H.off[c];
    const int n = (int)(H.off[c + 1] - b0);
    float *P = params + 5 * (size_t)c;
    // a helix needs hits on at least three vanes
    int distinct = 0;
    for (int i = 0; i < n && distinct < 3; ++i) {
        bool seen = false;
        for (int j = 0; j < i && !seen; ++j) seen = H.vane[b0 + j] == H.vane[b0 + i];
        distinct += seen ? 0 : 1;
    }
    if (n < 3 || n > kMaxRefitHits || distinct < 3) {
        no_helix(P, sign, aref, b0, n);
        status[c] = n < 3 ? 1 : n > kMaxRefitHits ? 2 : 3;
        return;
    }
    double x[kMaxRefitHits], y[kMaxRefitHits], al[kMaxRefitHits];
    double xm = 0.0, ym = 0.0;
    for (int i = 0; i < n; ++i) {
        const double ph = kTwoPi * (double)H.vane[b0 + i] / (double)H.n_vanes;
        const double rr = (double)H.r[b0 + i];
        x[i] = rr * cos(ph);
        y[i] = rr * sin(ph);
        xm += x[i];
        ym += y[i];
    }
    xm /= n;
    ym /= n;
    // algebraic circle fit: least squares of u^2 + v^2 + D u + E v + F = 0
    double suu = 0, suv = 0, svv = 0, su = 0, sv = 0, suw = 0, svw = 0, sw = 0;
    for (int i = 0; i < n; ++i) {
        const double u = x[i] - xm, v = y[i] - ym, w = u * u + v * v;
        suu += u * u;
        suv += u * v;
        svv += v * v;
        su += u;
        sv += v;
        suw += u * w;
        svw += v * w;
        sw += w;
    }
    // Gaussian elimination with partial pivoting of the 3 x 3 normal system
    double A[3][4] = {{suu, suv, su, -suw}, {suv, svv, sv, -svw}, {su, sv, (double)n, -sw}};
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int rrow = col + 1; rrow < 3; ++rrow)
            if (fabs(A[rrow][col]) > fabs(A[piv][col])) piv = rrow;
        if (piv != col)
            for (int k = 0; k < 4; ++k) {
                const double t = A[col][k];
                A[col][k] = A[piv][k];
                A[piv][k] = t;
            }
        if (A[col][col] == 0.0) {
            no_helix(P, sign, aref, b0, n);
            status[c] = 3;
            return;
        }
        for (int rrow = col + 1; rrow < 3; ++rrow) {
            const double f = A[rrow][col] / A[col][col];
            for (int k = col; k < 4; ++k) A[rrow][k] -= f * A[col][k];
        }
    }
    const double F = A[2][3] / A[2][2];
    const double E = (A[1][3] - A[1][2] * F) / A[1][1];
    const double D = (A[0][3] - A[0][1] * E - A[0][2] * F) / A[0][0];
    const double cx = xm - D / 2.0, cy = ym - E / 2.0;
    const double R2 = D * D / 4.0 + E * E / 4.0 - F;
    const double cn = sqrt(cx * cx + cy * cy);
    if (!(R2 > 0.0) || !(cn > 0.0) || sqrt(R2) > kRMaxMM) {
        no_helix(P, sign, aref, b0, n);
        status[c] = 3;
        return;
    }
    const double R = sqrt(R2);
    const double nx = cx / cn, ny = cy / cn;
    const double d0 = cn - R;
    const double phi0 = atan2(nx, -ny);
    // turning angles of the measured points past the perigee (clockwise)
    const double v0x = -R * nx, v0y = -R * ny;
    double zmin = 1e300, zmax = -1e300;
    for (int i = 0; i < n; ++i) {
        const double vx = x[i] - cx, vy = y[i] - cy;
        al[i] = -atan2(v0x * vy - v0y * vx, v0x * vx + v0y * vy);
        const double zz = (double)H.z[b0 + i];
        zmin = fmin(zmin, zz);
        zmax = fmax(zmax, zz);
    }
    // unwrap along the track (x[] reused for the unwrapped angles)
    double *a = x;
    if (zmax - zmin >= kZOrderMM) {
        // walk the hits in z order, ascending or descending, whichever turns
        // less in total; equal z in hit order
        int ord[kMaxRefitHits];
        double best_total = 0.0;
        for (int dir = 0; dir < 2; ++dir) {
            for (int i = 0; i < n; ++i) ord[i] = i;
            for (int i = 1; i < n; ++i) {   // stable insertion sort by (+-z)
                const int k = ord[i];
                const double zk = dir == 0 ? (double)H.z[b0 + k] : -(double)H.z[b0 + k];
                int j = i - 1;
                while (j >= 0) {
                    const double zj = dir == 0 ? (double)H.z[b0 + ord[j]] : -(double)H.z[b0 + ord[j]];
                    if (zj <= zk) break;
                    ord[j + 1] = ord[j];
                    --j;
                }
                ord[j + 1] = k;
            }
            double total = 0.0;
            for (int i = 1; i < n; ++i) total += wrap_2pi(al[ord[i]] - al[ord[i - 1]]);
            if (dir == 0 || total < best_total) {
                best_total = total;
                double acc = al[ord[0]];
                y[ord[0]] = acc;
                for (int i = 1; i < n; ++i) {
                    acc += wrap_2pi(al[ord[i]] - al[ord[i - 1]]);
                    y[ord[i]] = acc;
                }
            }
        }
        for (int i = 0; i < n; ++i) a[i] = y[i];
    } else {
        // the arc between the two sides of the largest angular gap
        int ord[kMaxRefitHits];
        for (int i = 0; i < n; ++i) ord[i] = i;
        for (int i = 1; i < n; ++i) {
            const int k = ord[i];
            int j = i - 1;
            while (j >= 0 && al[ord[j]] > al[k]) {
                ord[j + 1] = ord[j];
                --j;
            }
            ord[j + 1] = k;
        }
        int g = 0;
        double gmax = -1.0;
        for (int i = 0; i < n; ++i) {
            const double gap = i + 1 < n ? al[ord[i + 1]] - al[ord[i]] : al[ord[0]] + kTwoPi - al[ord[n - 1]];
            if (gap > gmax) {
                gmax = gap;
                g = i;
            }
        }
        const double a_start = al[ord[(g + 1) % n]];
        for (int i = 0; i < n; ++i) a[i] = a_start + wrap_2pi(al[i] - a_start);
    }
    // z against the arc length R a
    double sm = 0.0, zm = 0.0;
    for (int i = 0; i < n; ++i) {
        sm += R * a[i];
        zm += (double)H.z[b0 + i];
    }
    sm /= n;
    zm /= n;
    double sxz = 0.0, sxx = 0.0;
    for (int i = 0; i < n; ++i) {
        const double ds = R * a[i] - sm;
        sxz += ds * ((double)H.z[b0 + i] - zm);
        sxx += ds * ds;
    }
    const double tl = sxx > 0.0 ? sxz / sxx : 0.0;
    const double z0 = zm - tl * sm;
    // root of each hit at the initial circle: the one nearest the measured r
    for (int i = 0; i < n; ++i) {
        const double ph = kTwoPi * (double)H.vane[b0 + i] / (double)H.n_vanes;
        const double bb = cos(ph) * (d0 + R) * nx + sin(ph) * (d0 + R) * ny;
        const double disc = bb * bb - d0 * (d0 + 2.0 * R);
        const double sq = sqrt(fmax(disc, 0.0));
        const double rr = (double)H.r[b0 + i];
        sign[b0 + i] = fabs(bb + sq - rr) <= fabs(bb - sq - rr) ? 1.0f : -1.0f;
        aref[b0 + i] = (float)a[i];
    }
    P[0] = (float)(1.0 / R);
    P[1] = (float)phi0;
    P[2] = (float)d0;
    P[3] = (float)z0;
    P[4] = (float)tl;
    status[c] = 0;
}

// ---------------------------------------------------------------------------
// residuals and their derivatives (float32)
// ---------------------------------------------------------------------------

struct HitModel {
    float er, ez;          // residuals / sigma
    float jr[5], jz[5];    // d(er)/dp, d(ez)/dp
};

// Residuals of one hit and, with DERIV, their derivatives in p.
template <bool DERIV>
__device__ __forceinline__ void hit_model(const float p[5], float r, float z, int vane, int n_vanes, float s,
                                          float aref, float inv_sigma, HitModel &m) {
    const float kappa = p[0], phi0 = p[1], d0 = p[2], z0 = p[3], tl = p[4];
    const float rs = 1.0f / kappa;
    float sn, cs;
    sincosf(phi0, &sn, &cs);
    const float nx = sn, ny = -cs;          // normal
    const float ox = cs, oy = sn;           // direction at the perigee
    const float mm = d0 + rs;
    const float cx = mm * nx, cy = mm * ny;
    float uy, ux;
    sincosf(6.28318530717958647692f * (float)vane / (float)n_vanes, &uy, &ux);
    const float bb = ux * cx + uy * cy;
    const float q = d0 * (d0 + 2.0f * rs);
    const float disc = bb * bb - q;
    const bool in = disc > 0.0f;
    const float sq = in ? sqrtf(disc) : 0.0f;
    const float t = bb + s * sq;
    const float v0x = -rs * nx, v0y = -rs * ny;
    const float vx = t * ux - cx, vy = t * uy - cy;
    const float X = v0x * vy - v0y * vx;
    const float Y = v0x * vx + v0y * vy;
    const float sg = kappa > 0.0f ? 1.0f : -1.0f;
    const float alpha = -sg * atan2f(X, Y);
    const float twopi = 6.28318530717958647692f;
    const float da = alpha - aref;
    const float a = aref + (da - twopi * rintf(da / twopi));
    const float R = fabsf(rs);
    m.er = (r - t) * inv_sigma;
    m.ez = (z - (z0 + R * a * tl)) * inv_sigma;
    if (!DERIV) return;
    const float rs2 = rs * rs;
    // d c / d (kappa, phi0, d0)
    const float dcx[3] = {-rs2 * nx, mm * ox, nx};
    const float dcy[3] = {-rs2 * ny, mm * oy, ny};
    const float dq[3] = {-2.0f * d0 * rs2, 0.0f, 2.0f * d0 + 2.0f * rs};
    // d v0 / d (kappa, phi0, d0)
    const float dv0x[3] = {rs2 * nx, -rs * ox, 0.0f};
    const float dv0y[3] = {rs2 * ny, -rs * oy, 0.0f};
    const float den = X * X + Y * Y;
    const float dR = -sg * rs2;   // d |rs| / d kappa
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float db = ux * dcx[k] + uy * dcy[k];
        const float dsq = in ? (2.0f * bb * db - dq[k]) / (2.0f * sq) : 0.0f;
        const float dt = db + s * dsq;
        const float dvx = dt * ux - dcx[k], dvy = dt * uy - dcy[k];
        const float dX = dv0x[k] * vy + v0x * dvy - dv0y[k] * vx - v0y * dvx;
        const float dY = dv0x[k] * vx + v0x * dvx + dv0y[k] * vy + v0y * dvy;
        const float dal = -sg * (Y * dX - X * dY) / den;
        float dz = R * tl * dal;
        if (k == 0) dz += dR * a * tl;
        m.jr[k] = -dt * inv_sigma;
        m.jz[k] = -dz * inv_sigma;
    }
    m.jr[3] = 0.0f;
    m.jr[4] = 0.0f;
    m.jz[3] = -inv_sigma;
    m.jz[4] = -R * a * inv_sigma;
}

__global__ __launch_bounds__(kRefitThreads) void k_refit_chi2(RefitHits H, const float *sign, const float *aref,
                                                             const float *params, float inv_sigma, float *chi2) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= H.n_cand) return;
    float p[5];
    for (int q = 0; q < 5; ++q) p[q] = params[5 * (size_t)c + q];
    float acc = 0.0f;
    for (int64_t i = H.off[c]; i < H.off[c + 1]; ++i) {
        HitModel m;
        hit_model<false>(p, H.r[i], H.z[i], H.vane[i], H.n_vanes, sign[i], aref[i], inv_sigma, m);
        acc += m.er * m.er + m.ez * m.ez;
    }
    chi2[c] = acc;
}

// grad[c] = upstream[c] * d chi^2_c / d p_c = upstream[c] * 2 sum_i (er jr + ez jz)
__global__ __launch_bounds__(kRefitThreads) void k_refit_grad(RefitHits H, const float *sign, const float *aref,
                                                             const float *params, const float *upstream,
                                                             float inv_sigma, float *grad) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= H.n_cand) return;
    float p[5], g[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (int q = 0; q < 5; ++q) p[q] = params[5 * (size_t)c + q];
    for (int64_t i = H.off[c]; i < H.off[c + 1]; ++i) {
        HitModel m;
        hit_model<true>(p, H.r[i], H.z[i], H.vane[i], H.n_vanes, sign[i], aref[i], inv_sigma, m);
#pragma unroll
        for (int q = 0; q < 5; ++q) g[q] += m.er * m.jr[q] + m.ez * m.jz[q];
    }
    const float w = upstream != nullptr ? 2.0f * upstream[c] : 2.0f;
    for (int q = 0; q < 5; ++q) grad[5 * (size_t)c + q] = w * g[q];
}

// `steps` damped, scaled Gauss-Newton steps; chi2 (optional) at the end.
__global__ __launch_bounds__(kRefitThreads) void k_refit_gn(RefitHits H, const float *sign, const float *aref,
                                                           float *params, int steps, float mu, float inv_sigma,
                                                           const int32_t *status, float *chi2) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= H.n_cand) return;
    float p[5];
    for (int q = 0; q < 5; ++q) p[q] = params[5 * (size_t)c + q];
    const bool fit = status == nullptr || status[c] == 0;
    for (int it = 0; it < steps && fit; ++it) {
        float h[15] = {0.0f};   // upper triangle of J^T J, row-major
        float g[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        for (int64_t i = H.off[c]; i < H.off[c + 1]; ++i) {
            HitModel m;
            hit_model<true>(p, H.r[i], H.z[i], H.vane[i], H.n_vanes, sign[i], aref[i], inv_sigma, m);
            int o = 0;
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                g[a] += m.jr[a] * m.er + m.jz[a] * m.ez;
#pragma unroll
                for (int b = a; b < 5; ++b) h[o++] += m.jr[a] * m.jr[b] + m.jz[a] * m.jz[b];
            }
        }
        // Jacobi scaling, damping, Cholesky solve of (S H S + mu I) y = -S g
        float d[5];
        int o = 0;
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            const float v = h[o];
            d[a] = v > 0.0f ? sqrtf(v) : 1.0f;
            o += 5 - a;
        }
        float L[15];
        o = 0;
#pragma unroll
        for (int a = 0; a < 5; ++a)
#pragma unroll
            for (int b = a; b < 5; ++b) {
                L[o] = h[o] / (d[a] * d[b]) + (a == b ? mu : 0.0f);
                ++o;
            }
        // in-place Cholesky on the upper triangle: U^T U = L
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            const int ia = a * 5 - a * (a - 1) / 2;   // index of (a, a)
            float s = L[ia];
#pragma unroll
            for (int k = 0; k < a; ++k) {
                const float u = L[k * 5 - k * (k - 1) / 2 + (a - k)];
                s -= u * u;
            }
            ok = ok && s > 0.0f;
            const float ua = sqrtf(fmaxf(s, 1e-30f));
            L[ia] = ua;
#pragma unroll
            for (int b = a + 1; b < 5; ++b) {
                float t = L[ia + (b - a)];
#pragma unroll
                for (int k = 0; k < a; ++k) {
                    const int ik = k * 5 - k * (k - 1) / 2;
                    t -= L[ik + (a - k)] * L[ik + (b - k)];
                }
                L[ia + (b - a)] = t / ua;
            }
        }
        if (!ok) break;
        float y[5];
#pragma unroll
        for (int a = 0; a < 5; ++a) {   // U^T w = -S g
            float t = -g[a] / d[a];
#pragma unroll
            for (int k = 0; k < a; ++k) t -= L[k * 5 - k * (k - 1) / 2 + (a - k)] * y[k];
            y[a] = t / L[a * 5 - a * (a - 1) / 2];
        }
#pragma unroll
        for (int a = 4; a >= 0; --a) {  // U y = w
            float t = y[a];
#pragma unroll
            for (int b = a + 1; b < 5; ++b) t -= L[a * 5 - a * (a - 1) / 2 + (b - a)] * y[b];
            y[a] = t / L[a * 5 - a * (a - 1) / 2];
        }
        bool finite = true;
#pragma unroll
        for (int a = 0; a < 5; ++a) finite = finite && isfinite(p[a] + y[a] / d[a]);
        if (!finite) break;
#pragma unroll
        for (int a = 0; a < 5; ++a) p[a] += y[a] / d[a];
    }
    for (int q = 0; q < 5; ++q) params[5 * (size_t)c + q] = p[q];
    if (chi2 != nullptr) {
        float acc = 0.0f;
        for (int64_t i = H.off[c]; i < H.off[c + 1]; ++i) {
            HitModel m;
            hit_model<false>(p, H.r[i], H.z[i], H.vane[i], H.n_vanes, sign[i], aref[i], inv_sigma, m);
            acc += m.er * m.er + m.ez * m.ez;
        }
        chi2[c] = acc;
    }
}

// Gathers each candidate's hits (event-local indices in hit_index) from the
// batch's hit arrays: candidate c's hits land at [hit_offset_c, + n_hits_c).
__global__ __launch_bounds__(kRefitThreads) void k_refit_gather(int32_t n_cand, const hough_candidate *cand,
                                                               const int32_t *hit_index, const int64_t *ev_off,
                                                               const float *r, const float *z,
                                                               const int16_t *vane, int64_t *off, float *ro,
                                                               float *zo, int16_t *vo) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > n_cand) return;
    if (c == n_cand) {
        off[c] = n_cand > 0 ? cand[c - 1].hit_offset + cand[c - 1].n_hits : 0;
        return;
    }
    const hough_candidate cd = cand[c];
    off[c] = cd.hit_offset;
    const int64_t base = ev_off[cd.event];
    for (uint32_t j = 0; j < cd.n_hits; ++j) {
        const int64_t g = base + hit_index[cd.hit_offset + j];
        ro[cd.hit_offset + j] = r[g];
        zo[cd.hit_offset + j] = z[g];
        vo[cd.hit_offset + j] = vane[g];
    }
}

int grid(int n) { return (n + kRefitThreads - 1) / kRefitThreads; }

hough_status check(int32_t n_cand, const int64_t *off, const float *r, const float *z, const int16_t *vane,
                   int32_t n_vanes) {
    if (n_cand < 0 || n_vanes < 1) return HOUGH_ERR_INVALID_ARG;
    if (n_cand > 0 && (!off || !r || !z || !vane)) return HOUGH_ERR_INVALID_ARG;
    return HOUGH_OK;
}

hough_status launched() { return hipGetLastError() == hipSuccess ? HOUGH_OK : HOUGH_ERR_DEVICE; }

}  // namespace
}  // namespace hough

using namespace hough;

extern "C" {

hough_status hough_refit_gather(void *stream, int32_t n_cand, const hough_candidate *cand, const int32_t *hit_index,
                                const int64_t *event_offsets, const float *r, const float *z, const int16_t *vane,
                                int64_t *hit_offsets, float *r_out, float *z_out, int16_t *vane_out) {
    if (n_cand < 0 || !hit_offsets || (n_cand > 0 && (!cand || !hit_index || !event_offsets || !r || !z || !vane ||
                                                      !r_out || !z_out || !vane_out)))
        return HOUGH_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_refit_gather, dim3(grid(n_cand + 1)), dim3(kRefitThreads), 0,
                       static_cast<hipStream_t>(stream), n_cand, cand, hit_index, event_offsets, r, z, vane,
                       hit_offsets, r_out, z_out, vane_out);
    return launched();
}

hough_status hough_refit_init(void *stream, int32_t n_cand, const int64_t *hit_offsets, const float *r,
                              const float *z, const int16_t *vane, int32_t n_vanes, float *params, float *hit_sign,
                              float *hit_aref, int32_t *status) {
    hough_status st = check(n_cand, hit_offsets, r, z, vane, n_vanes);
    if (st) return st;
    if (n_cand > 0 && (!params || !hit_sign || !hit_aref || !status)) return HOUGH_ERR_INVALID_ARG;
    if (n_cand == 0) return HOUGH_OK;
    RefitHits H{n_cand, hit_offsets, r, z, vane, n_vanes};
    hipLaunchKernelGGL(k_refit_init, dim3(grid(n_cand)), dim3(kRefitThreads), 0, static_cast<hipStream_t>(stream),
                       H, params, hit_sign, hit_aref, status);
    return launched();
}

hough_status hough_refit_chi2(void *stream, int32_t n_cand, const int64_t *hit_offsets, const float *r,
                              const float *z, const int16_t *vane, int32_t n_vanes, const float *hit_sign,
                              const float *hit_aref, const float *params, float sigma, float *chi2) {
    hough_status st = check(n_cand, hit_offsets, r, z, vane, n_vanes);
    if (st) return st;
    if (!(sigma > 0.0f) || (n_cand > 0 && (!hit_sign || !hit_aref || !params || !chi2))) return HOUGH_ERR_INVALID_ARG;
    if (n_cand == 0) return HOUGH_OK;
    RefitHits H{n_cand, hit_offsets, r, z, vane, n_vanes};
    hipLaunchKernelGGL(k_refit_chi2, dim3(grid(n_cand)), dim3(kRefitThreads), 0, static_cast<hipStream_t>(stream),
                       H, hit_sign, hit_aref, params, 1.0f / sigma, chi2);
    return launched();
}

hough_status hough_refit_grad(void *stream, int32_t n_cand, const int64_t *hit_offsets, const float *r,
                              const float *z, const int16_t *vane, int32_t n_vanes, const float *hit_sign,
                              const float *hit_aref, const float *params, const float *grad_chi2, float sigma,
                              float *grad_params) {
    hough_status st = check(n_cand, hit_offsets, r, z, vane, n_vanes);
    if (st) return st;
    if (!(sigma > 0.0f) || (n_cand > 0 && (!hit_sign || !hit_aref || !params || !grad_params)))
        return HOUGH_ERR_INVALID_ARG;
    if (n_cand == 0) return HOUGH_OK;
    RefitHits H{n_cand, hit_offsets, r, z, vane, n_vanes};
    hipLaunchKernelGGL(k_refit_grad, dim3(grid(n_cand)), dim3(kRefitThreads), 0, static_cast<hipStream_t>(stream),
                       H, hit_sign, hit_aref, params, grad_chi2, 1.0f / sigma, grad_params);
    return launched();
}

hough_status hough_refit_gauss_newton(void *stream, int32_t n_cand, const int64_t *hit_offsets, const float *r,
                                      const float *z, const int16_t *vane, int32_t n_vanes, const float *hit_sign,
                                      const float *hit_aref, const int32_t *status, float *params, int32_t steps,
                                      float damping, float sigma, float *chi2) {
    hough_status st = check(n_cand, hit_offsets, r, z, vane, n_vanes);
    if (st) return st;
    if (!(sigma > 0.0f) || steps < 0 || !(damping >= 0.0f) ||
        (n_cand > 0 && (!hit_sign || !hit_aref || !params)))
        return HOUGH_ERR_INVALID_ARG;
    if (n_cand == 0) return HOUGH_OK;
    RefitHits H{n_cand, hit_offsets, r, z, vane, n_vanes};
    hipLaunchKernelGGL(k_refit_gn, dim3(grid(n_cand)), dim3(kRefitThreads), 0, static_cast<hipStream_t>(stream), H,
                       hit_sign, hit_aref, params, steps, damping, 1.0f / sigma, status, chi2);
    return launched();
}

}  // extern "C"
