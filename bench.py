"""Benchmark: Hough track finding at pileup 50 on one MI355X.

One step = one call of the finder (the whole find-and-remove hot path) over a
batch of 4096 synthetic pileup-50 events already resident in HBM (1024 x 1024
uint32 histogram, T = 6, window peaks with w = 1). Reports batched events/s
as the value, and beside it:
  * the plain one-event-per-call rate and latency percentiles;
  * the finder kernel's roofline figures: VALU ("roofline"), the LDS atomic
    rate of its votes against the device's measured rate ("lds_roofline"),
    HBM traffic from the committed rocprofv3 counter summary;
  * the CPU oracle on one core and on every core of the host's share, both
    before the GPU is touched;
  * the Eq. (5) track-finding efficiency on the generator truth;
  * the served stream, the helix refit and the coarse-to-fine search legs.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--plain-events P]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "events/s Hough track-finding at pileup 50 (batched vs plain) + p99 event latency"
N_EVENTS = 4096
PILEUP = 50
# unfused, unpacked float32 operations of Eq. (4) and its binning per vote:
# phi*c, z*s, add, subtract rho_min, multiply by inv_w
FLOPS_PER_VOTE = 5
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one float op per lane per clock
VALU_PEAK_TFLOPS = 256 * 64 * 2.4e9 / 1e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-events", type=int, default=512)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-events", type=int, default=50000,
                    help="requests per offered rate in the served-stream leg (0: skip it)")
    ap.add_argument("--serve-rates", default="20000,50000,100000")
    ap.add_argument("--serve-lanes", type=int, default=3)
    ap.add_argument("--serve-pool", type=int, default=4096)
    ap.add_argument("--refit-events", type=int, default=4096,
                    help="events of the Poisson(20) batch whose candidates the refit leg fits (0: skip it)")
    ap.add_argument("--refit-oracle", type=int, default=30,
                    help="pure candidates also fitted by the float64 oracle for the parameter error")
    ap.add_argument("--no-coarse-fine", action="store_true",
                    help="skip the coarse-to-fine leg (the paper's 18 x 100 -> 10 x 10 histograms)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this size first, as the reference kernel for "
                         "FETCH_SIZE / WRITE_SIZE counter scaling")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(events shard across GPUs with no communication; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    from paper_2511_02742_amd import eventgen

    t0 = time.time()
    batch = eventgen.pileup_batch(N_EVENTS, n_tracks=PILEUP, seed0=0)
    log("generated %d events in %.1f s: %s" % (N_EVENTS, time.time() - t0, eventgen.hit_histogram(batch)))

    # ---- CPU oracle on a bounded sample, before anything touches the GPU
    # (the all-cores figure starts worker processes)
    cpu = cpu_all = None
    if not args.no_cpu_baseline:
        from oracle import OracleConfig, oracle_find
        ocfg = OracleConfig()
        n_done = 0
        tc0 = time.perf_counter()
        while n_done < N_EVENTS and (time.perf_counter() - tc0 < args.cpu_seconds or n_done < 16):
            lo, hi = int(batch.offsets[n_done]), int(batch.offsets[n_done + 1])
            oracle_find(ocfg, batch.z[lo:hi], batch.vane[lo:hi], event_id=n_done)
            n_done += 1
        tc = time.perf_counter() - tc0
        cpu = {"value": round(n_done / tc, 2), "unit": "events/s", "cores": 1, "kind": "oracle",
               "sample": "first %d of the same %d pileup-50 events, one thread, %.1f s"
                         % (n_done, N_EVENTS, tc)}
        log("cpu oracle: %.1f events/s over %d events" % (n_done / tc, n_done))
        cpu_all = oracle_all_cores(batch, args.cpu_seconds, log)

    import torch

    from paper_2511_02742_amd.hough import HoughFinder

    dev = torch.device("cuda", 0)
    z = torch.from_numpy(batch.z).to(dev)
    vane = torch.from_numpy(batch.vane).to(dev)
    offs = torch.from_numpy(batch.offsets).to(dev)

    if args.copy_calibration_mib > 0:
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        # An elementwise kernel (not a DMA memcpy, which the counters miss)
        # that reads and writes exactly nb bytes each.
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize(dev)
        log("copy calibration (MulFunctor kernel): %d bytes read, %d bytes written" % (nb, nb))
        del src, dst

    f = HoughFinder(0)
    shape = f.launch_shape()
    out = f.alloc_outputs(N_EVENTS, batch.n_hits)
    stream = torch.cuda.current_stream(dev)

    # ---- batched: one call over all events --------------------------------
    for _ in range(args.warmup):
        f.find(z, vane, offs, out=out, stream=stream)
    torch.cuda.synchronize(dev)
    f.set_timing(True)
    f.timing(reset=True)
    torch.cuda.synchronize(dev)
    t1 = time.perf_counter()
    for _ in range(args.steps):
        f.find(z, vane, offs, out=out, stream=stream)
    torch.cuda.synchronize(dev)
    t2 = time.perf_counter()
    f.set_timing(False)
    kern_ms, launches = f.timing(reset=True)
    from paper_2511_02742_amd.hough import COUNT_NAMES
    info = dict(zip(COUNT_NAMES, (int(x) for x in out.counts.cpu().numpy())))
    assert info["status"] == 0, info
    main_cand, main_hits, _ = out.to_host()
    eff = eq5_efficiency(batch, main_cand, main_hits)
    log("Eq. (5) efficiency: %s" % eff)
    wall = t2 - t1
    ms_per_step = 1e3 * wall / args.steps
    value = N_EVENTS * args.steps / wall
    kern_avg_ms = kern_ms / max(launches, 1)
    log("batched: %.3f ms/step, %.0f events/s, finder kernel %.3f ms avg over %d launches"
        % (ms_per_step, value, kern_avg_ms, launches))

    # ---- plain: one event per call ----------------------------------------
    npl = min(args.plain_events, N_EVENTS)
    single = []
    for e in range(npl):
        lo, hi = int(batch.offsets[e]), int(batch.offsets[e + 1])
        o = torch.tensor([0, hi - lo], dtype=torch.int64, device=dev)
        single.append((z[lo:hi], vane[lo:hi], o, f.alloc_outputs(1, hi - lo)))
    for e in range(min(16, npl)):
        zz, vv, oo, oo_out = single[e]
        f.find(zz, vv, oo, out=oo_out, stream=stream)
    torch.cuda.synchronize(dev)
    lat = np.zeros(npl)
    tp0 = time.perf_counter()
    for e in range(npl):
        zz, vv, oo, oo_out = single[e]
        ts = time.perf_counter()
        f.find(zz, vv, oo, out=oo_out, stream=stream)
        stream.synchronize()
        lat[e] = time.perf_counter() - ts
    tp1 = time.perf_counter()
    plain_rate = npl / (tp1 - tp0)
    log("plain: %.0f events/s, p50 %.1f us, p99 %.1f us" % (plain_rate, 1e6 * np.percentile(lat, 50),
                                                              1e6 * np.percentile(lat, 99)))

    # ---- HBM traffic of the finder kernel from the committed counter summary
    # (reported only while the kernel source still matches the one profiled)
    traffic = profiled_traffic("k_find_pileup50", "hough_kernels.hip")

    # ---- roofline of the finder kernel ------------------------------------
    flops = FLOPS_PER_VOTE * info["evals"]
    achieved = flops / (kern_avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(VALU_PEAK_TFLOPS, 2),
                "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": "k_find", "kernel_avg_ms": round(kern_avg_ms, 4),
                "evals_per_launch": info["evals"], "flops_per_eval": FLOPS_PER_VOTE,
                "evals_per_s": round(info["evals"] / (kern_avg_ms * 1e-3), 1)}


    # ---- LDS atomic roofline of the finder's votes (the survey's denominator:
    # every histogram vote is one LDS atomic add)
    from paper_2511_02742_amd.hough import lds_peak
    peak_cf = lds_peak(0)
    peak_vote = lds_peak(1)
    votes_s = info["votes"] / (kern_avg_ms * 1e-3)
    lds = {"bound": "lds", "achieved": round(votes_s, 1), "unit": "lane atomics/s",
           "peak": round(peak_cf, 1), "frac": round(votes_s / peak_cf, 4),
           "peak_vote_pattern": round(peak_vote, 1), "frac_vote_pattern": round(votes_s / peak_vote, 4),
           "votes_per_launch": info["votes"], "kernel": "k_find", "kernel_avg_ms": round(kern_avg_ms, 4),
           "note": "peak: conflict-free ds_add_u32 without return; vote pattern: random bins of a 1024-word "
                   "row with return (hough_lds_peak, measured in this run)"}
    log("LDS roofline: %s" % lds)

    served = serve_bench(args, f, log) if args.serve_events > 0 else None
    refit = refit_bench(args, f, log) if args.refit_events > 0 else None
    coarse_fine = None if args.no_coarse_fine else coarse_fine_bench(args, batch, z, vane, offs, log, peak_vote)

    rec = {
        "metric": METRIC, "value": round(value, 1), "unit": "events/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "pileup-50 batch: %d events x 50 helix tracks + 1%% noise, seeds 0..%d, "
                               "1024x1024 uint32 histogram, T=6, nms w=1" % (N_EVENTS, N_EVENTS - 1),
                   "n_events": N_EVENTS, "hits_total": batch.n_hits, "n_theta": 1024, "n_rho": 1024,
                   "min_votes": 6, "peak_mode": "nms", "launch": shape},
        "plain": {"value": round(plain_rate, 1), "unit": "events/s", "events": npl,
                  "latency_us_p50": round(1e6 * float(np.percentile(lat, 50)), 2),
                  "latency_us_p99": round(1e6 * float(np.percentile(lat, 99)), 2)},
        "batched_latency_ms_p99": round(ms_per_step, 4),
        "speedup_batched_vs_plain": round(value / plain_rate, 2),
        "work": {k: info[k] for k in ("candidates", "hits", "evals", "iters", "max_iters", "passes", "tiled",
                                      "truncations", "hot_scans", "hotset_full", "recounts")},
        "efficiency_eq5": eff,
        "roofline": roofline,
        "lds_roofline": lds,
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
        "served": served,
        "refit": refit,
        "coarse_fine": coarse_fine,
    }
    print(json.dumps(rec), flush=True)


def serve_bench(args, finder, log):
    """Served stream: requests of mixed pileup (uniform over 1, 10, 25, 50,
    100 tracks, drawn from a pool of seeded events) arrive as a Poisson
    process at each offered rate and go through the server's continuous
    batching. Latency is the server's completion time minus the request's
    arrival time. A final burst (every request arriving at once) gives the
    most the served form sustains."""
    import numpy as np
    import torch
    from paper_2511_02742_amd import eventgen
    from paper_2511_02742_amd.hough import HoughServer

    pool = eventgen.mixed_pileup_batch(args.serve_pool, seed0=2_000_000)
    P = len(pool.offsets) - 1
    lens = np.diff(pool.offsets)
    # expected per-event results from one batched call on the pool
    dev = torch.device("cuda", 0)
    out = finder.find(torch.from_numpy(pool.z).to(dev), torch.from_numpy(pool.vane).to(dev),
                      torch.from_numpy(pool.offsets).to(dev))
    cand, _, info = out.to_host()
    assert info["status"] == 0
    want_nc = np.bincount(cand["event"], minlength=P)
    want_nh = np.bincount(cand["event"], weights=cand["n_hits"], minlength=P).astype(np.int64)

    rates = [float(r) for r in args.serve_rates.split(",") if r] + [float("inf")]
    res = []
    with HoughServer(0, lanes=args.serve_lanes, queue_events=1 << 21, queue_hits=1 << 28) as srv:
        # warm-up
        srv.submit(pool.z, pool.vane, pool.offsets[:65])
        srv.drain(60.0)
        srv.poll_records()
        for rate in rates:
            n = args.serve_events
            rng = np.random.default_rng(12345 + (0 if rate == float("inf") else int(rate)))
            idx = rng.integers(0, P, n)
            st0 = srv.stats()
            t_start = srv.clock() + 0.1
            arr = t_start + (np.zeros(n) if rate == float("inf") else np.cumsum(rng.exponential(1.0 / rate, n)))
            sub = 0
            recs = []
            got = 0
            chunk = 8192 if rate == float("inf") else 4096
            while got < n:
                now = srv.clock()
                while sub < n and arr[sub] - now < 0.2:
                    hi = min(n, sub + chunk)
                    sel = idx[sub:hi]
                    ln = lens[sel]
                    offs = np.zeros(len(sel) + 1, np.int64)
                    np.cumsum(ln, out=offs[1:])
                    gather = np.repeat(pool.offsets[sel] - offs[:-1], ln) + np.arange(offs[-1])
                    acc = srv.submit(pool.z[gather], pool.vane[gather], offs,
                                     tags=np.arange(sub, hi, dtype=np.uint64), t_arrival=arr[sub:hi])
                    assert acc == hi - sub, (acc, hi - sub)
                    sub = hi
                r, _, _ = srv.poll_records()
                if len(r):
                    recs.append(r)
                    got += len(r)
                else:
                    time.sleep(0.0002)
            r = np.concatenate(recs)
            st1 = srv.stats()
            assert (r["status"] == 0).all()
            ev = idx[r["tag"].astype(np.int64)]
            mism = int(((r["n_candidates"] != want_nc[ev]) | (r["n_hit_index"] != want_nh[ev])).sum())
            lat = r["t_done"] - r["t_arrival"]
            span = float(r["t_done"].max() - r["t_arrival"].min())
            launches = st1["launches"] - st0["launches"]
            ent = {"offered_per_s": None if rate == float("inf") else rate, "requests": n,
                   "sustained_per_s": round(n / span, 1),
                   "latency_us_p50": round(1e6 * float(np.percentile(lat, 50)), 1),
                   "latency_us_p99": round(1e6 * float(np.percentile(lat, 99)), 1),
                   "queue_us_p50": round(1e6 * float(np.percentile(r["t_admit"] - r["t_arrival"], 50)), 1),
                   "launches": launches, "events_per_launch": round(n / max(launches, 1), 2),
                   "max_lanes_busy": st1["max_lanes_busy"], "mismatches": mism}
            log("served %s: %s" % ("burst" if rate == float("inf") else "%.0f/s" % rate, ent))
            res.append(ent)
        dev_bytes = srv.stats()["device_bytes"]
    return {"workload": "mixed pileup {1,10,25,50,100} tracks + 1%% noise, pool of %d seeded events "
                        "(seeds 2000000..), Poisson arrivals" % P,
            "lanes": args.serve_lanes, "device_bytes": dev_bytes, "mean_hits": round(float(lens.mean()), 1),
            "rates": res}


def refit_bench(args, finder, log):
    """Helix refit of the candidates the finder returns for the uneven batch
    (Poisson(20) tracks per event, seeds 1000000..): gather, initial fit and
    20 Gauss-Newton steps on the GPU (timed with HIP events), the parameter
    error against the float64 oracle on a sample of candidates whose hits all
    come from one generated track, and the momentum resolution against the
    generator truth."""
    import math
    import numpy as np
    import torch
    from paper_2511_02742_amd import eventgen
    from paper_2511_02742_amd.hough import (REFIT_STEPS, momentum_mev, refit_gather, refit_gauss_newton,
                                            refit_init)

    b = eventgen.poisson_batch(args.refit_events)
    dev = torch.device("cuda", 0)
    t = {k: torch.from_numpy(getattr(b, k)).to(dev) for k in ("r", "z", "vane", "offsets")}
    out = finder.find(t["z"], t["vane"], t["offsets"])
    cand, hit_index, info = out.to_host()
    assert info["status"] == 0
    hits = refit_gather(out, t["offsets"], t["r"], t["z"], t["vane"])
    stream = torch.cuda.current_stream(dev)
    times = []
    for rep in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        p = refit_init(hits).contiguous()
        chi2 = refit_gauss_newton(hits, p)
        e1.record(stream)
        torch.cuda.synchronize(dev)
        if rep > 0:
            times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    status = hits.status.cpu().numpy()
    P = p.cpu().numpy().astype(np.float64)
    mom = momentum_mev(p.double()).cpu().numpy()
    n_cand = len(cand)
    # purity and truth momentum of each candidate
    pure = np.zeros(n_cand, bool)
    ptrue = np.zeros(n_cand)
    for c, cd in enumerate(cand):
        ev = b.events[cd["event"]]
        tr = ev.track[hit_index[cd["hit_offset"]:cd["hit_offset"] + cd["n_hits"]]]
        if tr[0] >= 0 and np.all(tr == tr[0]):
            pure[c] = True
            ptrue[c] = ev.p[tr[0]]
    fit = (status == 0)
    sel = fit & pure
    ratio = mom[sel] / ptrue[sel] - 1.0
    res = {"workload": "candidates of %d events, Poisson(20) tracks + 1%% noise (seeds 1000000..)" % args.refit_events,
           "candidates": n_cand, "fitted": int(fit.sum()), "pure_fitted": int(sel.sum()),
           "steps": REFIT_STEPS, "ms": round(ms, 4), "candidates_per_s": round(n_cand / (ms * 1e-3), 1),
           "momentum_bias": round(float(np.median(ratio)), 5),
           "momentum_resolution_68": round(float(np.quantile(np.abs(ratio - np.median(ratio)), 0.68)), 5)}
    if args.refit_oracle > 0 and not args.no_cpu_baseline:
        from oracle.refit_oracle import refit_gn, refit_init as o_init
        floors = np.array([1e-4, 1.0, 1.0, 1.0, 0.01])
        worst = np.zeros(5)
        done = 0
        r_np, z_np, v_np = b.r, b.z, b.vane
        for c in np.nonzero(sel)[0][:args.refit_oracle]:
            cd = cand[c]
            idx = b.offsets[cd["event"]] + hit_index[cd["hit_offset"]:cd["hit_offset"] + cd["n_hits"]]
            p0, s0, a0 = o_init(r_np[idx], z_np[idx], v_np[idx])
            po = refit_gn(p0, r_np[idx], z_np[idx], v_np[idx], s0, a0)
            e = np.abs(P[c] - po) / np.maximum(np.abs(po), floors)
            e[1] = abs(math.remainder(P[c][1] - po[1], 2 * math.pi))
            worst = np.maximum(worst, e)
            done += 1
        res["oracle_sample"] = done
        res["max_param_error_vs_f64"] = {k: float("%.3g" % v) for k, v in
                                         zip(("kappa", "phi0", "d0", "z0", "tan_lambda"), worst)}
    log("refit: %s" % res)
    return res


def _oracle_slice(args):
    """Worker: the oracle over one contiguous slice of events for about
    `seconds` (at least 4 events); returns (events done, seconds)."""
    z, vane, offsets, seconds = args
    from oracle import OracleConfig, oracle_find
    cfg = OracleConfig()
    done = 0
    t0 = time.perf_counter()
    while done < len(offsets) - 1 and (time.perf_counter() - t0 < seconds or done < 4):
        lo, hi = int(offsets[done]), int(offsets[done + 1])
        oracle_find(cfg, z[lo:hi], vane[lo:hi])
        done += 1
    return done, time.perf_counter() - t0


def oracle_all_cores(batch, seconds, log):
    """The same single-thread oracle in independent worker processes (one per
    core of the host's share, at most 16) over disjoint slices of the batch."""
    import multiprocessing as mp
    import numpy as np
    workers = max(1, min(16, os.cpu_count() or 1))
    bounds = np.linspace(0, N_EVENTS, workers + 1).astype(int)
    jobs = []
    for w in range(workers):
        e0, e1 = bounds[w], bounds[w + 1]
        lo, hi = int(batch.offsets[e0]), int(batch.offsets[e1])
        jobs.append((batch.z[lo:hi].copy(), batch.vane[lo:hi].copy(), batch.offsets[e0:e1 + 1] - lo, seconds))
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_slice, jobs)
    done = sum(r[0] for r in res)
    span = max(r[1] for r in res)
    log("cpu oracle, %d processes: %.1f events/s" % (workers, done / span))
    return {"value": round(done / span, 2), "unit": "events/s", "cores": workers, "kind": "oracle",
            "sample": "%d independent single-thread processes over disjoint slices of the same %d pileup-50 "
                      "events, %d events in %.1f s" % (workers, N_EVENTS, done, span)}


def profiled_traffic(name, source):
    """HBM bytes per launch (read + written) from the committed counter
    summary profiles/<name>.txt, or None when it is missing or was taken from
    another version of the kernel source."""
    try:
        from paper_2511_02742_amd.prof_summary import kernel_source_hash
        kv = {}
        with open(os.path.join(ROOT, "profiles", name + ".txt")) as fh:
            for line in fh:
                if ":" in line:
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_sha256_16") == kernel_source_hash(source) and "fetch_bytes_per_launch" in kv:
            return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    except (OSError, ValueError):
        pass
    return None


def _has_run(vanes, length, n_vanes=40):
    """Whether the vane set holds `length` consecutive vanes (cyclic)."""
    return any(all((v + i) % n_vanes in vanes for i in range(length)) for v in vanes)


def eq5_efficiency(batch, cand, hit_index, run=5):
    """Track-finding efficiency of Eq. (5), N_found / N_all: a generated track
    counts as found when one candidate holds its hits on `run` consecutive
    vanes. Returned over all generated tracks and over the tracks whose own
    hits span such a run (the ones a seed can find at all)."""
    import numpy as np
    found = set()
    for cd in cand:
        ev = batch.events[cd["event"]]
        idx = hit_index[cd["hit_offset"]:cd["hit_offset"] + cd["n_hits"]]
        tr, vn = ev.track[idx], ev.vane[idx]
        for t in np.unique(tr[tr >= 0]):
            if _has_run(set(vn[tr == t].tolist()), run):
                found.add((int(cd["event"]), int(t)))
    n_all = n_findable = n_found_findable = 0
    for e, ev in enumerate(batch.events):
        n_all += ev.n_tracks
        for t in np.unique(ev.track[ev.track >= 0]):
            if _has_run(set(ev.vane[ev.track == t].tolist()), run):
                n_findable += 1
                n_found_findable += (e, int(t)) in found
    return {"found": len(found), "all_tracks": n_all, "findable_tracks": n_findable,
            "efficiency": round(len(found) / max(n_all, 1), 4),
            "efficiency_findable": round(n_found_findable / max(n_findable, 1), 4)}


def seeded_fraction(batch, cand, hit_index, min_hits):
    """Share of the generated tracks with at least min_hits hits that some
    candidate seeds: at least min_hits of the candidate's hits, and more than
    half of them, come from that track."""
    import numpy as np
    seeded = set()
    for cd in cand:
        ev = batch.events[cd["event"]]
        tr = ev.track[hit_index[cd["hit_offset"]:cd["hit_offset"] + cd["n_hits"]]]
        tr = tr[tr >= 0]
        if len(tr) == 0:
            continue
        t, k = np.unique(tr, return_counts=True)
        i = int(np.argmax(k))
        if k[i] >= min_hits and 2 * k[i] > cd["n_hits"]:
            seeded.add((int(cd["event"]), int(t[i])))
    findable = 0
    hit = 0
    for e, ev in enumerate(batch.events):
        t, k = np.unique(ev.track[ev.track >= 0], return_counts=True)
        for tt in t[k >= min_hits]:
            findable += 1
            hit += (e, int(tt)) in seeded
    return hit / max(findable, 1), findable


def coarse_fine_bench(args, batch, z, vane, offs, log, lds_vote_peak=None):
    """The paper's two-stage histogram (18 x 100 coarse, 10 x 10 fine, on the
    180 x 1000 grid) on the same pileup-50 batch, against full-grid argmax and
    nms on the same grid: events/s, finder kernel time, Eq. (4) evaluations,
    candidates and the share of findable generated tracks each one seeds."""
    import numpy as np
    import torch
    from paper_2511_02742_amd.hough import HoughFinder
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    res = {"workload": "the same %d pileup-50 events, 180 x 1000 grid, T=6, a=0" % N_EVENTS}
    for name, kw in (("coarse_fine", {"peak_mode": 2}), ("argmax", {"peak_mode": 0}), ("nms", {"peak_mode": 1})):
        f = HoughFinder(0, n_theta=180, n_rho=1000, **kw)
        out = f.alloc_outputs(N_EVENTS, batch.n_hits)
        for _ in range(args.warmup):
            f.find(z, vane, offs, out=out, stream=stream)
        torch.cuda.synchronize(dev)
        f.set_timing(True)
        f.timing(reset=True)
        t1 = time.perf_counter()
        for _ in range(args.steps):
            f.find(z, vane, offs, out=out, stream=stream)
        torch.cuda.synchronize(dev)
        wall = time.perf_counter() - t1
        f.set_timing(False)
        kern_ms, launches = f.timing(reset=True)
        cand, hits, info = out.to_host()
        assert info["status"] == 0, info
        frac, findable = seeded_fraction(batch, cand, hits, 6)
        e5 = eq5_efficiency(batch, cand, hits)
        kavg = kern_ms / max(launches, 1)
        res[name] = {"events_per_s": round(N_EVENTS * args.steps / wall, 1),
                     "ms_per_step": round(1e3 * wall / args.steps, 4), "kernel_avg_ms": round(kavg, 4),
                     "kernel": "k_find_cf" if name == "coarse_fine" else "k_find",
                     "evals": info["evals"], "evals_per_s": round(info["evals"] / (kavg * 1e-3), 1),
                     "votes": info["votes"],
                     "lds_frac_vote_pattern": round(info["votes"] / (kavg * 1e-3) / lds_vote_peak, 4)
                     if lds_vote_peak else None,
                     "candidates": info["candidates"], "iters": info["iters"],
                     "seeded_track_fraction": round(frac, 4),
                     "efficiency_eq5": e5["efficiency"], "efficiency_eq5_findable": e5["efficiency_findable"]}
        res["findable_tracks"] = findable
        log("coarse-fine leg, %s: %s" % (name, res[name]))
    cf = res["coarse_fine"]
    flops = FLOPS_PER_VOTE * cf["evals"]
    achieved = flops / (cf["kernel_avg_ms"] * 1e-3) / 1e12
    cf["roofline"] = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(VALU_PEAK_TFLOPS, 2),
                      "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TFLOPS, 4),
                      "traffic": profiled_traffic("k_find_cf_pileup50", "hough_cf.hip")}
    return res


if __name__ == "__main__":
    main()
