"""Benchmark: Hough track finding at pileup 50 on one MI355X.

One step = one call of the finder (the whole find-and-remove hot path) over a
batch of 4096 synthetic pileup-50 events already resident in HBM (1024 x 1024
uint32 histogram, T = 6, window peaks with w = 1). Reports batched events/s
as the value, the plain one-event-per-call rate and latency percentiles
beside it, the finder kernel's roofline figures and the CPU oracle's rate on
a bounded sample of the same events.

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
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this size first, as the reference kernel for "
                         "FETCH_SIZE / WRITE_SIZE counter scaling")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(events shard across GPUs with no communication; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2511_02742_amd import eventgen
    from paper_2511_02742_amd.hough import HoughFinder

    dev = torch.device("cuda", 0)
    t0 = time.time()
    batch = eventgen.pileup_batch(N_EVENTS, n_tracks=PILEUP, seed0=0)
    log("generated %d events in %.1f s: %s" % (N_EVENTS, time.time() - t0, eventgen.hit_histogram(batch)))
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
    traffic = None
    try:
        from paper_2511_02742_amd.prof_summary import kernel_source_hash
        kv = {}
        with open(os.path.join(ROOT, "profiles", "k_find_pileup50.txt")) as fh:
            for line in fh:
                if ":" in line:
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_sha256_16") == kernel_source_hash() and "fetch_bytes_per_launch" in kv:
            traffic = float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    except (OSError, ValueError):
        traffic = None

    # ---- roofline of the finder kernel ------------------------------------
    flops = FLOPS_PER_VOTE * info["evals"]
    achieved = flops / (kern_avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(VALU_PEAK_TFLOPS, 2),
                "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": "k_find", "kernel_avg_ms": round(kern_avg_ms, 4),
                "evals_per_launch": info["evals"], "flops_per_eval": FLOPS_PER_VOTE,
                "evals_per_s": round(info["evals"] / (kern_avg_ms * 1e-3), 1)}

    # ---- CPU oracle on a bounded sample -----------------------------------
    cpu = None
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
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
