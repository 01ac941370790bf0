"""Where the finder's cycles go, per phase, from the HOUGH_PHASE_CLOCKS build.

Loads ``libhough_tf_phases.so`` (``python -m paper_2511_02742_amd.build
--phase-clocks``), runs the finder on seeded synthetic events with per-event
phase clocks on, and prints the mean cycles per event of each phase (thread
0's cycle counter between workgroup barriers) with the share of the event's
total. Workloads: the 4096-event pileup-50 batch on the default launch shape
and on a 512-thread, 14-row-tile shape (two events per CU), and one-event
calls at pileup 50, 100 and 150. ``--out NAME`` also writes profiles/NAME.md.

python -m paper_2511_02742_amd.phase_clocks [--out k_find_phases]
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

PHASES = ("alive list", "sweep / recount", "window test + sort", "association (other)", "large: banded sweep",
          "large: peak order", "large: association (other)", "tiled fallback", "rest", "assoc: claimed masks",
          "assoc: match masks", "assoc: claims", "assoc: emission", "assoc: hit lists", "recount")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    import torch
    from paper_2511_02742_amd import build, eventgen
    from paper_2511_02742_amd.hough import HoughFinder, load_library
    if not os.path.exists(build.LIB_PHASES):
        sys.exit("build the measurement library first: python -m paper_2511_02742_amd.build --phase-clocks")
    load_library(build.LIB_PHASES)
    dev = torch.device("cuda", 0)
    rows = []

    def run(name, f, batch, reps=3):
        z = torch.from_numpy(batch.z).to(dev)
        v = torch.from_numpy(batch.vane).to(dev)
        o = torch.from_numpy(batch.offsets).to(dev)
        ne = batch.n_events
        buf = torch.zeros(16 * ne, dtype=torch.int64, device=dev)
        out = f.alloc_outputs(ne, batch.n_hits)
        f.find(z, v, o, out=out)
        f.set_event_clock(buf)
        acc = np.zeros(16)
        for _ in range(reps):
            buf.zero_()
            f.find(z, v, o, out=out)
            torch.cuda.synchronize(dev)
            acc += buf.cpu().numpy().reshape(ne, 16).astype(np.float64).sum(axis=0)
        f.set_event_clock(None)
        per = acc[:len(PHASES)] / (reps * ne)
        rows.append((name, per))

    b50 = eventgen.pileup_batch(4096)
    run("4096 pileup-50 events, 1024 threads, 30-row tile", HoughFinder(0), b50)
    run("4096 pileup-50 events, 512 threads, 14-row tile", HoughFinder(0, wg_threads=512, tile_rows=14), b50)
    f = HoughFinder(0)
    for pile in (50, 100, 150):
        acc = []
        for s in range(16):
            one = eventgen.make_batch([eventgen.pileup_event(60000 + s, n_tracks=pile)])
            run("_", f, one, reps=2)
            acc.append(rows.pop()[1])
        rows.append(("one-event calls, pileup %d (16 events)" % pile, np.mean(acc, axis=0)))

    lines = ["| workload | " + " | ".join(PHASES) + " | total |", "|---" * (len(PHASES) + 2) + "|"]
    for name, per in rows:
        tot = per.sum()
        cells = ["%.0f k (%.0f %%)" % (c / 1e3, 100.0 * c / tot) for c in per]
        lines.append("| %s | %s | %.0f k |" % (name, " | ".join(cells), tot / 1e3))
    text = "\n".join(lines)
    print(text)
    if args.out:
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        with open(os.path.join(root, "profiles", args.out + ".md"), "w") as fh:
            fh.write("# %s\n\nMean cycles per event in each phase of k_find (shader clock of the event's "
                     "workgroup, thread 0, between workgroup barriers), from the HOUGH_PHASE_CLOCKS build.\n\n"
                     "Command:\n\n    python -m paper_2511_02742_amd.build --phase-clocks && "
                     "python -m paper_2511_02742_amd.phase_clocks --out %s\n\n%s\n" % (args.out, args.out, text))


if __name__ == "__main__":
    main()
