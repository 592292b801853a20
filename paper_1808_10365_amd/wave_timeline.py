"""Per-wavefront timeline of pass A on CHIME M=256 (``sk_plan_pass_a_timeline``).

Runs the deferred-store pass A (the library's choice for this workload) a few
times with the wavefronts of each SIMD kept level (the library's setting) and
left to the instruction arbiter, and prints, for the last launch of each:

* when the wavefronts started, ended their reads and ended their stores
  (microseconds from the first start);
* the mean end of the reads of the first and of the second wavefront on each
  SIMD (by wavefront index within the workgroup);
* the median end of the reads per XCD.

Usage: ``python3 -m paper_1808_10365_amd.wave_timeline [--reps K]`` on a GPU.
The input is the CHIME synthetic workload (N=2048, F=4, T=2^18, M=256).
"""
from __future__ import annotations

import argparse
import sys

import numpy as np


def summarize(tl: np.ndarray) -> dict:
    """Figures of one timeline (rows: start, reads, end, XCD, HW_ID, SIMD)."""
    t0 = tl[:, 0].min()
    us = lambda v: (v - t0) * 0.01   # 100 MHz clock
    start, reads, end = us(tl[:, 0]), us(tl[:, 1]), us(tl[:, 2])
    xcd, simd = tl[:, 3] & 15, tl[:, 5] & 3
    n = len(tl)
    wg, wave = np.arange(n) // 8, np.arange(n) % 8
    # Rank of each wavefront among those of its workgroup on the same SIMD.
    rank = np.zeros(n, dtype=int)
    for g in range(n // 8):
        seen = {}
        for j in range(8):
            k = g * 8 + j
            rank[k] = seen.get(simd[k], 0)
            seen[simd[k]] = rank[k] + 1
    return {
        "wavefronts": n,
        "start_us": (float(start.min()), float(start.max())),
        "reads_done_us": tuple(float(x) for x in np.percentile(reads, [0, 50, 100])),
        "end_us_max": float(end.max()),
        "stores_us_median": float(np.median(end - reads)),
        "reads_done_mean_by_simd_rank": [float(reads[rank == r].mean()) for r in range(rank.max() + 1)],
        "reads_done_median_by_xcd": {int(x): float(np.median(reads[xcd == x])) for x in sorted(set(xcd.tolist()))},
    }


def text(name: str, s: dict) -> str:
    out = [f"{name}: {s['wavefronts']} wavefronts",
           f"  started      {s['start_us'][0]:7.1f} .. {s['start_us'][1]:7.1f} us",
           "  reads done   min {:7.1f}  median {:7.1f}  max {:7.1f} us".format(*s["reads_done_us"]),
           f"  stores done  max {s['end_us_max']:7.1f} us (median store phase {s['stores_us_median']:.1f} us)",
           "  reads done, mean by order on the SIMD: " +
           ", ".join(f"{'first' if r == 0 else 'second' if r == 1 else f'#{r + 1}'} {v:.1f} us"
                     for r, v in enumerate(s["reads_done_mean_by_simd_rank"])),
           "  reads done, median by XCD: " +
           ", ".join(f"{x}: {v:.1f}" for x, v in s["reads_done_median_by_xcd"].items())]
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--reps", type=int, default=3, help="launches per setting (the last is summarised)")
    a = ap.parse_args(argv)
    import torch
    import synth
    import paper_1808_10365_amd as sk
    w = synth.chime(seed=3, block_len=256)
    x = torch.from_numpy(synth.generate(w)).to("cuda:0")
    plan = sk.Plan(w.n_inputs, w.n_channels, w.n_samples, w.block_len, norm_window=w.norm_window)
    try:
        for _ in range(5):
            plan.compute(x)
        torch.cuda.synchronize()
        for bal, name in ((True, "SIMD balance on (library setting)"), (False, "SIMD balance off (arbiter)")):
            tl = None
            for _ in range(a.reps):
                tl = plan.pass_a_timeline(x, simd_balance=bal)
            print(text(name, summarize(tl)), flush=True)
    finally:
        plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
