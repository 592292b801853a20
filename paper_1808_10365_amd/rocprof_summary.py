"""Short text summaries of rocprofv3 runs (the figures under profiles/).

Reads the SQLite database rocprofv3 writes (``-d DIR -o run``) and prints:

* ``trace DIR``: per-kernel dispatch count and duration (average, median,
  min, max, total) from the kernel trace; with ``--calls`` also the
  batched form's graph calls (a ``batch_pass_a_kernel`` dispatch followed
  by the batched scan / combine / state kernels up to the next pass A),
  grouped by their kernel sequence. The autotuner's and the pass A timer's
  launches each follow a device fill (the queue counter cleared with a
  memset), graph calls do not: sequences right after a
  ``__amd_rocclr_fillBuffer`` dispatch are not counted as calls;
* ``counters FETCH_DIR WRITE_DIR``: FETCH_SIZE and WRITE_SIZE per dispatch
  (KiB), scaled to bytes by what the same counters read for one device copy
  of ``--copy-bytes`` bytes (the ``__amd_rocclr_copyBuffer`` dispatch of
  ``bench.py --copy-probe-mib``);
* ``pmc DIR``: mean per dispatch of every counter collected, per kernel.

Usage: ``python -m paper_1808_10365_amd.rocprof_summary trace DIR [--calls] [--include REGEX]``.
"""
from __future__ import annotations

import argparse
import collections
import glob
import json
import os
import re
import sqlite3
import statistics
import sys


def _db(d: str) -> sqlite3.Connection:
    hits = sorted(glob.glob(os.path.join(d, "**", "*.db"), recursive=True))
    if not hits:
        raise SystemExit(f"no rocprofv3 database under {d}")
    return sqlite3.connect(hits[0])


def _short(name: str, width: int = 70) -> str:
    name = name.replace("void ", "")
    return name if len(name) <= width else name[: width - 3] + "..."


def kernel_rows(d: str):
    con = _db(d)
    return list(con.execute("select name, start, end from kernels order by start"))


def trace(d: str, calls: bool = False, include: str = "") -> str:
    rows = kernel_rows(d)
    per = collections.defaultdict(list)
    pat = re.compile(include) if include else None
    for n, s, e in rows:
        if pat is None or pat.search(n):
            per[n].append((e - s) / 1e3)
    out = [f"{'kernel':70s} {'n':>5s} {'avg_us':>10s} {'med_us':>10s} {'min_us':>10s} {'max_us':>10s} {'total_ms':>10s}"]
    for n, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"{_short(n):70s} {len(v):5d} {statistics.fmean(v):10.2f} {statistics.median(v):10.2f} "
                   f"{min(v):10.2f} {max(v):10.2f} {sum(v) / 1e3:10.3f}")
    if calls:
        out.append("")
        out.append("batched graph calls (pass A dispatch, not right after a fill, followed by pass B kernels "
                   "up to the next pass A):")
        seqs = []
        i = 0
        while i < len(rows):
            trial = i > 0 and "fillBuffer" in rows[i - 1][0]
            if "batch_pass_a_kernel" in rows[i][0] and not trial and i + 1 < len(rows) and \
                    ("batch_scan_kernel" in rows[i + 1][0] or "batch_combine_kernel" in rows[i + 1][0]):
                j = i + 1
                while j < len(rows) and rows[j][0].lstrip("void ").startswith("sk::batch_") and \
                        "batch_pass_a_kernel" not in rows[j][0]:
                    j += 1
                seqs.append(rows[i:j])
                i = j
                continue
            i += 1
        groups = collections.defaultdict(list)
        for sq in seqs:
            groups[tuple(k[0] for k in sq)].append(sq)
        for names_k, gs in sorted(groups.items(), key=lambda kv: (len(kv[0]), kv[0])):
            n_k = len(names_k)
            pa = [(g[0][2] - g[0][1]) / 1e3 for g in gs]
            pb = [(g[-1][2] - g[1][1]) / 1e3 for g in gs]
            wall = [(g[-1][2] - g[0][1]) / 1e3 for g in gs]
            out.append(f"  {len(gs)} calls of {n_k} kernels: pass A avg {statistics.fmean(pa):.2f} us "
                       f"(min {min(pa):.2f}), pass B first start to last end avg {statistics.fmean(pb):.2f} us, "
                       f"call first start to last end avg {statistics.fmean(wall):.2f} us")
            names = [_short(k[0], 40) for k in gs[0]]
            durs = [statistics.fmean([(g[m][2] - g[m][1]) / 1e3 for g in gs]) for m in range(n_k)]
            out.append("    " + " | ".join(f"{n} {t:.1f}" for n, t in zip(names, durs)))
    return "\n".join(out)


def _counter_means(d: str):
    con = _db(d)
    res = collections.defaultdict(lambda: collections.defaultdict(list))
    for name, counter, value in con.execute("select kernel_name, counter_name, value from counters_collection"):
        res[name][counter].append(value)
    return res


def counters(fetch_dir: str, write_dir: str, copy_bytes: int) -> dict:
    f = _counter_means(fetch_dir)
    w = _counter_means(write_dir)
    copy = [k for k in f if "copyBuffer" in k]
    fetch_scale = write_scale = None
    if copy and copy_bytes:
        fk = max(f[copy[0]]["FETCH_SIZE"])
        wk = max(w[copy[0]]["WRITE_SIZE"]) if copy[0] in w else None
        fetch_scale = copy_bytes / (fk * 1024.0)
        write_scale = copy_bytes / (wk * 1024.0) if wk else None
    table = {}
    for k in sorted(set(f) | set(w)):
        fv = f.get(k, {}).get("FETCH_SIZE", [])
        wv = w.get(k, {}).get("WRITE_SIZE", [])
        table[k] = {"dispatches": max(len(fv), len(wv)),
                    "fetch_kib": statistics.fmean(fv) if fv else None,
                    "write_kib": statistics.fmean(wv) if wv else None}
    return {"fetch_scale": fetch_scale, "write_scale": write_scale, "copy_bytes": copy_bytes, "kernels": table}


def counters_text(c: dict) -> str:
    out = [f"copy probe: {c['copy_bytes']} bytes read and written by one device copy; "
           f"FETCH_SIZE scale {c['fetch_scale']:.4f}, WRITE_SIZE scale {c['write_scale']:.4f} (bytes per KiB read)"
           if c["fetch_scale"] and c["write_scale"] else "no copy probe found: unscaled KiB only"]
    out.append(f"{'kernel':70s} {'n':>4s} {'FETCH KiB':>14s} {'WRITE KiB':>14s} {'HBM MB (scaled)':>16s}")
    for k, v in sorted(c["kernels"].items(), key=lambda kv: -((kv[1]["fetch_kib"] or 0) + (kv[1]["write_kib"] or 0))):
        mb = ""
        if c["fetch_scale"] and c["write_scale"] and v["fetch_kib"] is not None and v["write_kib"] is not None:
            mb = f"{(v['fetch_kib'] * 1024 * c['fetch_scale'] + v['write_kib'] * 1024 * c['write_scale']) / 1e6:16.2f}"
        fk = f"{v['fetch_kib']:14.1f}" if v["fetch_kib"] is not None else f"{'-':>14s}"
        wk = f"{v['write_kib']:14.1f}" if v["write_kib"] is not None else f"{'-':>14s}"
        out.append(f"{_short(k):70s} {v['dispatches']:4d} {fk} {wk} {mb}")
    return "\n".join(out)


def pmc_text(d: str) -> str:
    res = _counter_means(d)
    out = []
    for k, cs in sorted(res.items()):
        out.append(_short(k, 100))
        for c, v in sorted(cs.items()):
            out.append(f"    {c:24s} n={len(v):4d} mean={statistics.fmean(v):16.1f} min={min(v):16.1f} max={max(v):16.1f}")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--calls", action="store_true")
    t.add_argument("--include", default="", help="only kernels whose name matches this regular expression")
    c = sub.add_parser("counters")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--copy-bytes", type=int, default=0)
    c.add_argument("--json", action="store_true")
    p = sub.add_parser("pmc")
    p.add_argument("dir")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace(a.dir, a.calls, a.include))
    elif a.cmd == "counters":
        r = counters(a.fetch_dir, a.write_dir, a.copy_bytes)
        print(json.dumps(r, indent=1) if a.json else counters_text(r))
    else:
        print(pmc_text(a.dir))


if __name__ == "__main__":
    sys.exit(main())
