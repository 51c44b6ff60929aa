"""Text summary of a rocprofv3 kernel trace (``--kernel-trace --stats
--output-format csv``).

    python -m paper_2501_13512_amd.profile_summary OUT_DIR [--top N] [--tail NAME K] [--drop-trace]

Prints the kernels by total time (calls, total, mean), the trace's span,
busy and idle time, and the distribution of idle gaps between consecutive
kernels with the kernel pairs that account for most of the long gaps.
``--tail NAME K`` adds the mean, minimum and maximum duration of the last K
launches of the kernel whose name contains NAME (e.g. a benchmark's timed
repetitions at the end of a run).
``--drop-trace`` deletes the per-dispatch trace CSV afterwards (it can be
hundreds of MB for a whole solve).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import os


def _find(d, suffix):
    f = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    return f[0] if f else None


def summarize(d: str, top: int = 40, tail=None) -> str:
    out = []
    stats = _find(d, "kernel_stats.csv")
    if stats:
        rows = list(csv.DictReader(open(stats)))
        tot = sum(float(r["TotalDurationNs"]) for r in rows)
        out.append(f"{'kernel':72s} {'calls':>8s} {'total ms':>10s} {'avg us':>9s} {'%':>6s}")
        for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
            out.append(f"{r['Name'][:72]:72s} {int(r['Calls']):8d} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                       f"{float(r['AverageNs']) / 1e3:9.2f} {100 * float(r['TotalDurationNs']) / tot:6.2f}")
        out.append(f"total kernel time {tot / 1e6:.1f} ms")
    trace = _find(d, "kernel_trace.csv")
    if trace:
        t = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"])
             for r in csv.DictReader(open(trace))]
        t.sort()
        span = (t[-1][1] - t[0][0]) / 1e6
        busy = sum(e - s for s, e, _ in t) / 1e6
        out.append(f"trace: {len(t)} kernels, span {span:.1f} ms, busy {busy:.1f} ms, idle {span - busy:.1f} ms")
        gaps = [((b[0] - a[1]) / 1e3, a[2][:44], b[2][:44]) for a, b in zip(t[:-1], t[1:])]
        gv = sorted(g for g, _, _ in gaps)
        n = len(gv)
        if n:
            out.append(f"gaps us: median {gv[n // 2]:.2f} p90 {gv[int(n * .9)]:.2f} p99 {gv[int(n * .99)]:.2f} "
                       f"max {gv[-1]:.1f}")
            for th in (10, 20, 50, 100):
                out.append(f"  idle in gaps > {th} us: {sum(x for x in gv if x > th) / 1e3:.1f} ms "
                           f"({sum(1 for x in gv if x > th)} gaps)")
            big = collections.Counter()
            for g, a, b in gaps:
                if g > 20:
                    big[(a, b)] += g
            for (a, b), s in big.most_common(8):
                out.append(f"  {s / 1e3:8.2f} ms after {a} -> {b}")
        if tail:
            name, k = tail[0], int(tail[1])
            d_us = [(e - s0) / 1e3 for s0, e, n in t if name in n][-k:]
            if d_us:
                out.append(f"last {len(d_us)} launches of '{name}': mean {sum(d_us) / len(d_us):.2f} us, "
                           f"min {min(d_us):.2f}, max {max(d_us):.2f}")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("--top", type=int, default=40)
    ap.add_argument("--tail", nargs=2, metavar=("NAME", "K"))
    ap.add_argument("--drop-trace", action="store_true")
    a = ap.parse_args()
    print(summarize(a.dir, a.top, a.tail), flush=True)
    if a.drop_trace:
        tr = _find(a.dir, "kernel_trace.csv")
        if tr:
            os.remove(tr)


if __name__ == "__main__":
    main()
