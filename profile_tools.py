"""Summaries of rocprofv3 output for the measurement of libvie (not part of
the library).

    python profile_tools.py summary OUT_DIR [--top N] [--tail NAME K] [--window NAME START K] [--drop-trace]
    python profile_tools.py traffic FETCH_DIR WRITE_DIR WORKLOAD OUT.json [VALU_DIR]

``summary`` (a ``--kernel-trace --stats --output-format csv`` run): kernels by
total time (calls, total, mean), the trace's span, busy and idle time, the
distribution of idle gaps between consecutive kernels with the kernel pairs
that account for most of the long gaps, and the same per hardware queue;
``--tail NAME K``: mean, minimum and maximum duration of the last K
launches of the kernel whose name contains NAME; ``--window NAME START K``
(repeatable): the same for launches START .. START + K - 1 in time order.
``--drop-trace`` deletes the per-dispatch trace CSV afterwards (it can be
hundreds of MB for a whole solve).

``traffic`` (two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of a program
that also copies 512 MiB device to device, ``bench.py --calibration-copy``):
each counter is scaled by the factor that makes it read the copy's true byte
count (the largest ``__amd_rocclr_copyBuffer`` dispatches); the result is the
mean HBM bytes per dispatch of every z-pass kernel, written with a hash of
the kernel sources (``kernel_hash``) so that a reader can tell whether the
numbers still describe the current kernels.  VALU_DIR (optional): a ``--pmc
SQ_INSTS_VALU`` run of the same program (mean wavefront VALU instructions per
dispatch).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(ROOT, "paper_2501_13512_amd", "csrc")
COPY_BYTES = 512 * 1024 * 1024


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("mvm.hip", "fft_core.h", "cx.h"):
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def _find(d, suffix):
    f = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    return f[0] if f else None


def summarize(d: str, top: int = 40, tail=None, window=None) -> str:
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
        # kernels of several streams overlap: busy time is the union of the
        # kernels' intervals, a gap is a stretch where no kernel runs
        gaps = []
        busy_ns = 0
        cur_s, cur_e, cur_n = t[0]
        for s0, e0, n0 in t[1:]:
            if s0 > cur_e:
                busy_ns += cur_e - cur_s
                gaps.append(((s0 - cur_e) / 1e3, cur_n[:44], n0[:44]))
                cur_s, cur_e, cur_n = s0, e0, n0
            elif e0 > cur_e:
                cur_e, cur_n = e0, n0
        busy_ns += cur_e - cur_s
        busy = busy_ns / 1e6
        kern = sum(e - s for s, e, _ in t) / 1e6
        out.append(f"trace: {len(t)} kernels, span {span:.1f} ms, busy {busy:.1f} ms (some kernel running), "
                   f"idle {span - busy:.1f} ms, summed kernel time {kern:.1f} ms")
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
        out += _per_queue(trace)
        if tail:
            name, k = tail[0], int(tail[1])
            d_us = [(e - s0) / 1e3 for s0, e, n in t if name in n][-k:]
            if d_us:
                out.append(f"last {len(d_us)} launches of '{name}': mean {sum(d_us) / len(d_us):.2f} us, "
                           f"min {min(d_us):.2f}, max {max(d_us):.2f}")
        for name, start, k in window or []:
            all_us = [(e - s0) / 1e3 for s0, e, n in t if name in n]
            d_us = all_us[int(start):int(start) + int(k)]
            if d_us:
                out.append(f"launches {start}..{int(start) + len(d_us) - 1} of {len(all_us)} of '{name}' "
                           f"(in time order): mean {sum(d_us) / len(d_us):.2f} us, min {min(d_us):.2f}, "
                           f"max {max(d_us):.2f}, summed {sum(d_us) / 1e3:.1f} ms")
    return "\n".join(out)


def _per_queue(trace):
    """Per hardware queue (one per HIP stream in use): kernels, summed
    kernel time, the union of its kernels' intervals, and the kernels that
    take most of its time (the queue whose busy time is near the trace's
    span is the critical path)."""
    q = collections.defaultdict(list)
    for r in csv.DictReader(open(trace)):
        key = r.get("Queue_Id") or r.get("Stream_Id") or "0"
        q[key].append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    out = []
    for key, t in sorted(q.items(), key=lambda kv: -len(kv[1])):
        t.sort()
        busy, (cs, ce) = 0, t[0][:2]
        for s0, e0, _ in t[1:]:
            if s0 > ce:
                busy += ce - cs
                cs, ce = s0, e0
            elif e0 > ce:
                ce = e0
        busy += ce - cs
        span = t[-1][1] - t[0][0]
        per = collections.Counter()
        cnt = collections.Counter()
        for s0, e0, n in t:
            per[n] += e0 - s0
            cnt[n] += 1
        out.append(f"queue {key}: {len(t)} kernels, span {span / 1e6:.1f} ms, busy {busy / 1e6:.1f} ms, "
                   f"summed {sum(per.values()) / 1e6:.1f} ms")
        for n, ns in per.most_common(8):
            out.append(f"    {ns / 1e6:9.2f} ms {cnt[n]:8d} x {ns / cnt[n] / 1e3:7.2f} us  {n[:90]}")
        # this queue's idle time between consecutive kernels, by kernel pair
        pairs = collections.defaultdict(list)
        for (s0, e0, n0), (s1, _, n1) in zip(t, t[1:]):
            if s1 > e0:
                pairs[(n0.split("(")[0][-40:], n1.split("(")[0][-40:])].append(s1 - e0)
        for (a, b), g in sorted(pairs.items(), key=lambda kv: -sum(kv[1]))[:6]:
            g.sort()
            out.append(f"    idle {sum(g) / 1e6:8.2f} ms {len(g):7d} x median {g[len(g) // 2] / 1e3:7.2f} us  "
                       f"after {a} -> {b}")
    return out


def _rows(d):
    out = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        out += list(csv.DictReader(open(f)))
    return out


def _per_kernel(rows):
    acc = {}
    for r in rows:
        acc.setdefault(r["Kernel_Name"], []).append((int(r["Grid_Size"]), float(r["Counter_Value"])))
    return acc


def _label(name):
    m = re.search(r"k_zconv_col<(float|double), (\d+), (\d+)(?:, (\d+))?>", name)
    if m:   # the fourth template argument: 1 = rooftop spectral multiply
        kind = ", rooftop" if m.group(4) == "1" else ""
        return f"k_zconv_col<V{m.group(3)}{kind}>", m.group(1), int(m.group(2))
    m = re.search(r"k_zconv_mirror<(float|double), (\d+)>", name)
    if m:
        return "k_zconv_mirror", m.group(1), int(m.group(2))
    return None


def traffic(fetch_dir, write_dir, workload, out, valu_dir=None):
    fk = _per_kernel(_rows(fetch_dir))
    wk = _per_kernel(_rows(write_dir))
    vk = _per_kernel(_rows(valu_dir)) if valu_dir else {}
    copy = "__amd_rocclr_copyBuffer"
    fc = max(fk[copy], key=lambda t: t[0])
    big_f = [v for g, v in fk[copy] if g == fc[0]]
    big_w = [v for g, v in wk[copy] if g == fc[0]]
    f_factor = COPY_BYTES / (1024 * sum(big_f) / len(big_f))
    w_factor = COPY_BYTES / (1024 * sum(big_w) / len(big_w))
    entries = []
    for name, vals in fk.items():
        lab = _label(name)
        if not lab or name not in wk:
            continue
        kib_f = sum(v for _, v in vals) / len(vals)
        kib_w = sum(v for _, v in wk[name]) / len(wk[name])
        entries.append({"kernel": lab[0], "precision": lab[1], "lz": lab[2], "rocprof_name": name,
                        "workload": workload, "dispatches": len(vals),
                        "fetch_kib": kib_f, "write_kib": kib_w,
                        "bytes_per_launch": 1024 * (kib_f * f_factor + kib_w * w_factor),
                        "source_hash": kernel_hash()})
        if name in vk:
            entries[-1]["valu_insts_per_launch"] = sum(v for _, v in vk[name]) / len(vk[name])
    doc = {"note": "HBM bytes per dispatch = FETCH_SIZE * f + WRITE_SIZE * w (KiB * 1024); f, w make the counters "
                   "read the true bytes of a 512 MiB device copy in the same runs",
           "fetch_factor": f_factor, "write_factor": w_factor, "entries": entries}
    json.dump(doc, open(out, "w"), indent=1)
    print(json.dumps({"fetch_factor": f_factor, "write_factor": w_factor, "n": len(entries)}))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "traffic":
        traffic(*sys.argv[2:7])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["summary"])
    ap.add_argument("dir")
    ap.add_argument("--top", type=int, default=40)
    ap.add_argument("--tail", nargs=2, metavar=("NAME", "K"))
    ap.add_argument("--window", nargs=3, action="append", metavar=("NAME", "START", "K"))
    ap.add_argument("--drop-trace", action="store_true")
    a = ap.parse_args()
    print(summarize(a.dir, a.top, a.tail, a.window), flush=True)
    if a.drop_trace:
        tr = _find(a.dir, "kernel_trace.csv")
        if tr:
            os.remove(tr)


if __name__ == "__main__":
    main()
