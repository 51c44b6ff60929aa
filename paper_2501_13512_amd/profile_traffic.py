"""HBM traffic per launch of libvie kernels from rocprofv3 counter runs.

    python -m paper_2501_13512_amd.profile_traffic FETCH_DIR WRITE_DIR WORKLOAD OUT.json [VALU_DIR]

FETCH_DIR / WRITE_DIR: output directories of two ``rocprofv3 --pmc FETCH_SIZE``
and ``rocprofv3 --pmc WRITE_SIZE`` runs (``--output-format csv``) of a
program that also copies 512 MiB device to device (``bench.py
--calibration-copy``).  Each counter is scaled by the factor that makes it
read the copy's true byte count (the largest ``__amd_rocclr_copyBuffer``
dispatches); the result is the mean HBM bytes per dispatch of every z-pass
kernel variant, written with a hash of the kernel sources so that a reader
can tell whether the numbers still describe the current kernels.
VALU_DIR (optional): a ``rocprofv3 --pmc SQ_INSTS_VALU`` run of the same
program; adds the mean wavefront VALU instructions per dispatch.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 512 * 1024 * 1024


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("mvm.hip", "fft_core.h", "cx.h"):
        h.update(open(os.path.join(PKG, "csrc", f), "rb").read())
    return h.hexdigest()[:16]


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
    m = re.search(r"k_zconv_col<(float|double), (\d+), (\d+)>", name)
    if m:
        return f"k_zconv_col<V{m.group(3)}>", m.group(1), int(m.group(2))
    m = re.search(r"k_zconv_mirror<(float|double), (\d+)>", name)
    if m:
        return "k_zconv_mirror", m.group(1), int(m.group(2))
    return None


def main(fetch_dir, write_dir, workload, out, valu_dir=None):
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


if __name__ == "__main__":
    main(*sys.argv[1:6])
