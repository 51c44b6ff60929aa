"""Write the oracle reference files of the full-size metasurface case and of the first outer steps on the plasmonic cell.

Calls only ``oracle/`` and ``workloads``.  Each run writes
``oracle_metasurface_<run>.json`` (settings, outer step count, residual
history, inner step counts of every preconditioner application, refinement
counts, timing) and ``oracle_metasurface_<run>_etot.npy``: E_tot at every
scatterer voxel, [3, n] in the order of ``numpy.nonzero(mask)`` over the
[z, y, x] grid; complex128 for ``tight`` (compared to 1e-10), complex64 for
the others (compared at the 1e-5 level; ``shrink`` converts a complex128
file).  The pad-4 runs' fields serve only the spread file and are not
kept in the repository.

Runs (the case is 128x128x32 at lambda/40, 64 pillar blocks + slab):

* ``tight``       FP64, no preconditioner, outer tolerance 1e-12 (the
                  discrete solution is unique, so every converged variant
                  reaches it);
* ``case``        FP64 block-preconditioned at the case tolerances (outer
                  1e-5, inner 1e-2), circulant lengths 2n;
* ``case_pad4``   the same with every circulant length 2n + 4 (the same
                  operator with different rounding: how far rounding alone
                  moves the iterates at these tolerances);
* ``mixed``       complex64 products with FP64 refinement, block
                  preconditioned at the benchmark's settings (outer 2e-6,
                  inner 1e-2, at most 3 corrections);
* ``mixed_pad4``  the same with lengths 2n + 4;
* ``bench_fp64``  FP64 block-preconditioned at the benchmark's settings;
* ``shrink``      rewrites the non-tight fields as complex64;
* ``spread``      reads the stored fields and writes
                  ``oracle_metasurface_spread.json``: relative field
                  differences between the runs and the step counts side by
                  side;
* ``plasmonic_first``  the plasmonic cell (96x96x64 at lambda/40: 16 metal
                  sphere blocks, the absorbing layer and the slab), FP64
                  block-preconditioned at its tolerances (outer 1e-6, inner
                  3e-2), capped at 3 outer steps: the residual after every
                  step and the inner step counts of every application
                  (``oracle_plasmonic_first.json``, no field).
* ``plasmonic_small_tight``  the reduced plasmonic cell (48x48x32, 2x2
                  spheres), FP64 without preconditioner to 1e-8: E_tot at
                  every voxel of the cell, complex128
                  (``oracle_plasmonic_small_tight_etot.npy``).

BLAS is held to one thread so inner products are summed in a fixed order
(the results do not depend on the machine's core count); ``--workers`` only
splits independent FFTs.

    python tests/golden/make_goldens.py --workers 4 tight
    python tests/golden/make_goldens.py case
    python tests/golden/make_goldens.py spread
"""
import os

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import json  # noqa: E402
import sys  # noqa: E402
import time  # noqa: E402

import numpy as np  # noqa: E402
import scipy.fft  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import krylov, operator as op, physics  # noqa: E402

CASE = "metasurface"
TIGHT_TOL = 1e-12
BENCH_TOL = 2e-6

RUNS = {
    "tight": dict(kind="fp64", prec=False, tol=TIGHT_TOL, maxit=20000, pad=0),
    "case": dict(kind="fp64", prec=True, tol=None, pad=0),
    "case_pad4": dict(kind="fp64", prec=True, tol=None, pad=4),
    "mixed": dict(kind="mixed", prec=True, tol=BENCH_TOL, pad=0),
    "mixed_pad4": dict(kind="mixed", prec=True, tol=BENCH_TOL, pad=4),
    "bench_fp64": dict(kind="fp64", prec=True, tol=BENCH_TOL, pad=0),
    "plasmonic_first": dict(kind="fp64", prec=True, tol=None, pad=0, maxit=3, case="plasmonic", field=False),
    "plasmonic_small_tight": dict(kind="fp64", prec=False, tol=1e-8, maxit=20000, pad=0, case="plasmonic_small",
                                  exact=True),
}


def path(run, ext):
    suffix = "_etot.npy" if ext == "npy" else ".json"
    if run.startswith("plasmonic"):
        return os.path.join(HERE, f"oracle_{run}{suffix}")
    return os.path.join(HERE, f"oracle_{CASE}_{run}{suffix}")


def scatterer_values(g, E):
    k, j, i = np.nonzero(g.mask)
    return np.ascontiguousarray(E[:, k, j, i])


def run(name: str) -> dict:
    spec = RUNS[name]
    case = W.by_name(spec.get("case", CASE))
    g = op.Grid.from_case(case)
    e = physics.plane_wave(g, case.kdir, case.pol)
    tol = spec["tol"] if spec["tol"] is not None else case.tol_outer
    maxit = spec.get("maxit", case.maxit_outer)
    blocks = (case.block_id, case.n_blocks) if spec["prec"] else (None, 0)
    t0 = time.time()
    if spec["kind"] == "mixed":
        sol = krylov.solve_mixed(g, e, tol, maxit, blocks[0], blocks[1], case.tol_inner, case.maxit_inner,
                                 max_refine=3, pad=spec["pad"])
    else:
        sol = krylov.solve(g, e, tol, maxit, blocks[0], blocks[1], case.tol_inner, case.maxit_inner,
                           pad=spec["pad"])
    secs = time.time() - t0
    d = {
        "case": case.name, "run": name,
        "source": "oracle/ (krylov.solve_mixed)" if spec["kind"] == "mixed" else "oracle/ (krylov.solve)",
        "script": "tests/golden/make_goldens.py",
        "precision": "complex64 products, FP64 vectors and refinement" if spec["kind"] == "mixed" else "FP64",
        "precondition": spec["prec"], "pad": spec["pad"],
        "tol_outer": tol, "maxit_outer": maxit,
        "outer_iters": sol.info.iterations, "status": sol.info.status, "half_step": sol.info.half_step,
        "history": sol.info.history,
        "etot_norm": float(np.linalg.norm(sol.E_tot)),
        "n_scatterer": int(np.count_nonzero(g.mask)),
        "oracle_seconds": secs,
    }
    if spec["prec"]:
        d["tol_inner"] = case.tol_inner
        d["maxit_inner"] = case.maxit_inner
        d["inner_counts"] = sol.inner_counts
    if spec["kind"] == "mixed":
        d.update(max_refine=3, refine_steps=sol.refine_steps, refine_iters=sol.refine_iters,
                 relres_true=sol.relres_true, true_history=sol.true_history)
    if spec.get("field", True):
        f = scatterer_values(g, sol.E_tot)
        exact = spec.get("exact", name == "tight")
        np.save(path(name, "npy"), f if exact else f.astype(np.complex64), allow_pickle=False)
    return d


def spread() -> dict:
    fields, meta = {}, {}
    for name in RUNS:
        if RUNS[name].get("case", CASE) != CASE:
            continue
        if os.path.exists(path(name, "npy")) and os.path.exists(path(name, "json")):
            fields[name] = np.load(path(name, "npy"), allow_pickle=False)
            meta[name] = json.load(open(path(name, "json")))
    out = {"case": CASE, "script": "tests/golden/make_goldens.py spread",
           "outer_iters": {k: v["outer_iters"] for k, v in meta.items()},
           "refine_steps": {k: v.get("refine_steps", 0) for k, v in meta.items()},
           "rel_field_diff": {}}
    names = sorted(fields)
    for a in names:
        for b in names:
            if a < b:
                out["rel_field_diff"][f"{a}|{b}"] = float(np.linalg.norm(fields[a] - fields[b]) /
                                                          np.linalg.norm(fields[b]))
    return out


if __name__ == "__main__":
    args = sys.argv[1:]
    workers = 1
    if "--workers" in args:
        i = args.index("--workers")
        workers = int(args[i + 1])
        del args[i:i + 2]
    for name in args:
        if name == "shrink":
            for run_name in RUNS:
                f = path(run_name, "npy")
                if run_name != "tight" and os.path.exists(f):
                    a = np.load(f, allow_pickle=False)
                    if a.dtype == np.complex128:
                        np.save(f, a.astype(np.complex64), allow_pickle=False)
                        print("shrunk", os.path.basename(f), flush=True)
            continue
        if name == "spread":
            d = spread()
            with open(os.path.join(HERE, f"oracle_{CASE}_spread.json"), "w") as f:
                json.dump(d, f, indent=1)
            print(json.dumps(d, indent=1), flush=True)
            continue
        with scipy.fft.set_workers(workers):
            d = run(name)
        with open(path(name, "json"), "w") as f:
            json.dump(d, f, separators=(",", ":"))
        print(name, d["outer_iters"], d["status"], d.get("refine_steps", ""), f"{d['oracle_seconds']:.0f}s",
              flush=True)
