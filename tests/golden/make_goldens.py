"""Write the oracle reference files for the full-size benchmark cases.

Calls only ``oracle/`` and ``workloads``.  Two kinds of file per case:

* ``oracle_<case>.json``: the FP64 oracle solve at the case's tolerances
  (block preconditioner): outer step count, the inner step counts of every
  preconditioner application, the residual history, the norm of E_tot over
  the scatterer, and E_tot at 1024 scatterer voxels drawn with
  default_rng(99).
* ``oracle_<case>_tight.json`` (``--tight``): the FP64 oracle solve without
  preconditioner to relative residual 1e-10 (the discrete solution is
  unique, so any converged variant reaches it), E_tot at the same voxels.

    python tests/golden/make_goldens.py metasurface
    python tests/golden/make_goldens.py --tight metasurface
"""
import json
import os
import sys
import time

import numpy as np
import scipy.fft

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import krylov, operator as op, physics  # noqa: E402

TIGHT_TOL = 1e-10


def _samples(g, E):
    k, j, i = np.nonzero(g.mask)
    rng = np.random.default_rng(99)
    pick = np.sort(rng.choice(i.size, size=min(1024, i.size), replace=False))
    vox = np.stack([i[pick], j[pick], k[pick]], axis=1)
    return vox, E[:, k[pick], j[pick], i[pick]]          # [3, n]


def golden(name: str, tight: bool) -> dict:
    case = W.by_name(name)
    g = op.Grid.from_case(case)
    e = physics.plane_wave(g, case.kdir, case.pol)
    t0 = time.time()
    if tight:
        sol = krylov.solve(g, e, TIGHT_TOL, 20000)
    else:
        sol = krylov.solve(g, e, case.tol_outer, case.maxit_outer, case.block_id, case.n_blocks,
                           case.tol_inner, case.maxit_inner)
    secs = time.time() - t0
    vox, E = _samples(g, sol.E_tot)
    d = {
        "case": name,
        "source": ("oracle FP64 solve without preconditioner to relative residual 1e-10" if tight else
                   "oracle FP64 solve (oracle/krylov.py solve) at the case tolerances") +
                  "; tests/golden/make_goldens.py",
        "tol_outer": TIGHT_TOL if tight else case.tol_outer,
        "outer_iters": sol.info.iterations, "status": sol.info.status,
        "history": sol.info.history,
        "etot_norm": float(np.linalg.norm(sol.E_tot)),
        "voxels_xyz": vox.tolist(),
        "etot_re": E.real.tolist(), "etot_im": E.imag.tolist(),
        "oracle_seconds": secs,
    }
    if not tight:
        d["tol_inner"] = case.tol_inner
        d["inner_counts"] = sol.inner_counts
    return d


if __name__ == "__main__":
    args = sys.argv[1:]
    tight = "--tight" in args
    names = [a for a in args if not a.startswith("--")]
    with scipy.fft.set_workers(os.cpu_count() or 1):   # independent transforms, same results
        for name in names:
            d = golden(name, tight)
            path = os.path.join(HERE, f"oracle_{name}{'_tight' if tight else ''}.json")
            with open(path, "w") as f:
                json.dump(d, f, separators=(",", ":"))
            print(name, d["outer_iters"], d["status"], f"{d['oracle_seconds']:.0f}s", flush=True)
