"""Write the oracle reference files for the full-size benchmark cases.

Calls only ``oracle/`` and ``workloads``.  For each case it runs the FP64
oracle solve at the case's tolerances (block preconditioner) and stores:
outer step count, the inner step counts of every preconditioner
application, the residual history, the norm of E_tot over the scatterer,
and E_tot at 1024 scatterer voxels drawn with default_rng(99).

    python tests/golden/make_goldens.py metasurface plasmonic
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import krylov, operator as op, physics  # noqa: E402


def golden(name: str) -> dict:
    case = W.by_name(name)
    g = op.Grid.from_case(case)
    e = physics.plane_wave(g, case.kdir, case.pol)
    t0 = time.time()
    sol = krylov.solve(g, e, case.tol_outer, case.maxit_outer, case.block_id, case.n_blocks,
                       case.tol_inner, case.maxit_inner)
    secs = time.time() - t0
    k, j, i = np.nonzero(g.mask)
    rng = np.random.default_rng(99)
    pick = np.sort(rng.choice(i.size, size=min(1024, i.size), replace=False))
    vox = np.stack([i[pick], j[pick], k[pick]], axis=1)
    E = sol.E_tot[:, k[pick], j[pick], i[pick]]          # [3, n]
    return {
        "case": name,
        "source": "oracle FP64 solve (oracle/krylov.py solve) at the case tolerances; tests/golden/make_goldens.py",
        "tol_outer": case.tol_outer, "tol_inner": case.tol_inner,
        "outer_iters": sol.info.iterations, "status": sol.info.status,
        "inner_counts": sol.inner_counts, "history": sol.info.history,
        "etot_norm": float(np.linalg.norm(sol.E_tot)),
        "voxels_xyz": vox.tolist(),
        "etot_re": E.real.tolist(), "etot_im": E.imag.tolist(),
        "oracle_seconds": secs,
    }


if __name__ == "__main__":
    for name in sys.argv[1:]:
        d = golden(name)
        path = os.path.join(HERE, f"oracle_{name}.json")
        with open(path, "w") as f:
            json.dump(d, f, separators=(",", ":"))
        print(name, d["outer_iters"], d["status"], f"{d['oracle_seconds']:.0f}s", flush=True)
