"""The stored full-size oracle reference files (tests/golden/oracle_metasurface*.json,
written by tests/golden/make_goldens.py from oracle/ only) are consistent:
same sampled voxels, the tight solve reached 1e-10, and the solve at the
case tolerance (1e-5) is close to the tight one but measurably not equal
(a 1e-5 residual leaves a field error of a few 1e-5)."""
import json
import os

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    g = json.load(open(os.path.join(HERE, name)))
    return g, np.asarray(g["etot_re"]) + 1j * np.asarray(g["etot_im"])


def test_metasurface_reference_files_agree():
    a, ea = _load("oracle_metasurface.json")
    b, eb = _load("oracle_metasurface_tight.json")
    assert a["voxels_xyz"] == b["voxels_xyz"]
    assert len(a["voxels_xyz"]) == 1024
    assert a["status"] == b["status"] == "converged"
    assert b["history"][-1] <= 1e-10
    assert a["history"][-1] <= a["tol_outer"]
    d = np.linalg.norm(ea - eb) / np.linalg.norm(eb)
    assert 1e-7 < d < 1e-4
    assert abs(a["etot_norm"] - b["etot_norm"]) <= 1e-4 * b["etot_norm"]
    # every preconditioner application recorded one count per block
    assert all(len(app) == 65 for app in a["inner_counts"])
    assert len(a["inner_counts"]) in (2 * a["outer_iters"] - 1, 2 * a["outer_iters"])
