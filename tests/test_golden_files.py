"""The stored full-size oracle reference files (tests/golden/
oracle_metasurface_*.json and *_etot.npy, written by
tests/golden/make_goldens.py from oracle/ only) are consistent: every run
converged, the fields cover every scatterer voxel (complex128 for the tight
solve, complex64 for the others), the tight (1e-12) field
is the reference the others approach (a solve to 1e-5 or 2e-6 is close to
it but measurably not equal), the mixed-precision runs ended with an FP64
true residual at their tolerance, and the spread file matches the fields."""
import json
import os

import numpy as np
import pytest

import workloads as W

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(run):
    meta = json.load(open(os.path.join(HERE, f"oracle_metasurface_{run}.json")))
    path = os.path.join(HERE, f"oracle_metasurface_{run}_etot.npy")
    return meta, (np.load(path, allow_pickle=False) if os.path.exists(path) else None)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_metasurface_reference_files_agree():
    case = W.metasurface()
    n_s = int(np.count_nonzero(case.eps != 1.0))
    tight, et = _load("tight")
    assert tight["status"] == "converged" and tight["history"][-1] <= 1e-12
    assert et.shape == (3, n_s) and et.dtype == np.complex128
    c, ec = _load("case")
    assert c["status"] == "converged" and c["history"][-1] <= c["tol_outer"] == case.tol_outer
    assert ec.shape == et.shape
    assert 1e-7 < _rel(ec, et) < 1e-4
    # every preconditioner application recorded one count per block
    assert all(len(app) == 65 for app in c["inner_counts"])
    assert len(c["inner_counts"]) in (2 * c["outer_iters"] - 1, 2 * c["outer_iters"])
    m, em = _load("mixed")
    assert m["relres_true"] <= m["tol_outer"] and m["refine_steps"] <= m["max_refine"]
    if em is not None:
        assert _rel(em, et) < 1e-4
    sp = json.load(open(os.path.join(HERE, "oracle_metasurface_spread.json")))
    assert sp["outer_iters"]["case"] == c["outer_iters"] and sp["outer_iters"]["mixed"] == m["outer_iters"]
    # the spread file was written from the complex128 fields; the stored
    # case field is complex64 (rounding ~1e-7 relative)
    assert ec.dtype == np.complex64
    assert sp["rel_field_diff"]["case|tight"] == pytest.approx(_rel(ec, et), rel=1e-3)
    assert 0 < sp["rel_field_diff"]["case|case_pad4"] < 1e-4


def test_plasmonic_small_reference_file():
    """The reduced plasmonic cell's plain FP64 oracle solve (the reference of
    the GPU's flexible-GMRES block-preconditioned solves): converged to 1e-8,
    E_tot at every voxel of the cell, complex128."""
    case = W.plasmonic_small()
    n_s = int(np.count_nonzero(case.eps != 1.0))
    meta = json.load(open(os.path.join(HERE, "oracle_plasmonic_small_tight.json")))
    assert meta["status"] == "converged" and meta["history"][-1] <= 1e-8 and not meta["precondition"]
    e = np.load(os.path.join(HERE, "oracle_plasmonic_small_tight_etot.npy"), allow_pickle=False)
    assert e.shape == (3, n_s) and e.dtype == np.complex128
    assert np.isfinite(e).all() and np.linalg.norm(e) == pytest.approx(meta["etot_norm"], rel=1e-12)
