"""C-ABI checks that need no GPU: the library loads, exports every entry
point of include/vie.h, validates arguments, and its host helper (the
incident plane wave) matches the oracle's."""
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import operator as op, physics, rooftop
from paper_2501_13512_amd import vie as V

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "vie.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vie_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported():
    syms = _header_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(V._lib, s), s
    assert sorted(V.ABI_SYMBOLS) == syms


def test_abi_version():
    assert V.vie_abi_version() == 15


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device error path")
def test_context_without_device_is_edevice():
    with pytest.raises(V.VieError) as e:
        V.vie_context_create(0)
    assert e.value.code == V.VIE_EDEVICE
    assert "device" in V.vie_last_error()


def test_null_arguments_are_einval():
    out = V._vp()
    assert V._lib.vie_context_create(0, 0, None) == V.VIE_EINVAL
    g = V.make_grid(2, 2, 2, 1, 1, 1, 10)
    assert V._lib.vie_problem_create(None, V.ctypes.byref(g), None, None, 0, V.ctypes.byref(out)) == V.VIE_EINVAL
    assert V._lib.vie_matvec(None, 0, None, None, None) == V.VIE_EINVAL
    assert V._lib.vie_solve(None, None, None, None, None, None) == V.VIE_EINVAL
    assert V._lib.vie_problem_get_info(None, None) == V.VIE_EINVAL
    assert V._lib.vie_problem_destroy(None) == V.VIE_OK
    assert V._lib.vie_context_destroy(None) == V.VIE_OK


@pytest.mark.parametrize("kdir,pol", [((0, 0, 1), (1, 0, 0)), ((0.6, 0, 0.8), (0.8, 0, -0.6)),
                                      ((0, 1, 0), (0, 0, 1j))])
def test_plane_wave_matches_oracle(kdir, pol):
    case = W.random_tiny(3, (5, 4, 7), spacing=(0.03, 0.05, 0.04), wavelength=0.7)
    g = op.Grid.from_case(case)
    want = physics.plane_wave(g, kdir, pol)
    got = V.vie_plane_wave(V.make_grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.wavelength),
                           kdir, pol)
    assert np.abs(got - want).max() <= 1e-13


@pytest.mark.parametrize("kdir,pol", [((0, 0, 1), (1, 0, 0)), ((0.6, 0, 0.8), (0.8, 0, -0.6)),
                                      ((0, 1, 0), (0, 0, 1j))])
def test_face_plane_wave_matches_rooftop_oracle(kdir, pol):
    """The rooftop unknowns' incident field: component c at its face centre,
    half a cell along axis c from the voxel centre."""
    case = W.random_tiny(4, (5, 4, 7), spacing=(0.03, 0.05, 0.04), wavelength=0.7)
    g = op.Grid.from_case(case)
    want = rooftop.plane_wave(g, kdir, pol)
    got = V.vie_plane_wave_faces(V.make_grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz,
                                             case.wavelength), kdir, pol)
    assert np.abs(got - want).max() <= 1e-13


def test_plane_wave_rejects_non_unit_direction():
    g = V.make_grid(2, 2, 2, 1, 1, 1, 10)
    with pytest.raises(V.VieError) as e:
        V.vie_plane_wave(g, (0, 0, 2), (1, 0, 0))
    assert e.value.code == V.VIE_EINVAL


def test_plan_of_the_metasurface_case():
    """Host-only block plan: the metasurface's 64 pillar boxes form one shape
    group on a 32x32x48 transform, the slab another on 256x256x16; the full
    grid uses 256x256x64."""
    case = W.metasurface()
    g = V.make_grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.wavelength)
    info, groups, bgrp = V.vie_plan(g, case.eps, case.block_id, case.n_blocks)
    assert (info.lx, info.ly, info.lz) == (256, 256, 64)
    assert info.n_blocks == 65 and info.n_groups == len(groups) == 2
    shapes = sorted(((gp.lx, gp.ly, gp.lz), gp.n_systems) for gp in groups)
    assert shapes == [((32, 32, 48), 64), ((256, 256, 16), 1)]
    pillar = [i for i, gp in enumerate(groups) if gp.n_systems == 64][0]
    assert list(bgrp[:64]) == [pillar] * 64 and bgrp[64] == 1 - pillar
    assert info.footprint_bytes > 0 and info.zpass_variant[0] == -1
    with pytest.raises(V.VieError) as e:
        bad = case.block_id.copy()
        bad[tuple(np.argwhere(case.eps != 1)[0])] = case.n_blocks   # out of range on a scatterer voxel
        V.vie_plan(g, case.eps, bad, case.n_blocks)
    assert e.value.code == V.VIE_EINVAL
