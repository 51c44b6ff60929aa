"""Python binding of libvie (ctypes; argument marshalling only).

Every function below has the name of the C entry point it calls (see
``include/vie.h``) and does no arithmetic of its own: all steps of the solve
run in the HIP library.  Device buffers are torch tensors on the GPU
(complex128, contiguous, shape ``[3, nz, ny, nx]``); torch is used for device
memory and the current HIP stream only.

Importing this module loads ``libvie.so`` built in place by
``paper_2501_13512_amd.build``; it raises ``ImportError`` if the library is
missing, so nothing can silently fall back to another implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvie.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libvie.so is not built ({LIB_PATH}); run `python -m paper_2501_13512_amd.build`")


def _share_torch_hip_runtime() -> None:
    """PyTorch wheels bundle their own HIP runtime (same soname as the system
    one).  Loading it before libvie makes libvie bind to that copy, so the
    process has one HIP runtime whether torch or this module is imported
    first; with two, the runtime initialised second finds no device."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        return
    for d in spec.submodule_search_locations:
        hip = os.path.join(d, "lib", "libamdhip64.so")
        if os.path.exists(hip):
            ctypes.CDLL(hip, mode=ctypes.RTLD_GLOBAL)
            return


_share_torch_hip_runtime()
_lib = ctypes.CDLL(LIB_PATH)

VIE_OK, VIE_NOT_CONVERGED = 0, 1
VIE_EINVAL, VIE_ENOMEM, VIE_EDEVICE, VIE_EBREAKDOWN, VIE_EBUSY, VIE_ECANCELLED, VIE_EINTERNAL = -1, -2, -3, -4, -5, -6, -7
VIE_ETIMEDOUT = -8
VIE_FP64, VIE_MIXED, VIE_MIXED_INNER = 0, 1, 2
VIE_FLAG_NO_GRAPHS = 1
VIE_FLAG_NO_BLOCK_KERNEL = 2
VIE_SOLVER_BICGSTAB, VIE_SOLVER_FGMRES, VIE_SOLVER_CGS = 0, 1, 2
STATUS_NAMES = {0: "VIE_OK", 1: "VIE_NOT_CONVERGED", -1: "VIE_EINVAL", -2: "VIE_ENOMEM", -3: "VIE_EDEVICE",
                -4: "VIE_EBREAKDOWN", -5: "VIE_EBUSY", -6: "VIE_ECANCELLED", -7: "VIE_EINTERNAL", -8: "VIE_ETIMEDOUT"}

ABI_SYMBOLS = ("vie_abi_version", "vie_last_error", "vie_context_create", "vie_context_destroy",
               "vie_problem_create", "vie_problem_create_overlap", "vie_problem_create_rooftop", "vie_problem_destroy", "vie_problem_get_info", "vie_problem_set_zpass", "vie_problem_set_plane",
               "vie_plane_wave", "vie_plane_wave_faces", "vie_plan",
               "vie_matvec", "vie_matvec_profile", "vie_group_profile", "vie_block_matvec", "vie_precond_apply", "vie_solve", "vie_solve_device",
               "vie_solve_batch", "vie_solve_many",
               "vie_server_start", "vie_footprint", "vie_submit", "vie_wait", "vie_cancel",
               "vie_total_field_box", "vie_far_field", "vie_far_field_noalloc", "vie_rcs")


class VieError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__(f"{func}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class vie_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("wavelength", ctypes.c_double)]


class vie_opts(ctypes.Structure):
    _fields_ = [("tol_outer", ctypes.c_double), ("tol_inner", ctypes.c_double),
                ("maxit_outer", ctypes.c_int32), ("maxit_inner", ctypes.c_int32),
                ("max_refine", ctypes.c_int32), ("precondition", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("poll_lag", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("solver", ctypes.c_int32), ("restart", ctypes.c_int32)]


class vie_stats(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("refine_iters", ctypes.c_int32), ("final_state", ctypes.c_int32),
                ("inner_iters_total", ctypes.c_int64), ("precond_applies", ctypes.c_int64),
                ("relres_recursive", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("seconds", ctypes.c_double), ("inner_hist", ctypes.POINTER(ctypes.c_int32)),
                ("inner_hist_cap", ctypes.c_int64), ("inner_hist_len", ctypes.c_int64)]


class vie_problem_info(ctypes.Structure):
    _fields_ = [("lx", ctypes.c_int32), ("ly", ctypes.c_int32), ("lz", ctypes.c_int32),
                ("n_blocks", ctypes.c_int32), ("n_groups", ctypes.c_int32),
                ("footprint_bytes", ctypes.c_int64), ("n_block_solver_groups", ctypes.c_int32),
                ("zpass_variant", ctypes.c_int32 * 2), ("zpass_tune_ms", (ctypes.c_float * 5) * 2),
                ("plane_variant", ctypes.c_int32 * 2), ("plane_tune_ms", (ctypes.c_float * 3) * 2)]


class vie_group_plan(ctypes.Structure):
    _fields_ = [("lx", ctypes.c_int32), ("ly", ctypes.c_int32), ("lz", ctypes.c_int32),
                ("bx", ctypes.c_int32), ("by", ctypes.c_int32), ("bz", ctypes.c_int32),
                ("n_systems", ctypes.c_int32), ("one_workgroup", ctypes.c_int32)]


_vp = ctypes.c_void_p
_lib.vie_abi_version.restype = ctypes.c_int32
_lib.vie_abi_version.argtypes = []
_lib.vie_last_error.restype = ctypes.c_char_p
_lib.vie_last_error.argtypes = []
for _name, _args in {
    "vie_context_create": [ctypes.c_int32, ctypes.c_size_t, ctypes.POINTER(_vp)],
    "vie_context_destroy": [_vp],
    "vie_problem_create": [_vp, ctypes.POINTER(vie_grid), _vp, _vp, ctypes.c_int32, ctypes.POINTER(_vp)],
    "vie_problem_create_overlap": [_vp, ctypes.POINTER(vie_grid), _vp, _vp, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.POINTER(_vp)],
    "vie_problem_create_rooftop": [_vp, ctypes.POINTER(vie_grid), _vp, _vp, ctypes.c_int32, ctypes.POINTER(_vp)],
    "vie_problem_destroy": [_vp],
    "vie_problem_get_info": [_vp, ctypes.POINTER(vie_problem_info)],
    "vie_problem_set_zpass": [_vp, ctypes.c_int32, ctypes.c_int32],
    "vie_problem_set_plane": [_vp, ctypes.c_int32, ctypes.c_int32],
    "vie_plane_wave": [ctypes.POINTER(vie_grid), _vp, _vp, _vp],
    "vie_plane_wave_faces": [ctypes.POINTER(vie_grid), _vp, _vp, _vp],
    "vie_plan": [ctypes.POINTER(vie_grid), _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(vie_problem_info),
                 _vp, ctypes.c_int32, _vp],
    "vie_matvec": [_vp, ctypes.c_int32, _vp, _vp, _vp],
    "vie_matvec_profile": [_vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int32, _vp],
    "vie_group_profile": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp],
    "vie_block_matvec": [_vp, ctypes.c_int32, _vp, _vp, _vp],
    "vie_precond_apply": [_vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp,
                          ctypes.POINTER(ctypes.c_int64)],
    "vie_solve": [_vp, _vp, ctypes.POINTER(vie_opts), _vp, _vp, ctypes.POINTER(vie_stats)],
    "vie_solve_device": [_vp, _vp, ctypes.POINTER(vie_opts), _vp, _vp, ctypes.POINTER(vie_stats), _vp],
    "vie_solve_batch": [_vp, ctypes.c_int32, _vp, ctypes.POINTER(vie_opts), _vp, _vp, ctypes.POINTER(vie_stats),
                        _vp],
    "vie_solve_many": [ctypes.c_int32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(vie_opts),
                       ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(vie_stats), _vp],
    "vie_server_start": [_vp, ctypes.c_int32, ctypes.c_int32],
    "vie_footprint": [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
    "vie_submit": [_vp, _vp, _vp, _vp, ctypes.c_int32, _vp, ctypes.POINTER(vie_opts), ctypes.POINTER(_vp)],
    "vie_wait": [_vp, ctypes.c_double, _vp, ctypes.POINTER(vie_stats), _vp],
    "vie_cancel": [_vp],
    "vie_total_field_box": [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp],
    "vie_far_field": [_vp, _vp, ctypes.c_int32, _vp, _vp, _vp],
    "vie_far_field_noalloc": [_vp, _vp, ctypes.c_int32, _vp, _vp, _vp],
    "vie_rcs": [_vp, _vp, ctypes.c_int32, _vp, _vp, _vp],
}.items():
    getattr(_lib, _name).restype = ctypes.c_int
    getattr(_lib, _name).argtypes = _args


def _check(code: int, func: str, warn_ok: bool = False) -> int:
    if code == VIE_OK or (warn_ok and code > 0):
        return code
    raise VieError(code, func, vie_last_error())


# ------------------------------------------------------------------ raw calls
def vie_abi_version() -> int:
    return int(_lib.vie_abi_version())


def vie_last_error() -> str:
    return _lib.vie_last_error().decode()


def vie_context_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    out = _vp()
    _check(_lib.vie_context_create(device, hbm_budget_bytes, ctypes.byref(out)), "vie_context_create")
    return out.value


def vie_context_destroy(ctx: int) -> None:
    _check(_lib.vie_context_destroy(ctx), "vie_context_destroy")


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def vie_problem_create(ctx: int, grid: vie_grid, eps_r: np.ndarray, block_id: Optional[np.ndarray],
                       n_blocks: int) -> int:
    eps = np.ascontiguousarray(eps_r, dtype=np.complex128)
    bid = None if block_id is None else np.ascontiguousarray(block_id, dtype=np.int32)
    out = _vp()
    _check(_lib.vie_problem_create(ctx, ctypes.byref(grid), _np_ptr(eps), _np_ptr(bid), int(n_blocks),
                                   ctypes.byref(out)), "vie_problem_create")
    return out.value


def vie_problem_create_overlap(ctx: int, grid: vie_grid, eps_r: np.ndarray, block_id: np.ndarray, n_blocks: int,
                               overlap: int) -> int:
    eps = np.ascontiguousarray(eps_r, dtype=np.complex128)
    bid = np.ascontiguousarray(block_id, dtype=np.int32)
    out = _vp()
    _check(_lib.vie_problem_create_overlap(ctx, ctypes.byref(grid), _np_ptr(eps), _np_ptr(bid), int(n_blocks),
                                           int(overlap), ctypes.byref(out)), "vie_problem_create_overlap")
    return out.value


def vie_problem_create_rooftop(ctx: int, grid: vie_grid, eps_r: np.ndarray, block_id: Optional[np.ndarray] = None,
                               n_blocks: int = 0) -> int:
    eps = np.ascontiguousarray(eps_r, dtype=np.complex128)
    bid = None if block_id is None else np.ascontiguousarray(block_id, dtype=np.int32)
    out = _vp()
    _check(_lib.vie_problem_create_rooftop(ctx, ctypes.byref(grid), _np_ptr(eps), _np_ptr(bid), int(n_blocks),
                                           ctypes.byref(out)), "vie_problem_create_rooftop")
    return out.value


def vie_problem_destroy(p: int) -> None:
    _check(_lib.vie_problem_destroy(p), "vie_problem_destroy")


def vie_problem_get_info(p: int) -> vie_problem_info:
    info = vie_problem_info()
    _check(_lib.vie_problem_get_info(p, ctypes.byref(info)), "vie_problem_get_info")
    return info


def vie_problem_set_zpass(p: int, precision: int, variant: int) -> None:
    _check(_lib.vie_problem_set_zpass(p, int(precision), int(variant)), "vie_problem_set_zpass")


def vie_problem_set_plane(p: int, precision: int, variant: int) -> None:
    _check(_lib.vie_problem_set_plane(p, int(precision), int(variant)), "vie_problem_set_plane")


def vie_plan(grid: vie_grid, eps: np.ndarray, block_id: Optional[np.ndarray], n_blocks: int, overlap: int = 0,
             groups_cap: int = 64):
    """Host-only block plan: (vie_problem_info, [vie_group_plan, ...], group of every block or None)."""
    e = np.ascontiguousarray(eps, dtype=np.complex128)
    b = None if block_id is None else np.ascontiguousarray(block_id, dtype=np.int32)
    info = vie_problem_info()
    groups = (vie_group_plan * max(groups_cap, 1))()
    bg = np.full(max(int(n_blocks), 1), -1, dtype=np.int32) if b is not None else None
    _check(_lib.vie_plan(ctypes.byref(grid), _np_ptr(e), _np_ptr(b) if b is not None else None, int(n_blocks),
                         int(overlap), ctypes.byref(info), groups, int(groups_cap),
                         _np_ptr(bg) if bg is not None else None), "vie_plan")
    return info, [groups[i] for i in range(min(info.n_groups, groups_cap))], (bg[:n_blocks] if bg is not None else None)


def vie_plane_wave(grid: vie_grid, kdir: Sequence[float], pol: Sequence[complex]) -> np.ndarray:
    k = np.ascontiguousarray(kdir, dtype=np.float64)
    pl = np.ascontiguousarray(np.asarray(pol, dtype=np.complex128))
    out = np.empty((3, grid.nz, grid.ny, grid.nx), dtype=np.complex128)
    _check(_lib.vie_plane_wave(ctypes.byref(grid), _np_ptr(k), _np_ptr(pl), _np_ptr(out)), "vie_plane_wave")
    return out


def vie_plane_wave_faces(grid: vie_grid, kdir: Sequence[float], pol: Sequence[complex]) -> np.ndarray:
    k = np.ascontiguousarray(kdir, dtype=np.float64)
    pl = np.ascontiguousarray(np.asarray(pol, dtype=np.complex128))
    out = np.empty((3, grid.nz, grid.ny, grid.nx), dtype=np.complex128)
    _check(_lib.vie_plane_wave_faces(ctypes.byref(grid), _np_ptr(k), _np_ptr(pl), _np_ptr(out)),
           "vie_plane_wave_faces")
    return out


def _dev(t) -> int:
    if t is None:
        return None
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("device buffers must be contiguous GPU tensors")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def vie_matvec(p: int, precision: int, x, y, stream=None) -> None:
    _check(_lib.vie_matvec(p, precision, _dev(x), _dev(y), _stream(stream)), "vie_matvec")


def vie_matvec_profile(p: int, precision: int, x, y, reps: int, stream=None) -> np.ndarray:
    ms = np.zeros(5, dtype=np.float64)
    _check(_lib.vie_matvec_profile(p, precision, _dev(x), _dev(y), _stream(stream), int(reps), _np_ptr(ms)),
           "vie_matvec_profile")
    return ms


def vie_group_profile(p: int, precision: int, group: int, n_active: int, reps: int, stream=None) -> np.ndarray:
    ms = np.zeros(5, dtype=np.float64)
    _check(_lib.vie_group_profile(p, precision, int(group), int(n_active), int(reps), _stream(stream), _np_ptr(ms)),
           "vie_group_profile")
    return ms


def vie_block_matvec(p: int, precision: int, x, y, stream=None) -> None:
    _check(_lib.vie_block_matvec(p, precision, _dev(x), _dev(y), _stream(stream)), "vie_block_matvec")


def vie_precond_apply(p: int, precision: int, tol_inner: float, maxit_inner: int, w, y, stream=None,
                      flags: int = 0) -> int:
    it = ctypes.c_int64(0)
    _check(_lib.vie_precond_apply(p, precision, tol_inner, maxit_inner, flags, _dev(w), _dev(y), _stream(stream),
                                  ctypes.byref(it)), "vie_precond_apply")
    return int(it.value)


def vie_solve(p: int, e_inc: np.ndarray, opts: vie_opts, stats: vie_stats, want_pol: bool = False):
    e = np.ascontiguousarray(e_inc, dtype=np.complex128)
    e_tot = np.empty_like(e)
    pol = np.empty_like(e) if want_pol else None
    code = _check(_lib.vie_solve(p, _np_ptr(e), ctypes.byref(opts), _np_ptr(e_tot), _np_ptr(pol),
                                 ctypes.byref(stats)), "vie_solve", warn_ok=True)
    return code, e_tot, pol


def vie_solve_device(p: int, e_inc, opts: vie_opts, e_tot, pol, stats: vie_stats, stream=None) -> int:
    return _check(_lib.vie_solve_device(p, _dev(e_inc), ctypes.byref(opts), _dev(e_tot), _dev(pol),
                                        ctypes.byref(stats), _stream(stream)), "vie_solve_device", warn_ok=True)


def vie_solve_batch(p: int, nrhs: int, e_inc, opts: vie_opts, e_tot, pol=None, stats=None, stream=None) -> int:
    """stats: None or a ctypes array of nrhs vie_stats."""
    st = ctypes.cast(stats, ctypes.POINTER(vie_stats)) if stats is not None else None
    return _check(_lib.vie_solve_batch(p, int(nrhs), _dev(e_inc), ctypes.byref(opts), _dev(e_tot), _dev(pol), st,
                                       _stream(stream)), "vie_solve_batch", warn_ok=True)


def vie_solve_many(problems, e_inc, opts: vie_opts, e_tot, pol=None, stats=None, stream=None) -> int:
    """problems: n problem handles; e_inc, e_tot (and pol): n device buffers
    (torch tensors or device addresses); stats: None or a ctypes array of n
    vie_stats."""
    n = len(problems)
    arr = lambda xs: (_vp * n)(*[_dev(x) for x in xs])   # noqa: E731
    hp = (_vp * n)(*problems)
    st = ctypes.cast(stats, ctypes.POINTER(vie_stats)) if stats is not None else None
    return _check(_lib.vie_solve_many(n, hp, arr(e_inc), ctypes.byref(opts), arr(e_tot),
                                      arr(pol) if pol is not None else None, st, _stream(stream)),
                  "vie_solve_many", warn_ok=True)


def _host_problem_arrays(eps, block_id):
    e = np.ascontiguousarray(eps, dtype=np.complex128)
    b = None if block_id is None else np.ascontiguousarray(block_id, dtype=np.int32)
    return e, b


def vie_server_start(ctx: int, slots: int, queue_cap: int) -> None:
    _check(_lib.vie_server_start(ctx, int(slots), int(queue_cap)), "vie_server_start")


def vie_footprint(ctx: int, grid: vie_grid, eps: np.ndarray, block_id: Optional[np.ndarray], n_blocks: int) -> int:
    e, b = _host_problem_arrays(eps, block_id)
    out = ctypes.c_size_t(0)
    _check(_lib.vie_footprint(ctx, ctypes.byref(grid), _np_ptr(e), _np_ptr(b), int(n_blocks), ctypes.byref(out)),
           "vie_footprint")
    return int(out.value)


def vie_submit(ctx: int, grid: vie_grid, eps: np.ndarray, block_id: Optional[np.ndarray], n_blocks: int,
               e_inc: np.ndarray, opts: vie_opts) -> int:
    """Queue a solve; returns the ticket (pass it to vie_wait once)."""
    e, b = _host_problem_arrays(eps, block_id)
    inc = np.ascontiguousarray(e_inc, dtype=np.complex128)
    t = _vp()
    _check(_lib.vie_submit(ctx, ctypes.byref(grid), _np_ptr(e), _np_ptr(b), int(n_blocks), _np_ptr(inc),
                           ctypes.byref(opts), ctypes.byref(t)), "vie_submit")
    return t.value


def vie_wait(ticket: int, shape, timeout_s: float = -1.0):
    """Wait for a request.  Returns (status, e_tot [3, nz, ny, nx] or None,
    stats, times [queued, set-up, solve] in seconds); raises VieError on
    VIE_ETIMEDOUT (the ticket stays valid) and on errors."""
    e_tot = np.empty((3,) + tuple(shape), dtype=np.complex128)
    st = vie_stats()
    times = np.zeros(3, dtype=np.float64)
    code = _check(_lib.vie_wait(ticket, float(timeout_s), _np_ptr(e_tot), ctypes.byref(st), _np_ptr(times)),
                  "vie_wait", warn_ok=True)
    return code, e_tot, st, times


def vie_cancel(ticket: int) -> None:
    _check(_lib.vie_cancel(ticket), "vie_cancel")


def vie_total_field_box(p: int, precision: int, pol, e_inc, e_box, stream=None) -> None:
    _check(_lib.vie_total_field_box(p, precision, _dev(pol), _dev(e_inc), _dev(e_box), _stream(stream)),
           "vie_total_field_box")


def vie_far_field(p: int, pol, rhat: np.ndarray, stream=None) -> np.ndarray:
    r = np.ascontiguousarray(rhat, dtype=np.float64).reshape(-1, 3)
    out = np.empty((r.shape[0], 3), dtype=np.complex128)
    _check(_lib.vie_far_field(p, _dev(pol), int(r.shape[0]), _np_ptr(r), _np_ptr(out), _stream(stream)),
           "vie_far_field")
    return out


def vie_far_field_noalloc(p: int, pol, n_dir: int, rhat_dev, f_dev, stream=None) -> None:
    """Far field into a caller's device buffer (rhat_dev: n_dir x 3 float64,
    f_dev: n_dir x 3 complex128, both device tensors); allocates nothing."""
    _check(_lib.vie_far_field_noalloc(p, _dev(pol), int(n_dir), _dev(rhat_dev), _dev(f_dev), _stream(stream)),
           "vie_far_field_noalloc")


def vie_rcs(p: int, pol, rhat: np.ndarray, stream=None) -> np.ndarray:
    r = np.ascontiguousarray(rhat, dtype=np.float64).reshape(-1, 3)
    out = np.empty(r.shape[0], dtype=np.float64)
    _check(_lib.vie_rcs(p, _dev(pol), int(r.shape[0]), _np_ptr(r), _np_ptr(out), _stream(stream)), "vie_rcs")
    return out


# ------------------------------------------------------------------ conveniences
def make_grid(nx, ny, nz, dx, dy, dz, wavelength) -> vie_grid:
    return vie_grid(int(nx), int(ny), int(nz), float(dx), float(dy), float(dz), float(wavelength))


def make_opts(tol_outer=1e-6, tol_inner=1e-2, maxit_outer=1000, maxit_inner=500, max_refine=3,
              precondition=True, precision=VIE_FP64, poll_lag=1, flags=0, solver=0, restart=30) -> vie_opts:
    return vie_opts(float(tol_outer), float(tol_inner), int(maxit_outer), int(maxit_inner), int(max_refine),
                    1 if precondition else 0, int(precision), int(poll_lag), int(flags), int(solver), int(restart))


def stats_dict(st: vie_stats) -> dict:
    return {f: getattr(st, f) for f, _ in vie_stats._fields_ if f != "inner_hist"}


class Problem:
    """Owns a context (optional) and a problem handle."""

    def __init__(self, grid: vie_grid, eps: np.ndarray, block_id: Optional[np.ndarray] = None, n_blocks: int = 0,
                 ctx: Optional[int] = None, device: int = 0, overlap: int = 0, rooftop: bool = False):
        self._own_ctx = ctx is None
        self.ctx = vie_context_create(device) if ctx is None else ctx
        self.grid = grid
        if rooftop:
            if overlap:
                raise ValueError("rooftop problems take no overlap")
            self.handle = vie_problem_create_rooftop(self.ctx, grid, eps, block_id, n_blocks)
        elif overlap and block_id is not None:
            self.handle = vie_problem_create_overlap(self.ctx, grid, eps, block_id, n_blocks, overlap)
        else:
            self.handle = vie_problem_create(self.ctx, grid, eps, block_id, n_blocks)

    @property
    def shape(self) -> Tuple[int, int, int, int]:
        return (3, self.grid.nz, self.grid.ny, self.grid.nx)

    def info(self) -> vie_problem_info:
        return vie_problem_get_info(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            vie_problem_destroy(self.handle)
            self.handle = None
        if getattr(self, "_own_ctx", False) and getattr(self, "ctx", None):
            vie_context_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
