"""Benchmark: block-preconditioned VIE-FFT solves on one MI355X.

One step = one complete solve of the metasurface-like workload (8x8
dielectric pillars on a slab, 128x128x32 voxels at lambda/40, 65 blocks,
mixed precision, outer tol 1e-5, inner tol 1e-2) with the incident field
already in HBM: block gather, batched inner BiCGSTAB-FFT solves, scatter,
outer FFT products, BiCGSTAB vector updates and the FP64 refinement check,
all in libvie.  The problem (1/chi, block plan, Green spectra) is set up
once before the timed region; its set-up time is reported separately.

Prints one JSON line.  Extra fields: per-solve latency p50/p99, outer and
inner step counts, the FP64 true residual, the sampled field error against
the oracle's reference file (if present), the FFT product's per-pass times
and the roofline of its dominant pass, and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def pass_bytes(nx, ny, nz, lx, ly, lz, s):
    """Algorithmic bytes of the five passes of one product (s = bytes per
    complex element of the transform: 8 in complex64, 16 in complex128;
    input and output vectors and 1/chi are complex128)."""
    nv = nx * ny * nz
    A = 3 * nz * ny * lx           # x-padded rows
    B = 3 * nz * ly * lx           # x,y-padded planes
    oct_ = 6 * (lx // 2 + 1) * (ly // 2 + 1) * (lz // 2 + 1)
    v = 16
    return [
        3 * nv * v + A * s,                        # x forward (pruned)
        A * s + B * s,                             # y forward (pruned)
        B * s + oct_ * s + B * s,                  # z fwd + spectral multiply + z inv
        B * s + A * s,                             # y inverse (cropped)
        A * s + 3 * nv * v + nv * v + 3 * nv * v,  # x inverse + local term
    ]


PASS_NAMES = ["k_row_fwd", "k_col(fwd)", "k_zconv", "k_col(inv)", "k_row_inv_local"]


def golden_error(case, e_tot):
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{case.name}.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    vox = np.asarray(g["voxels_xyz"])
    want = np.asarray(g["etot_re"]) + 1j * np.asarray(g["etot_im"])
    got = e_tot[:, vox[:, 2], vox[:, 1], vox[:, 0]]
    return {"sampled_rel_err": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
            "oracle_outer_iters": g["outer_iters"], "n_samples": int(vox.shape[0])}


def cpu_baseline(case, outer_iters_hint):
    """Time the CPU oracle on a bounded sample: one outer BiCGSTAB step of the
    same solve (two preconditioner applications plus two products), scaled
    by the oracle's outer step count for the full solve."""
    from oracle import krylov, operator as op, physics
    g = op.Grid.from_case(case)
    e = physics.plane_wave(g, case.kdir, case.pol)
    t0 = time.perf_counter()
    sol = krylov.solve(g, e, case.tol_outer, 1, case.block_id, case.n_blocks, case.tol_inner, case.maxit_inner)
    step_s = time.perf_counter() - t0
    est = step_s * max(outer_iters_hint, 1)
    return {"value": 1.0 / est, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"one outer step of the FP64 oracle solve of the same workload ({step_s:.1f} s, "
                      f"includes set-up), scaled by {outer_iters_hint} outer steps",
            "seconds_per_outer_step": step_s}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--case", default="metasurface")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-reps", type=int, default=20)
    ap.add_argument("--maxit-outer", type=int, default=None,
                    help="cap the outer steps (profiling runs only; the result is then not a full solve)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU runs are not part of this "
              f"build", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2501_13512_amd import vie as V

    case = W.by_name(args.case)
    prec = V.VIE_MIXED if args.precision == "mixed" else V.VIE_FP64
    grid = V.make_grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.wavelength)
    ctx = V.vie_context_create(0)
    t0 = time.perf_counter()
    P = V.Problem(grid, case.eps, case.block_id, case.n_blocks, ctx=ctx)
    setup_s = time.perf_counter() - t0
    info = P.info()
    e_inc = torch.from_numpy(V.vie_plane_wave(grid, case.kdir, case.pol)).cuda()
    e_tot = torch.empty_like(e_inc)
    maxit = case.maxit_outer if args.maxit_outer is None else args.maxit_outer
    opts = V.make_opts(tol_outer=case.tol_outer, tol_inner=case.tol_inner, maxit_outer=maxit,
                       maxit_inner=case.maxit_inner, precondition=True, precision=prec, max_refine=3)
    st = V.vie_stats()
    for _ in range(args.warmup):
        V.vie_solve_device(P.handle, e_inc, opts, e_tot, None, st)
    torch.cuda.synchronize()
    lat = []
    stats = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t1 = time.perf_counter()
        code = V.vie_solve_device(P.handle, e_inc, opts, e_tot, None, st)
        lat.append(time.perf_counter() - t1)
        stats.append(V.stats_dict(st))
        if code != V.VIE_OK and args.maxit_outer is None:
            print(f"solve returned {V.STATUS_NAMES.get(code, code)}", file=sys.stderr)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start

    # FFT product of the full grid, per pass, HIP events on the launch stream
    x = e_tot.clone()
    y = torch.empty_like(x)
    pass_ms = V.vie_matvec_profile(P.handle, prec, x, y, args.profile_reps)
    s_el = 8 if prec == V.VIE_MIXED else 16
    pbytes = pass_bytes(case.nx, case.ny, case.nz, info.lx, info.ly, info.lz, s_el)
    dom = int(np.argmax(pass_ms))
    achieved = pbytes[dom] / (pass_ms[dom] * 1e-3) / 1e9
    mvm_ms = float(np.sum(pass_ms))
    mvm_gbs = sum(pbytes) / (mvm_ms * 1e-3) / 1e9

    res = {
        "metric": "solves/s at 1e-5 rel field err + MVM HBM GB/s vs peak; p50/p99 solve latency",
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 FFT products, f64 vectors/reductions" if prec == V.VIE_MIXED else "f64",
        "data": "synthetic (seeded metasurface-like geometry; no dataset)",
        "config": {"workload": f"{case.name} {case.nx}x{case.ny}x{case.nz}, {info.n_blocks} blocks in "
                               f"{info.n_groups} shape groups, {args.precision}, outer tol {case.tol_outer:g}, "
                               f"inner tol {case.tol_inner:g}",
                   "grid": [case.nx, case.ny, case.nz], "fft": [info.lx, info.ly, info.lz],
                   "precision": args.precision, "parallelism": "1 GPU"},
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)), "p99": 1e3 * float(np.percentile(lat, 99))},
        "setup_ms": 1e3 * setup_s,
        "outer_iters": stats[-1]["outer_iters"],
        "inner_iters_total": stats[-1]["inner_iters_total"],
        "refine_steps": stats[-1]["refine_steps"],
        "relres_true": stats[-1]["relres_true"],
        "mvm": {"ms": mvm_ms, "algorithmic_GBps": mvm_gbs, "pass_ms": [float(v) for v in pass_ms],
                "pass_bytes": pbytes, "pass_names": PASS_NAMES},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": PASS_NAMES[dom] + f" (full-grid product, {args.precision})"},
    }
    ge = golden_error(case, e_tot.cpu().numpy())
    if ge is not None:
        res["field_check"] = ge
    if not args.no_cpu_baseline:
        hint = ge["oracle_outer_iters"] if ge else stats[-1]["outer_iters"]
        res["cpu_baseline"] = cpu_baseline(case, hint)
    P.close()
    V.vie_context_destroy(ctx)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
