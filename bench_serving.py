"""Batched-sweep and serving measurements with libvie's request server.

  python bench_serving.py sweep  [--n 64] [--slots 4]
  python bench_serving.py fleet  [--n 64]
  python bench_serving.py stream [--rates 1,2,5,10,20,50] [--n 200] [--max-voxels N] [--slots 4]

sweep: the solves of the batched sweep (workloads.sweep_case, mixed
precision, block preconditioner, outer tol 1e-6, inner 1e-2) all submitted
at once.  fleet: the same solves as one batch per grid shape
(vie_solve_many: every launch covers all problems of a shape, their blocks
solved together), the shapes' batches on concurrent streams, problems set
up from host arrays inside the timed region; against the same problems solved one by one on the GPU (mixed) and
the plain FP64 path.  stream: a Poisson request stream (workloads.arrivals /
serving_request) replayed in real time, one JSON line per rate; by default
every request is served (grids up to 256x256x64); requests larger than
--max-voxels are left out of the measured stream (stated in the output).

Each request goes through vie_submit / vie_wait with host arrays (set-up,
upload and download included).  Reported: solves/s (requests / time from
the first arrival to the last result), latency p50/p99 (arrival to result on
the host), and the same figures for the plain FP64 GPU path run one request
at a time in arrival order (FIFO, each request's FP64 solve timed alone),
plus the largest relative field difference between a served result and
its FP64 solve.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def _grid(V, c):
    return V.make_grid(c.nx, c.ny, c.nz, c.dx, c.dy, c.dz, c.wavelength)


def _opts(V, W, c, precision):
    # at most one correction solve: a request whose main loop stops at its
    # step cap does not spend three more caps on corrections
    pre = W.request_precondition(c)
    return V.make_opts(tol_outer=c.tol_outer, tol_inner=c.tol_inner, maxit_outer=c.maxit_outer,
                       maxit_inner=c.maxit_inner, precondition=pre, precision=precision, max_refine=1)


def served(V, W, ctx, cases, arrive):
    """Replay the arrivals; returns per-request (status, latency s, e_tot,
    times) in submission order."""
    n = len(cases)
    out = [None] * n
    t0 = time.perf_counter()

    def waiter(k, ticket, c):
        try:
            code, e_tot, st, times = V.vie_wait(ticket, c.shape)
            iters = st.outer_iters
        except V.VieError as err:          # the request failed: keep its status
            code, e_tot, times, iters = err.code, np.full((3,) + c.shape, np.nan + 0j), np.zeros(3), -1
        out[k] = (code, time.perf_counter() - t0 - arrive[k], e_tot, times, iters)
        print(f"served {k}: {V.STATUS_NAMES.get(code, code)} {c.nx}x{c.ny}x{c.nz} outer {iters} "
              f"latency {out[k][1]:.2f} s", file=sys.stderr, flush=True)

    threads = []
    for k, c in enumerate(cases):
        delay = arrive[k] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        pre = W.request_precondition(c)
        e = V.vie_plane_wave(_grid(V, c), c.kdir, c.pol)
        t = V.vie_submit(ctx, _grid(V, c), c.eps, c.block_id if pre else None, c.n_blocks if pre else 0, e,
                         _opts(V, W, c, V.VIE_MIXED))
        th = threading.Thread(target=waiter, args=(k, t, c))
        th.start()
        threads.append(th)
    for th in threads:
        th.join()
    return out, time.perf_counter() - t0


def fp64_alone(V, W, ctx, c):
    pre = W.request_precondition(c)
    t = time.perf_counter()
    P = V.Problem(_grid(V, c), c.eps, c.block_id if pre else None, c.n_blocks if pre else 0, ctx=ctx)
    st = V.vie_stats()
    code, e_tot, _ = V.vie_solve(P.handle, V.vie_plane_wave(P.grid, c.kdir, c.pol), _opts(V, W, c, V.VIE_FP64), st)
    P.close()
    return code, time.perf_counter() - t, e_tot


def fifo(arrive, service):
    end, lat = 0.0, []
    for a, s in zip(arrive, service):
        start = max(a, end)
        end = start + s
        lat.append(end - a)
    return lat, end


def stream_cases(W, rate, n, max_voxels=None):
    """The first n requests of the stream at `rate` (optionally without those
    above max_voxels voxels) and their arrival times from the first one."""
    arrive_all = W.arrivals(rate, n)
    cases, arrive, skipped = [], [], []
    for i in range(n):
        c = W.serving_request(rate, i)
        if max_voxels and c.nx * c.ny * c.nz > max_voxels:
            skipped.append(i)
            continue
        cases.append(c)
        arrive.append(arrive_all[i])
    arrive = np.asarray(arrive)
    return cases, arrive - arrive[0], skipped


def measure(V, W, cases, arrive, slots, mode, rate, skipped, max_voxels):
    """Serve `cases` (mixed precision) through a fresh context's server, then
    run the plain FP64 GPU path of each request alone; one result dict."""
    ctx = V.vie_context_create(0)
    V.vie_server_start(ctx, slots, max(1024, len(cases)))
    res, wall = served(V, W, ctx, cases, arrive)
    lat = np.array([r[1] for r in res])
    codes = [r[0] for r in res]
    span = float(max(arrive[k] + lat[k] for k in range(len(cases))) - arrive[0])
    service, diffs = [], []
    for k, c in enumerate(cases):
        code, secs, e64 = fp64_alone(V, W, ctx, c)
        service.append(secs)
        print(f"fp64 alone {k}: {V.STATUS_NAMES.get(code, code)} {secs:.2f} s", file=sys.stderr, flush=True)
        e_mix = res[k][2]
        diffs.append(float(np.linalg.norm(e_mix - e64) / max(np.linalg.norm(e64), 1e-300)))
    blat, bend = fifo(arrive, service)
    V.vie_context_destroy(ctx)
    return {
        "mode": mode, "n": len(cases), "slots": slots, "rate_req_per_s": rate,
        "skipped_requests": skipped, "max_voxels": max_voxels,
        "grids": sorted({f"{c.nx}x{c.ny}x{c.nz}" for c in cases}),
        "tol_outer": sorted({c.tol_outer for c in cases}),
        "served_mixed": {"solves_per_s": len(cases) / span, "latency_ms": {
            "p50": 1e3 * float(np.percentile(lat, 50)), "p99": 1e3 * float(np.percentile(lat, 99))},
            "status_counts": {V.STATUS_NAMES.get(s, s): codes.count(s) for s in set(codes)},
            "mean_queue_s": float(np.mean([r[3][0] for r in res])),
            "mean_setup_s": float(np.mean([r[3][1] for r in res])),
            "mean_solve_s": float(np.mean([r[3][2] for r in res]))},
        "plain_fp64_sequential": {"solves_per_s": len(cases) / bend, "latency_ms": {
            "p50": 1e3 * float(np.percentile(blat, 50)), "p99": 1e3 * float(np.percentile(blat, 99))},
            "mean_service_s": float(np.mean(service))},
        "max_rel_field_diff_mixed_vs_fp64": max(diffs),
        "median_rel_field_diff_mixed_vs_fp64": float(np.median(diffs)),
    }


def fleet(V, W, n):
    """The sweep as one vie_solve_many call per grid shape."""
    import torch
    cases = [W.sweep_case(b) for b in range(n)]
    shapes = {}
    for i, c in enumerate(cases):
        shapes.setdefault((c.nx, c.ny, c.nz), []).append(i)
    ctx = V.vie_context_create(0)
    opts = lambda c, prec: _opts(V, W, c, prec)   # noqa: E731
    # warm-up: kernels and spectra of every shape class (one small batch each)
    for idx in shapes.values():
        sub = [cases[i] for i in idx[:2]]
        Ps = [V.Problem(_grid(V, c), c.eps, c.block_id, c.n_blocks, ctx=ctx) for c in sub]
        es = [torch.from_numpy(V.vie_plane_wave(P.grid, c.kdir, c.pol)).cuda() for P, c in zip(Ps, sub)]
        ys = [torch.empty_like(e) for e in es]
        V.vie_solve_many([P.handle for P in Ps], es, opts(sub[0], V.VIE_MIXED), ys)
        for P in Ps:
            P.close()
    torch.cuda.synchronize()
    out, per_shape = {}, {}

    def run_shape(shape, idx):
        # one thread and one stream per grid shape: the shapes' batches overlap
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            t1 = time.perf_counter()
            sub = [cases[i] for i in idx]
            Ps = [V.Problem(_grid(V, c), c.eps, c.block_id, c.n_blocks, ctx=ctx) for c in sub]
            es = [torch.from_numpy(V.vie_plane_wave(P.grid, c.kdir, c.pol)).cuda() for P, c in zip(Ps, sub)]
            ys = [torch.empty_like(e) for e in es]
            st = (V.vie_stats * len(Ps))()
            code = V.vie_solve_many([P.handle for P in Ps], es, opts(sub[0], V.VIE_MIXED), ys, stats=st,
                                    stream=stream)
            stream.synchronize()
            dt = time.perf_counter() - t1
            for k, i in enumerate(idx):
                out[i] = (ys[k].cpu().numpy(), int(st[k].outer_iters), float(st[k].relres_true))
            per_shape["x".join(map(str, shape))] = {
                "problems": len(idx), "seconds": dt, "status": V.STATUS_NAMES.get(code, code),
                "outer_iters": [int(st[k].outer_iters) for k in range(len(idx))]}
            for P in Ps:
                P.close()
        print(f"fleet {shape}: {len(idx)} problems in {dt:.2f} s", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    threads = [threading.Thread(target=run_shape, args=(shape, idx)) for shape, idx in shapes.items()]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    wall = time.perf_counter() - t0
    # the same problems one by one (mixed, then plain FP64), set-up included
    alone, fp64 = {}, []
    t2 = time.perf_counter()
    for i, c in enumerate(cases):
        P = V.Problem(_grid(V, c), c.eps, c.block_id, c.n_blocks, ctx=ctx)
        e = torch.from_numpy(V.vie_plane_wave(P.grid, c.kdir, c.pol)).cuda()
        y = torch.empty_like(e)
        st = V.vie_stats()
        V.vie_solve_device(P.handle, e, opts(c, V.VIE_MIXED), y, None, st)
        torch.cuda.synchronize()
        alone[i] = y.cpu().numpy()
        P.close()
    t_alone = time.perf_counter() - t2
    diffs = []
    for i, c in enumerate(cases):
        code, secs, e64 = fp64_alone(V, W, ctx, c)
        fp64.append(secs)
        diffs.append(float(np.linalg.norm(out[i][0] - e64) / np.linalg.norm(e64)))
    V.vie_context_destroy(ctx)
    return {"mode": "fleet", "n": n, "shapes": per_shape,
            "batched_mixed": {"solves_per_s": n / wall, "seconds": wall},
            "mixed_one_by_one": {"solves_per_s": n / t_alone, "seconds": t_alone},
            "plain_fp64_one_by_one": {"solves_per_s": n / sum(fp64), "seconds": sum(fp64)},
            "max_rel_field_diff_batched_vs_fp64": max(diffs),
            "median_rel_field_diff_batched_vs_fp64": float(np.median(diffs)),
            "max_rel_field_diff_batched_vs_alone": max(float(np.linalg.norm(out[i][0] - alone[i]) /
                                                              np.linalg.norm(alone[i])) for i in range(n))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["sweep", "fleet", "stream"])
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--rates", default="1,2,5,10,20,50")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--max-voxels", type=int, default=None)
    args = ap.parse_args()

    import workloads as W
    from paper_2501_13512_amd import vie as V

    if args.mode == "fleet":
        print(json.dumps(fleet(V, W, args.n or 64)), flush=True)
        return
    if args.mode == "sweep":
        n = args.n or 64
        cases = [W.sweep_case(b) for b in range(n)]
        print(json.dumps(measure(V, W, cases, np.zeros(n), args.slots, "sweep", None, [], None)), flush=True)
        return
    for rate in [float(r) for r in args.rates.split(",") if r]:
        cases, arrive, skipped = stream_cases(W, rate, args.n or 200, args.max_voxels)
        print(json.dumps(measure(V, W, cases, arrive, args.slots, "stream", rate, skipped, args.max_voxels)),
              flush=True)


if __name__ == "__main__":
    main()
