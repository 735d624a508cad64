#!/usr/bin/env python
"""Benchmark of the repeated-block SpMM hot path on one MI355X.

Workload: the channel-shaped base of 192 x 128 cells (x periodic on
[0, 2 pi], y tanh-clustered with factor 1.5 on [-1, 1], zero-flux walls)
extruded into k = 64 periodic planes (dz = pi / 64): 1,572,864 cells, FP64.

One step is one pass of the hot path:
  1. div SpMM      b = M u        (u: N(0,1) face velocities, seed 2)
  2. Poisson CG    L phi = b      (FP64, zero guess, to relative residual 1e-8)
  3. grad SpMM     u <- u - G phi
  4. lap SpMM      Y_r = L X_r over rotating buffer sets larger than 1 GiB,
                   so every launch reads HBM, not the 256 MB Infinity Cache.

The JSON line reports the lap SpMM's algorithmic bandwidth (value, GB/s) with
its roofline, the Poisson time to 1e-8, the k-sweep against k separate
single-column products (the k x SpMV comparison), the assembled-3D CSR
comparators, and the CPU oracle timed on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-sweep]
       python bench.py --profile      (few steps, for rocprofv3 kernel traces)
       python bench.py --counters     (lap + copy kernels only, for rocprofv3 --pmc)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, AMD specification
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector, AMD specification
COLD_BYTES = 1.1 * 2 ** 30     # rotating working set per sweep (> 4x the 256 MB Infinity Cache)
BASE = (192, 128)
K_MAIN = 64
K_SWEEP = (1, 4, 16, 64)
COUNTER_FILE = os.path.join(ROOT, "profiles", "lap_f64_channel192x128_k64_counters.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("kernels.h", "spmm.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_2508_06710_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def spmm_bytes(nnz_b, n_b, k, v=8):
    """Algorithmic bytes of one Laplacian SpMM: the base block once (values,
    int32 column indices, int32 row pointers), the coupling weights once, X
    read once and Y written once."""
    return (v + 4) * nnz_b + 4 * (n_b + 1) + v * n_b + 2 * v * n_b * k


def spmm_flops(nnz_b, n_b, k):
    return 2 * nnz_b * k + 3 * n_b * k


def csr3d_bytes(nnz3, n3, v=8):
    return (v + 4) * nnz3 + 4 * (n3 + 1) + 2 * v * n3


class Timer:
    """HIP events on torch's current stream, which every library call uses."""

    def __init__(self, torch):
        self.torch = torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.a.record()
        return self

    def __exit__(self, *exc):
        self.b.record()

    def ms(self):
        self.b.synchronize()
        return self.a.elapsed_time(self.b)


def rotating_sets(op, fvx, torch, x_rows):
    per = 2 * op.n_b * op.ld * 8
    R = max(2, math.ceil(COLD_BYTES / per))
    X = [op.empty() for _ in range(R)]
    Y = [op.empty() for _ in range(R)]
    for t in X:
        t.copy_(x_rows)
    return X, Y


def lap_sweep(op, X, Y, torch, reps=1):
    """Mean time per lap SpMM over the rotating pairs (launched from C)."""
    t = Timer(torch)
    with t:
        for _ in range(reps):
            op.lap_many(X, Y)
    return t.ms() / (reps * len(X))


def tune(op, fvx, dtype=None):
    """Autotuned tile for this operator (outside every timed region)."""
    dt = fvx.F64 if dtype is None else dtype
    tile, src = op.tune_cached(dtype=dt, cache_path=os.environ.get("FVX_TUNE_CACHE"),
                               scratch_bytes=512 * 2 ** 20, reps=2)
    log(f"tile k={op.k} {'f64' if dt == fvx.F64 else 'f32'}: {tile} ({src})")
    return tile


def build_case(fvx, inputs, k):
    spec = inputs.channel_base(*BASE)
    mesh = fvx.Mesh.from_spec(spec)
    op = fvx.Operator(mesh, k, math.pi / k, fvx.PERIODIC_Z, with_f32=True)
    return spec, mesh, op


def load_counters(sha):
    if not os.path.exists(COUNTER_FILE):
        return None
    with open(COUNTER_FILE) as fh:
        c = json.load(fh)
    if c.get("source_sha") != sha:
        return None
    return c


def counters_mode(fvx, inputs, torch):
    """A short run for rocprofv3 --pmc: 8 cold lap launches, then 8 copies of
    a known size (the calibration of FETCH_SIZE / WRITE_SIZE)."""
    spec, mesh, op = build_case(fvx, inputs, K_MAIN)
    tune(op, fvx)
    x = op.to_rows(inputs.uniform(0, 0, op.n_b * op.k))
    X, Y = rotating_sets(op, fvx, torch, x)
    for i in range(8):
        op.lap(X[i], Y[i])
    nbytes = 256 * 2 ** 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = [torch.empty_like(src) for _ in range(2)]
    for i in range(8):
        fvx.copy(dst[i % 2], src)
    torch.cuda.synchronize()
    log(f"counters run done: lap bytes/launch {spmm_bytes(op.nnz_b, op.n_b, op.k)}, copy bytes {nbytes}")


def cpu_baseline(inputs, oracle, b_plane, k, rtol):
    """The oracle as it stands, on the host cores: its assembled-3D CSR SpMV
    (timed repeatedly) and its textbook CG to rtol on the same right-hand side."""
    spec = inputs.channel_base(*BASE)
    g = oracle.geometry(spec)
    m3 = oracle.Mesh3D(g, k, math.pi / k, oracle.PERIODIC_Z)
    t0 = time.perf_counter()
    L = m3.lap()
    t_asm = time.perf_counter() - t0
    x = inputs.uniform(0, 0, m3.N)
    y = oracle.spmv(L, x)
    reps, t_spmv = 0, 0.0
    while reps < 20 and t_spmv < 5.0:
        t0 = time.perf_counter()
        oracle.spmv(L, x, out=y)
        t_spmv += time.perf_counter() - t0
        reps += 1
    t_spmv /= reps
    log(f"oracle spmv {t_spmv * 1e3:.2f} ms ({reps} reps), assembly {t_asm:.1f} s")
    t0 = time.perf_counter()
    r = oracle.cg(m3, L, b_plane, rtol, max_iter=20000)
    t_cg = time.perf_counter() - t0
    log(f"oracle CG {r.iters[0]} iters {t_cg:.1f} s")
    nb = g.n_cells
    nnz_b = nb + 2 * g.n_faces
    return {
        "value": spmm_bytes(nnz_b, nb, k) / t_spmv / 1e9,
        "unit": "GB/s",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": (f"oracle assembled-3D CSR SpMV on the {BASE[0]}x{BASE[1]}x{k} channel, "
                   f"{reps} repetitions, GB/s counted with the SpMM's algorithmic bytes; "
                   f"plus one oracle CG to {rtol:g} on the projection right-hand side"),
        "spmv_ms": t_spmv * 1e3,
        "poisson_s_to_1e-8": t_cg,
        "poisson_iters": r.iters[0],
        "cpu_model": _cpu_model(),
        "nproc": os.cpu_count(),
    }


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--profile", action="store_true")
    ap.add_argument("--counters", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(the multi-GPU sharding is a design, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import inputs
    import paper_2508_06710_amd as fvx

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.counters:
        counters_mode(fvx, inputs, torch)
        return
    if args.profile:
        args.steps, args.warmup, args.no_cpu, args.no_sweep = 2, 1, True, True

    rtol = 1e-8
    log("building the channel operator")
    spec, mesh, op = build_case(fvx, inputs, K_MAIN)
    tile = tune(op, fvx)
    tune(op, fvx, fvx.F32)
    n_b, k, N = op.n_b, op.k, op.n_b * op.k
    Bk = spmm_bytes(op.nnz_b, n_b, k)
    Fk = spmm_flops(op.nnz_b, n_b, k)

    # Face velocities u ~ N(0,1), seed 2 (plane-major over in-plane faces, then
    # faces between planes), and the lap sweep inputs U[-1,1], seed 0.
    u = inputs.normal(2, 0, op.F_b * k + n_b * k)
    U0 = op.to_rows(u[:op.F_b * k], rows=op.F_b)
    W0 = op.to_rows(u[op.F_b * k:])
    U, W = torch.empty_like(U0), torch.empty_like(W0)
    X, Y = rotating_sets(op, fvx, torch, op.to_rows(inputs.uniform(0, 0, N)))
    D = op.empty()
    PHI = op.zeros()
    op.workspace(op.solve_opts(rtol=rtol))
    log(f"{N} cells, {len(X)} rotating lap buffer pairs ({len(X) * 2 * n_b * op.ld * 8 / 2**30:.2f} GiB)")

    def step():
        fvx.copy(U, U0)
        fvx.copy(W, W0)
        t_div = Timer(torch)
        with t_div:
            op.div(U, W, D)
        t_sol = Timer(torch)
        with t_sol:
            _, st = op.solve(D, PHI, rtol=rtol)
        t_grad = Timer(torch)
        with t_grad:
            op.grad_axpy(-1.0, PHI, U, W)
        t_lap = lap_sweep(op, X, Y, torch)
        return dict(div_ms=t_div.ms(), solve_ms=t_sol.ms(), grad_ms=t_grad.ms(), lap_ms=t_lap, stats=st)

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for i in range(args.steps):
        recs.append(step())
        log(f"step {i + 1}/{args.steps}: solve {recs[-1]['solve_ms']:.2f} ms, "
            f"{recs[-1]['stats']['iters']} iters, lap {recs[-1]['lap_ms'] * 1e3:.2f} us")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps

    lap_ms = float(np.mean([r["lap_ms"] for r in recs]))
    achieved = Bk / (lap_ms * 1e-3) / 1e9
    st = recs[-1]["stats"]
    solve_s = float(np.median([r["solve_ms"] for r in recs])) / 1e3
    # Divergence after projection, relative to before (checks the step).
    d_after = op.to_planes(op.div(U, W))
    div_ratio = float(np.linalg.norm(d_after) / np.linalg.norm(op.to_planes(D)))

    sha = kernel_source_sha()
    cnt = load_counters(sha)
    traffic = None
    if cnt:
        traffic = cnt["fetch_bytes_per_launch"] + cnt["write_bytes_per_launch"]
    out = {
        "metric": "SpMM GB/s & % HBM roofline vs k×SpMV; Poisson time to rel. residual 1e-8",
        "value": achieved,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"channel {BASE[0]}x{BASE[1]} base x {k} periodic planes ({N} cells), "
                               "lap SpMM + div/grad + FP64 CG to 1e-8",
                   "base": f"{BASE[0]}x{BASE[1]}", "k": k, "cells": N, "nnz_b": op.nnz_b,
                   "rtol": rtol},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_lap<double,V,true,4,S>", "tile": list(tile), "bytes_per_launch": Bk,
                     "launch_us": lap_ms * 1e3, "fp64_tflops": Fk / (lap_ms * 1e-3) / 1e12,
                     "fp64_peak_tflops": FP64_PEAK_TFLOPS, "intensity_flop_per_byte": Fk / Bk,
                     "source_sha": sha},
        "poisson": {"s_to_1e-8": solve_s, "iters": st["iters"], "relres_true": st["relres_true"],
                    "ms_per_iter": solve_s * 1e3 / max(1, st["iters"]),
                    "div_after_over_before": div_ratio},
        "phases_ms": {p: float(np.mean([r[p] for r in recs])) for p in ("div_ms", "solve_ms", "grad_ms", "lap_ms")},
    }

    if not args.no_sweep:
        out.update(extra_measurements(fvx, inputs, torch, np, op, mesh, rtol, D))
        if out.get("copy_ceiling_GBs"):
            out["roofline"]["frac_of_copy"] = achieved / out["copy_ceiling_GBs"]

    if not args.no_cpu:
        log("timing the CPU oracle")
        b_plane = op.to_planes(D)
        out["cpu_baseline"] = cpu_baseline(inputs, __import__("oracle"), b_plane, k, rtol)
    print(json.dumps(out), flush=True)


def extra_measurements(fvx, inputs, torch, np, op, mesh, rtol, D):
    """k sweep (SpMM vs k single-column products and vs the assembled 3D CSR
    SpMV), the copy ceiling, the assembled-CSR CG comparator and the mixed
    precision solve.  Measured outside the timed steps."""
    res = {}
    # copy ceiling: 1 GiB each way, rotating
    nbytes = 2 ** 30
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    fvx.copy(dst, src)
    t = Timer(torch)
    with t:
        for i in range(5):
            fvx.copy(dst if i % 2 == 0 else src, src if i % 2 == 0 else dst)
    res["copy_ceiling_GBs"] = 5 * 2 * nbytes / (t.ms() * 1e-3) / 1e9
    del src, dst
    log(f"copy ceiling {res['copy_ceiling_GBs']:.0f} GB/s")

    import oracle  # closed-form bounds of Section 2 only (Eq. 2, 3a)
    sweep = []
    t1 = None
    for k in K_SWEEP:
        opk = op if k == op.k else fvx.Operator(mesh, k, math.pi / k, fvx.PERIODIC_Z, with_f32=False)
        tile_k = tune(opk, fvx)
        Nk = opk.n_b * k
        x = opk.to_rows(inputs.uniform(0, 0, Nk))
        X, Y = rotating_sets(opk, fvx, torch, x)
        lap_sweep(opk, X[:2], Y[:2], torch)
        tk = lap_sweep(opk, X, Y, torch, reps=2)
        del X, Y
        Bk, Fk = spmm_bytes(opk.nnz_b, opk.n_b, k), spmm_flops(opk.nnz_b, opk.n_b, k)
        ptr, col, val = fvx.expand_csr(mesh, k, math.pi / k, fvx.PERIODIC_Z)
        A = fvx.CsrMatrix(ptr, col, val)
        per = 2 * Nk * 8
        R = max(2, math.ceil(COLD_BYTES / per))
        xs = [torch.as_tensor(inputs.uniform(0, 0, Nk)).cuda() for _ in range(min(R, 4))]
        xs = [xs[i % len(xs)].clone() for i in range(R)]
        ys = [torch.empty_like(xs[0]) for _ in range(R)]
        # The comparator's sweep is captured once in a HIP graph so that its
        # launches are not paced by the Python loop.
        A.spmv(xs[0], ys[0])
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph):
                for xx, yy in zip(xs, ys):
                    A.spmv(xx, yy)
        torch.cuda.current_stream().wait_stream(side)
        graph.replay()
        tm = Timer(torch)
        with tm:
            graph.replay()
            graph.replay()
        t3 = tm.ms() / (2 * R)
        del graph
        del xs, ys, A
        if k == 1:
            t1 = tk
        rec = {"k": k, "tile": list(tile_k), "spmm_us": tk * 1e3, "spmm_GBs": Bk / (tk * 1e-3) / 1e9,
               "frac_hbm": Bk / (tk * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "intensity": Fk / Bk, "fp64_TFLOPs": Fk / (tk * 1e-3) / 1e12,
               "csr3d_us": t3 * 1e3, "csr3d_GBs": csr3d_bytes(len(col), Nk) / (t3 * 1e-3) / 1e9,
               "speedup_vs_csr3d": t3 / tk,
               "P_k": (k * t1 / tk) if t1 else None,
               "P_ub_eq3a": oracle.p_spmm_ub(opk.nnz_b, opk.n_b, opk.n_b, k)}
        sweep.append(rec)
        log(f"k={k}: spmm {rec['spmm_us']:.2f} us ({rec['spmm_GBs']:.0f} GB/s), csr3d {rec['csr3d_us']:.2f} us, "
            f"P_k {rec['P_k']}")
    res["k_sweep"] = sweep

    # Plain FP64 SpMV-CG on the assembled matrix, same right-hand side.
    ptr, col, val = fvx.expand_csr(mesh, op.k, op.dz, fvx.PERIODIC_Z)
    A = fvx.CsrMatrix(ptr, col, val)
    b = torch.empty(op.n_b * op.k, dtype=torch.float64, device="cuda")
    fvx.lib().fvx_unpack(op._h, 0, op.n_b, fvx._ptr(D), fvx._ptr(b), fvx._stream())
    A.solve(b, rtol=rtol)
    tm = Timer(torch)
    with tm:
        _, st3 = A.solve(b, rtol=rtol)
    res["csr3d_cg"] = {"s_to_1e-8": tm.ms() / 1e3, "iters": st3["iters"], "relres_true": st3["relres_true"]}
    del A
    # Mixed precision solve to 1e-8 on the SpMM operator.
    op.solve(D, rtol=rtol, precision=fvx.MIXED)
    tm = Timer(torch)
    with tm:
        _, stm = op.solve(D, rtol=rtol, precision=fvx.MIXED, inner_rtol=1e-4)
    res["mixed_cg"] = {"s_to_1e-8": tm.ms() / 1e3, "inner_iters": stm["iters"], "outer": stm["outer"],
                       "relres_true": stm["relres_true"]}
    log(f"csr3d CG {res['csr3d_cg']['s_to_1e-8']:.3f} s, mixed {res['mixed_cg']['s_to_1e-8']:.3f} s")
    return res


if __name__ == "__main__":
    main()
