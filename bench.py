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


def cart_lines(nx, ny, rows_per_tile, cap):
    """Grid lines per row group of the Cartesian lap kernel under a
    workgroup cap (the library's rule)."""
    if cap <= 0 or -(-(nx * ny) // rows_per_tile) <= cap:
        return 1
    r = 2 if -(-nx // rows_per_tile) * -(-ny // 2) <= cap else 4
    while r > ny:
        r //= 2
    return r


def lap_kernel_name(tile, k, base=BASE):
    """The lap SpMM kernel a tile selects (vec, lanes, block, remap, cap, stage, nt)."""
    vec, lpr, block, _, cap, stage, nt = tile
    span = vec * lpr
    passes = k // span if k % span == 0 else 0
    if span == k and lpr >= 8 and not stage:  # the channel base is a Cartesian 5-point grid
        lines = cart_lines(base[0], base[1], block // lpr, cap)
        width = lpr  # the row-group width is a template constant; no column scale
        if lines > 1:
            return f"k_lap_cart_lines<double,{vec},true,{bool(nt)},True,{lines},{width},False>"
        return f"k_lap_cart<double,{vec},true,{bool(nt)},True,{width},False>"  # 32-bit offsets below 4 GiB
    if passes in (2, 4) and not stage and block <= 512:
        return f"k_lap_passes<double,{vec},true,4,{bool(nt)},{passes}>"
    return f"k_lap<double,{vec},true,4,{bool(stage)},{bool(nt)}>"


def spmm_bytes(nnz_b, n_b, k, v=8):
    """Algorithmic bytes of one Laplacian SpMM: the base block once (values,
    int32 column indices, int32 row pointers), the coupling weights once, X
    read once and Y written once."""
    return (v + 4) * nnz_b + 4 * (n_b + 1) + v * n_b + 2 * v * n_b * k


def spmm_flops(nnz_b, n_b, k):
    return 2 * nnz_b * k + 3 * n_b * k


def stencil_bytes(n_b, k, stencil, v=8):
    """Algorithmic bytes of one structured 13/27-point SpMM: the 8 in-plane
    entries per base row (values and int32 columns), the 27-point's second
    value per entry (planes l+-1), the diagonal, the plane weight w, the
    13-point's w2 (planes l+-2), X read once and Y written once."""
    vals = 8 * (2 if stencil == 27 else 1) + 2 + (1 if stencil == 13 else 0)
    return 32 * n_b + v * vals * n_b + 2 * v * n_b * k


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


def refine_tile(op, fvx, torch, X, Y):
    """The autotuner times its candidates on scratch buffers of its own; for
    the headline operator its pick is refined under the headline's cold
    sweep: the tuner's tile and its neighbours (XCD remap on and off,
    workgroups of 64 to 512 threads, no cap or a cap of 1024 or 2048
    workgroups, the same row mapping) are timed with
    lap_sweep on the rotating buffers and the fastest is kept and written to
    the tile cache, so the profiling and counter runs use the same tile
    (outside every timed region)."""
    path = os.environ.get("FVX_TUNE_CACHE")
    if path and os.path.exists(path):
        with open(path) as fh:
            entry = json.load(fh).get(op._tile_key(fvx.F64), {})
        if entry.get("source") == "refined":  # refined by an earlier run: keep it (profiling runs)
            op.set_tile(*entry["tile"])
            return tuple(entry["tile"])
    base = tuple(op.get_tile())
    vec, lpr, _, _, _, stage, nt = base
    cands = {base} | {(vec, lpr, b, rm, cap, stage, nt) for b in (64, 128, 256, 512) for rm in (0, 1)
                      for cap in (0, 1024, 2048) if b >= lpr}
    best, bt = base, None
    for t in sorted(cands):
        op.set_tile(*t)
        lap_sweep(op, X[:2], Y[:2], torch)
        tt = min(lap_sweep(op, X, Y, torch) for _ in range(2))
        if bt is None or tt < bt:
            best, bt = t, tt
    op.set_tile(*best)
    op.remember_tile(best, os.environ.get("FVX_TUNE_CACHE"))
    log(f"tile k={op.k} f64 refined on the cold sweep: {best} ({bt * 1e3:.2f} us; tuner's {base})")
    return best


def tune_cg(op, fvx, dtype=None):
    """Autotuned CG tile for this operator (outside every timed region)."""
    dt = fvx.F64 if dtype is None else dtype
    tile, src = op.tune_cg_cached(dtype=dt, cache_path=os.environ.get("FVX_TUNE_CACHE"))
    log(f"cg tile k={op.k} {'f64' if dt == fvx.F64 else 'f32'}: {tile} ({src})")
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
    """A short run for rocprofv3 --pmc: 8 cold lap launches of the headline
    tile, then 8 of each other kernel instance its row mapping can select
    (the Cartesian kernel with 1, 2 or 4 grid lines per row group, chosen by
    the workgroup cap), then 8 copies of a known size (the calibration of
    FETCH_SIZE / WRITE_SIZE)."""
    spec, mesh, op = build_case(fvx, inputs, K_MAIN)
    tile = tune(op, fvx)
    x = op.to_rows(inputs.uniform(0, 0, op.n_b * op.k))
    X, Y = rotating_sets(op, fvx, torch, x)
    seen = {lap_kernel_name(tile, op.k)}
    tiles = [tile]
    for cap in (0, 2048, 1024):
        alt = tuple(tile[:4]) + (cap,) + tuple(tile[5:])
        if lap_kernel_name(alt, op.k) not in seen:
            seen.add(lap_kernel_name(alt, op.k))
            tiles.append(alt)
    for n, t in enumerate(tiles):
        op.set_tile(*t)
        for i in range(8):
            op.lap(X[8 * n + i], Y[8 * n + i])
        log(f"counters: 8 launches of {lap_kernel_name(t, op.k)} (tile {t})")
    op.set_tile(*tile)
    nbytes = 256 * 2 ** 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = [torch.empty_like(src) for _ in range(2)]
    for i in range(8):
        fvx.copy(dst[i % 2], src)
    torch.cuda.synchronize()
    log(f"counters run done: lap bytes/launch {spmm_bytes(op.nnz_b, op.n_b, op.k)}, copy bytes {nbytes}")


def mixed_profile_mode(fvx, inputs, torch):
    """A short run for rocprofv3 kernel traces of the mixed-precision solve on
    the channel workload: one warm-up and one timed solve to 1e-8 of the
    projection right-hand side."""
    spec, mesh, op = build_case(fvx, inputs, K_MAIN)
    tune(op, fvx)
    tune(op, fvx, fvx.F32)
    tune_cg(op, fvx)
    tune_cg(op, fvx, fvx.F32)
    u = inputs.normal(2, 0, op.F_b * op.k + op.n_b * op.k)
    D = op.div(op.to_rows(u[:op.F_b * op.k], rows=op.F_b), op.to_rows(u[op.F_b * op.k:]))
    for _ in range(2):
        _, st = op.solve(D, rtol=1e-8, precision=fvx.MIXED)
    torch.cuda.synchronize()
    log(f"mixed profile run done: {st['iters']} inner iterations, {st['outer']} corrections, {st['seconds']:.4f} s")


def net_profile_mode(fvx, inputs, torch):
    """A short run for rocprofv3 kernel traces of the learned-guess kernels on
    the 64 x 64 x 8 channel: 10 inferences (one sample) and 5 training steps
    (16 samples)."""
    cfg = inputs.SMALL_CHANNEL
    spec, k, dz = cfg["base"], cfg["k"], cfg["dz"]
    mesh = fvx.Mesh.from_spec(spec)
    op = fvx.Operator(mesh, k, dz, fvx.PERIODIC_Z, with_f32=False)
    net = fvx.GuessNet(spec.nx, spec.ny, k, batch=16, params=inputs.net_init(6, zero_output_layer=False))
    b = op.to_rows(inputs.rhs_uniform(1, op.n_b * k))
    X0 = op.zeros()
    for _ in range(10):
        net.guess(op, b, b, X0)
    x = torch.as_tensor(inputs.uniform(2, 0, 16 * 2 * op.n_b * k).astype("float32")).cuda()
    t = torch.as_tensor(inputs.uniform(2, 1, 16 * op.n_b * k).astype("float32")).cuda()
    x = x.view(16, 2, k, spec.ny, spec.nx)
    t = t.view(16, 1, k, spec.ny, spec.nx)
    for _ in range(5):
        net.train_step(x, t, 1e-4)
    torch.cuda.synchronize()
    log("net profile run done")


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
    ap.add_argument("--profile-net", action="store_true")
    ap.add_argument("--profile-mixed", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-airfoil", action="store_true")
    ap.add_argument("--no-guess", action="store_true")
    ap.add_argument("--no-stencil", action="store_true")
    ap.add_argument("--profile-stencil", action="store_true")
    ap.add_argument("--profile-pcg", action="store_true")
    ap.add_argument("--profile-amg", action="store_true")
    ap.add_argument("--profile-ns", action="store_true")
    ap.add_argument("--no-ns", action="store_true")
    ap.add_argument("--guess-epochs", type=int, default=20)
    ap.add_argument("--guess-lr", type=float, default=1e-4)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path runs on a single device)", file=sys.stderr)
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
    if args.profile_net:
        net_profile_mode(fvx, inputs, torch)
        return
    if args.profile_mixed:
        mixed_profile_mode(fvx, inputs, torch)
        return
    if args.profile_stencil:
        stencil_profile_mode(fvx, inputs, torch)
        return
    if args.profile_pcg:
        pcg_profile_mode(fvx, inputs, torch)
        return
    if args.profile_amg:
        amg_profile_mode(fvx, inputs, torch)
        return
    if args.profile_ns:
        ns_profile_mode(fvx, inputs, torch)
        return
    if args.profile:
        args.steps, args.warmup, args.no_cpu, args.no_sweep = 2, 1, True, True
        args.no_batch = args.no_airfoil = args.no_guess = args.no_stencil = args.no_ns = True

    rtol = 1e-8
    log("building the channel operator")
    spec, mesh, op = build_case(fvx, inputs, K_MAIN)
    tile = tune(op, fvx)
    tune(op, fvx, fvx.F32)
    cg_tiles = {"f64": list(tune_cg(op, fvx)), "f32": list(tune_cg(op, fvx, fvx.F32))}
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
    tile = refine_tile(op, fvx, torch, X, Y)
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
    norm = lambda n: n.replace(" ", "").lower()
    if cnt:  # counters of this very kernel instance
        entries = [cnt] + list(cnt.get("by_kernel", {}).values())
        hit = [e for e in entries if norm(e.get("kernel", "")) == norm(lap_kernel_name(tile, k))]
        if hit:
            traffic = hit[0]["fetch_bytes_per_launch"] + hit[0]["write_bytes_per_launch"]
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
                     "kernel": lap_kernel_name(tile, k), "tile": list(tile), "bytes_per_launch": Bk,
                     "launch_us": lap_ms * 1e3, "fp64_tflops": Fk / (lap_ms * 1e-3) / 1e12,
                     "fp64_peak_tflops": FP64_PEAK_TFLOPS, "intensity_flop_per_byte": Fk / Bk,
                     "source_sha": sha},
        "poisson": {"s_to_1e-8": solve_s, "iters": st["iters"], "relres_true": st["relres_true"], "cg_tiles": cg_tiles,
                    "ms_per_iter": solve_s * 1e3 / max(1, st["iters"]),
                    "div_after_over_before": div_ratio},
        "phases_ms": {p: float(np.mean([r[p] for r in recs])) for p in ("div_ms", "solve_ms", "grad_ms", "lap_ms")},
    }

    if not args.no_sweep:
        out.update(extra_measurements(fvx, inputs, torch, np, op, mesh, rtol, D))
        if out.get("copy_ceiling_GBs"):
            out["roofline"]["frac_of_copy"] = achieved / out["copy_ceiling_GBs"]

    if not args.no_stencil:
        out["stencils"] = stencil_leg(fvx, inputs, torch, np)
        torch.cuda.empty_cache()
        out["refine_mapping"] = refine_leg(fvx, inputs, torch, np)
        torch.cuda.empty_cache()
        out["generic_spmm"] = generic_leg(fvx, inputs, torch, np)
        torch.cuda.empty_cache()
    if not args.no_ns:
        out["ns_step"] = ns_leg(fvx, inputs, torch, np)
        torch.cuda.empty_cache()
    if not args.no_batch:
        out["batched"] = batch_leg(fvx, inputs, torch, np, rtol)
        torch.cuda.empty_cache()
    if not args.no_airfoil:
        out["airfoil"] = airfoil_leg(fvx, inputs, torch, np)
        torch.cuda.empty_cache()
    if not args.no_guess:
        out["learned_guess"] = guess_leg(fvx, inputs, torch, np, args.guess_epochs, args.guess_lr, rtol)
        torch.cuda.empty_cache()

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
        t3 = time_csr_spmv(fvx, torch, inputs, ptr, col, val, Nk)
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
    res["large_sweep"] = large_sweep(fvx, inputs, torch, np)

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
    res["poisson_pcg"] = pcg_leg(fvx, torch, op, D, rtol)
    res["poisson_amg"] = amg_leg(fvx, torch, inputs, op, D, rtol)
    log(f"csr3d CG {res['csr3d_cg']['s_to_1e-8']:.3f} s, mixed {res['mixed_cg']['s_to_1e-8']:.3f} s")
    return res


def graph_time(torch, calls):
    """Mean time per call of a list of launches captured once in a HIP graph
    (so that the launches are not paced by the Python loop); the graph is
    replayed once untimed and twice timed."""
    calls[0]()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph):
            for f in calls:
                f()
    torch.cuda.current_stream().wait_stream(side)
    graph.replay()
    tm = Timer(torch)
    with tm:
        graph.replay()
        graph.replay()
    t = tm.ms() / (2 * len(calls))
    del graph
    return t


def time_csr_spmv(fvx, torch, inputs, ptr, col, val, n3):
    """Mean time of the assembled 3D CSR SpMV over rotating vectors, its
    sweep captured once in a HIP graph so that the launches are not paced by
    the Python loop."""
    A = fvx.CsrMatrix(ptr, col, val)
    per = 2 * n3 * 8
    R = max(2, math.ceil(COLD_BYTES / per))
    xs = [torch.as_tensor(inputs.uniform(0, 0, n3)).cuda() for _ in range(min(R, 4))]
    xs = [xs[i % len(xs)].clone() for i in range(R)]
    ys = [torch.empty_like(xs[0]) for _ in range(R)]
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
    t = tm.ms() / (2 * R)
    del graph, xs, ys, A
    return t


def stencil_leg(fvx, inputs, torch, np):
    """The 7-, 13- and 27-point operators (first neighbours; first and second
    neighbours; all 26 neighbours) on the channel base: SpMM bandwidth against
    the HBM roofline with tuned tiles, the speed-up over k single-column
    products (P_k = k t_1 / t_k, the quantity of Fig. 8) beside its
    bandwidth bound k B_1 / B_k, and the assembled 3D CSR SpMV of the same
    matrix.  The CSR bytes ratio is the speed-up the repeated-block format
    allows over the assembled matrix when both run at the same bandwidth."""
    spec = inputs.channel_base(*BASE)
    mesh = fvx.Mesh.from_spec(spec)
    out = []
    t1 = {}
    for stencil in (7, 13, 27):
        for k in (1, 16, 64):
            dz = math.pi / k
            op = fvx.Operator(mesh, k, dz, fvx.PERIODIC_Z, with_f32=True, stencil=stencil)
            n3 = op.n_b * k
            t3 = nnz3 = None
            if k > 1:
                ptr, col, val = fvx.expand_csr(mesh, k, dz, fvx.PERIODIC_Z, stencil=stencil)
                nnz3 = len(col)
                t3 = time_csr_spmv(fvx, torch, inputs, ptr, col, val, n3)
                del ptr, col, val
            for dt, name, v in ((fvx.F64, "f64", 8), (fvx.F32, "f32", 4)):
                tile = tune(op, fvx, dt)
                x = op.to_rows(inputs.uniform(0, 0, n3), dtype=dt)
                R = max(3, math.ceil(COLD_BYTES / (2 * op.n_b * op.ld * v)))
                X = [x.clone() for _ in range(R)]
                Y = [torch.empty_like(x) for _ in range(R)]
                lap_sweep(op, X[:2], Y[:2], torch)
                t = lap_sweep(op, X, Y, torch, reps=2)
                del X, Y, x
                Bk = spmm_bytes(op.nnz_b, op.n_b, k, v) if stencil == 7 else stencil_bytes(op.n_b, k, stencil, v)
                if k == 1:
                    t1[(stencil, name)] = (t, Bk)
                rec = {"stencil": stencil, "k": k, "dtype": name, "tile": list(tile), "bytes_per_launch": Bk,
                       "spmm_us": t * 1e3, "spmm_GBs": Bk / (t * 1e-3) / 1e9,
                       "frac_hbm": Bk / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}
                if k > 1:
                    ta, Ba = t1[(stencil, name)]
                    rec.update({"P_k": k * ta / t, "P_bound_bytes": k * Ba / Bk})
                if k > 1 and dt == fvx.F64:
                    rec.update({"nnz_per_row_3d": nnz3 / n3, "csr3d_us": t3 * 1e3, "speedup_vs_csr3d": t3 / t,
                                "bytes_ratio_csr3d": csr3d_bytes(nnz3, n3) / Bk})
                out.append(rec)
                log(f"stencil {stencil} k={k} {name}: {rec['spmm_GBs']:.0f} GB/s "
                    f"({100 * rec['frac_hbm']:.0f}% of 8 TB/s)"
                    + (f", P_k {rec['P_k']:.1f} (bound {rec['P_bound_bytes']:.1f})" if k > 1 else "")
                    + (f", {rec['speedup_vs_csr3d']:.2f}x the 3D CSR SpMV" if "csr3d_us" in rec else ""))
            del op
            torch.cuda.empty_cache()
    return out


def stencil_profile_mode(fvx, inputs, torch):
    """A short run for rocprofv3 of the 13- and 27-point SpMMs on the channel
    base with 64 planes: 8 cold FP64 launches of each (tuned tiles), then 8
    copies of a known size (the calibration of FETCH_SIZE / WRITE_SIZE)."""
    spec = inputs.channel_base(*BASE)
    mesh = fvx.Mesh.from_spec(spec)
    for stencil in (13, 27):
        op = fvx.Operator(mesh, K_MAIN, math.pi / K_MAIN, fvx.PERIODIC_Z, with_f32=False, stencil=stencil)
        tune(op, fvx)
        x = op.to_rows(inputs.uniform(0, 0, op.n_b * op.k))
        X, Y = rotating_sets(op, fvx, torch, x)
        for i in range(8):
            op.lap(X[i], Y[i])
        torch.cuda.synchronize()
        log(f"stencil {stencil}: bytes/launch {stencil_bytes(op.n_b, op.k, stencil)}")
        del X, Y, op
        torch.cuda.empty_cache()
    nbytes = 256 * 2 ** 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = [torch.empty_like(src) for _ in range(2)]
    for i in range(8):
        fvx.copy(dst[i % 2], src)
    torch.cuda.synchronize()
    log("stencil profile run done")


def refine_leg(fvx, inputs, torch, np):
    """The inline-refinement coarse-to-fine mapping as a rectangular SpMM
    (fvx_sparse_spmm): the 96 x 64 channel base refined twice in x and y
    (24,576 fine rows, 6,144 coarse columns, bilinear weights) applied to
    k flow states at once, k = 1, 16, 64, FP64 and FP32, tiles tuned per k
    and precision; bandwidth against
    the HBM roofline and P_k = k t_1 / t_k beside Eq. 3a's bound for these
    n_r, n_c and nnz.  The sweep over rotating buffers is captured in a HIP
    graph, so the launches are not paced by the Python loop."""
    import oracle  # closed-form bound of Eq. 3a only
    spec = inputs.channel_base(96, 64)
    m = fvx.Mesh.from_spec(spec)
    ptr, col, val = m.prolongation(2)
    P = fvx.SparseMatrix(ptr, col, val, m.n_cells)
    n_r, n_c, nnz = P.n_rows, P.n_cols, P.nnz
    out, t1 = [], {}
    for k in (1, 16, 64):
        for name, tdt, v in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
            ld = max(k, 4) if k > 1 else 1
            R = max(3, math.ceil(COLD_BYTES / ((n_r + n_c) * ld * v)))
            X = [torch.as_tensor(inputs.uniform(0, 0, n_c * ld).reshape(n_c, ld)).to(tdt).cuda() for _ in range(R)]
            Y = [torch.empty((n_r, ld), dtype=tdt, device="cuda") for _ in range(R)]
            P.tune(X[0], Y[0], k=k, reps=3)
            t = graph_time(torch, [lambda xx=xx, yy=yy: P.spmm(xx, yy, k=k) for xx, yy in zip(X, Y)])
            del X, Y
            B = (v + 4) * nnz + 4 * (n_r + 1) + v * (n_c + n_r) * k
            if k == 1:
                t1[name] = t
            rec = {"k": k, "dtype": name, "n_rows": n_r, "n_cols": n_c, "nnz": nnz, "bytes_per_launch": B,
                   "spmm_us": t * 1e3, "spmm_GBs": B / (t * 1e-3) / 1e9, "frac_hbm": B / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}
            if k > 1:
                rec.update({"P_k": k * t1[name] / t, "P_ub_eq3a": oracle.p_spmm_ub(nnz, n_r, n_c, k)})
            out.append(rec)
            log(f"refine mapping k={k} {name}: {rec['spmm_us']:.2f} us, {rec['spmm_GBs']:.0f} GB/s"
                + (f", P_k {rec['P_k']:.1f} (Eq. 3a bound {rec['P_ub_eq3a']:.1f})" if k > 1 else ""))
    return out


def ns_leg(fvx, inputs, torch, np, rtol=1e-8):
    """The whole incompressible time step (Heun RK3, a projection per stage,
    Poisson solves warm-started from the previous pressure, preconditioned by
    the Chebyshev polynomial or by the multigrid) on the channel base: the coupled 192 x 128 x 64 channel, and
    independent flow states (the base plane repeated k = 1, 16, 64 times
    without coupling) for the whole-iteration speed-up P_k,ite = k t_1 / t_k
    (the paper's P_m,ite).  Random initial velocities, projected by the
    warm-up steps; the mean of 3 timed steps."""
    spec = inputs.channel_base(*BASE)
    mesh = fvx.Mesh.from_spec(spec)
    out = {}
    cheb = dict(rtol=rtol, precond=fvx.PRECOND_CHEBYSHEV, guess=fvx.GUESS_GIVEN)

    def run(op, label, kw):
        U = [op.to_rows(inputs.uniform(0, d, op.n_b * op.k)) for d in range(3)]
        Uf = op.zeros(op.F_b)
        Wz = op.zeros() if op.zfaces else None
        P = op.zeros()
        dt, nu = 1e-3, 1.0 / 180.0
        for _ in range(2):
            op.ns_step(U, Uf, Wz, P, dt, nu, **kw)
        tm = Timer(torch)
        its = 0
        with tm:
            for _ in range(3):
                st = op.ns_step(U, Uf, Wz, P, dt, nu, **kw)
                its += st["iters"]
        t = tm.ms() / 3
        log(f"ns step {label}: {t:.2f} ms per step, {its / 3:.0f} CG iterations per step")
        return {"ms_per_step": t, "cg_iters_per_step": its / 3, "cells": op.n_b * op.k}

    op = fvx.Operator(mesh, K_MAIN, math.pi / K_MAIN, fvx.PERIODIC_Z, with_f32=False)
    tune(op, fvx)
    tune_cg(op, fvx)
    out["channel_coupled_k64"] = run(op, "coupled channel k=64", cheb)
    amg = fvx.Amg(op)
    out["channel_coupled_k64_amg"] = run(op, "coupled channel k=64, multigrid", dict(cheb, precond=0, amg=amg))
    del op, amg
    states, states_amg = {}, {}
    for k in (1, 16, 64):
        opk = fvx.Operator(mesh, k, math.pi / K_MAIN, fvx.NONE, with_f32=False)
        tune(opk, fvx)
        tune_cg(opk, fvx)
        states[k] = run(opk, f"independent states k={k}", cheb)
        amg = fvx.Amg(opk)
        states_amg[k] = run(opk, f"independent states k={k}, multigrid", dict(cheb, precond=0, amg=amg))
        del opk, amg
        torch.cuda.empty_cache()
    for st in (states, states_amg):
        for k in (16, 64):
            st[k]["P_k_ite"] = k * st[1]["ms_per_step"] / st[k]["ms_per_step"]
    out["independent_states"] = {str(k): v for k, v in states.items()}
    out["independent_states_amg"] = {str(k): v for k, v in states_amg.items()}
    return out


def ns_profile_mode(fvx, inputs, torch):
    """A short run for rocprofv3 kernel traces of the time step on the coupled
    channel (192 x 128 x 64): two steps."""
    spec = inputs.channel_base(*BASE)
    op = fvx.Operator(fvx.Mesh.from_spec(spec), K_MAIN, math.pi / K_MAIN, fvx.PERIODIC_Z, with_f32=False)
    tune(op, fvx)
    tune_cg(op, fvx)
    U = [op.to_rows(inputs.uniform(0, d, op.n_b * op.k)) for d in range(3)]
    Uf, Wz, P = op.zeros(op.F_b), op.zeros(), op.zeros()
    for _ in range(2):
        st = op.ns_step(U, Uf, Wz, P, 1e-3, 1.0 / 180.0, rtol=1e-8, precond=fvx.PRECOND_CHEBYSHEV,
                        guess=fvx.GUESS_GIVEN)
    torch.cuda.synchronize()
    log(f"ns profile run done: {st['iters']} CG iterations in the last step")


def generic_leg(fvx, inputs, torch, np):
    """Section 2's setting: a square sparse matrix with n = 10^6 rows and 7 or
    13 nonzeros per row (periodic 100^3 structured matrices) times m
    right-hand sides with the general CSR SpMM (fvx_sparse_spmm, tuned per
    m): P_m = m t_1 / t_m against its own single-column product, beside the
    upper and lower bounds of Eqs. 3a and 3b for the same nnz, n_r, n_c, and
    against m products with the CSR-vector SpMV (fvx_csr_spmv).  Sweeps
    captured in HIP graphs."""
    import oracle  # closed-form bounds of Section 2 only (Eqs. 3a, 3b)
    out = []
    for points in (7, 13):
        ptr, col, val = inputs.structured_csr(100, points)
        n, nnz = len(ptr) - 1, len(col)
        M = fvx.SparseMatrix(ptr, col, val, n, with_f32=False)
        A = fvx.CsrMatrix(ptr, col, val)
        x = torch.as_tensor(inputs.uniform(0, 0, n)).cuda()
        R1 = max(2, math.ceil(COLD_BYTES / (16 * n)))
        xs = [x.clone() for _ in range(R1)]
        ys = [torch.empty_like(x) for _ in range(R1)]
        t_spmv = graph_time(torch, [lambda a=a, b=b: A.spmv(a, b) for a, b in zip(xs, ys)])
        del xs, ys
        for m in (1, 2, 4, 8, 16, 32, 64, 128):
            ld = m if m < 4 else m + (-m) % 4
            R = max(2, math.ceil(COLD_BYTES / (16 * n * ld)))
            x0 = torch.as_tensor(inputs.uniform(1, m, n * ld).reshape(n, ld)).cuda()
            X = [x0] + [x0.clone() for _ in range(R - 1)]
            Y = [torch.empty((n, ld), dtype=torch.float64, device="cuda") for _ in range(R)]
            M.tune(X[0], Y[0], k=m, reps=3)
            t = graph_time(torch, [lambda a=a, b=b: M.spmm(a, b, k=m) for a, b in zip(X, Y)])
            del X, Y
            B = 12 * nnz + 4 * (n + 1) + 16 * n * m
            if m == 1:
                t_own = t
            rec = {"nnz_per_row": points, "m": m, "spmm_us": t * 1e3, "spmm_GBs": B / (t * 1e-3) / 1e9,
                   "frac_hbm": B / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, "spmv_us": t_spmv * 1e3,
                   "P_m_vs_csr_spmv": m * t_spmv / t, "P_m": m * t_own / t,
                   "P_ub_eq3a": oracle.p_spmm_ub(nnz, n, n, m), "P_lb_eq3b": oracle.p_spmm_lb(nnz, n, m)}
            out.append(rec)
            log(f"generic SpMM {points} nnz/row m={m}: {rec['spmm_us']:.1f} us ({rec['spmm_GBs']:.0f} GB/s), "
                f"P_m {rec['P_m']:.2f} (bounds {rec['P_lb_eq3b']:.2f}..{rec['P_ub_eq3a']:.2f}; "
                f"vs the CSR-vector SpMV {rec['P_m_vs_csr_spmv']:.2f})")
            torch.cuda.empty_cache()
        del M, A
    return out


def pcg_leg(fvx, torch, op, D, rtol):
    """Preconditioned CG on the benchmark's projection right-hand side: Jacobi
    and the Chebyshev polynomial (degree 8 on [2/300, 2], the library's
    defaults), FP64 and mixed precision; the best of 3 timed solves each."""
    out = {}
    cases = {"jacobi": dict(precond=fvx.PRECOND_JACOBI),
             "chebyshev": dict(precond=fvx.PRECOND_CHEBYSHEV),
             "mixed_chebyshev": dict(precond=fvx.PRECOND_CHEBYSHEV, precision=fvx.MIXED)}
    for name, kw in cases.items():
        op.solve(D, rtol=rtol, **kw)
        best, st = None, None
        for _ in range(3):
            tm = Timer(torch)
            with tm:
                _, st = op.solve(D, rtol=rtol, **kw)
            best = tm.ms() if best is None else min(best, tm.ms())
        o = op.solve_opts(**kw)
        out[name] = {"s_to_1e-8": best / 1e3, "iters": st["iters"], "outer": st["outer"],
                     "relres_true": st["relres_true"], "cheb_degree": int(o.cheb_degree),
                     "cheb_ratio": float(o.cheb_ratio)}
        log(f"pcg {name}: {best:.2f} ms, {st['iters']} iterations, true residual {st['relres_true']:.2e}")
    return out


def amg_leg(fvx, torch, inputs, op, D, rtol):
    """CG preconditioned by one V-cycle of the aggregation multigrid (default
    options: Chebyshev degree 2 on [2/8, 2], pairwise aggregation with beta
    0.25, plane merging when the plane coupling dominates, coarsest level at
    most 2048 unknowns) on the benchmark's projection right-hand side, FP64 and
    mixed precision, the best of 3 timed solves each; the time of one V-cycle
    and, per level, the level's SpMM (its operator on the level's k planes;
    graph-timed, inputs warm in the caches) -- the per-level SpMM table of the
    paper's multigrid appendix."""
    t0 = time.perf_counter()
    amg = fvx.Amg(op)
    out = {"setup_s": time.perf_counter() - t0, "levels": []}
    for name, kw in (("f64", {}), ("mixed", dict(precision=fvx.MIXED))):
        op.solve(D, rtol=rtol, amg=amg, **kw)
        best, st = None, None
        for _ in range(3):
            tm = Timer(torch)
            with tm:
                _, st = op.solve(D, rtol=rtol, amg=amg, **kw)
            best = tm.ms() if best is None else min(best, tm.ms())
        out[name] = {"s_to_1e-8": best / 1e3, "iters": st["iters"], "outer": st["outer"],
                     "relres_true": st["relres_true"]}
        log(f"amg {name}: {best:.2f} ms, {st['iters']} iterations, true residual {st['relres_true']:.2e}")
    Z = torch.empty_like(D)
    out["vcycle_us"] = graph_time(torch, [lambda: amg.apply(D, Z)] * 10) * 1e3
    for lvl, (n_b, k, nnz_b, kind) in enumerate(amg.levels()):
        lop = amg.level_op(lvl)
        X = lop.to_rows(inputs.uniform(0, 0, n_b * k))
        Y = torch.empty_like(X)
        t = graph_time(torch, [lambda: lop.lap(X, Y)] * 20)
        B = spmm_bytes(lop.nnz_b, n_b, k)
        out["levels"].append({"n_b": n_b, "k": k, "nnz_b": nnz_b, "next": ["coarsest", "base", "planes"][kind],
                              "spmm_us": t * 1e3, "spmm_GBs": B / (t * 1e-3) / 1e9})
        log(f"amg level {lvl}: n_b {n_b} k {k} nnz_b {nnz_b} -> {out['levels'][-1]['next']}, "
            f"SpMM {t * 1e3:.2f} us")
    log(f"amg V-cycle {out['vcycle_us']:.1f} us")
    return out


def amg_profile_mode(fvx, inputs, torch):
    """A short run for rocprofv3 kernel traces of the multigrid-preconditioned
    CG on the channel workload: one warm-up and one timed FP64 solve to 1e-8."""
    spec, mesh, op = build_case(fvx, inputs, K_MAIN)
    tune(op, fvx)
    tune_cg(op, fvx)
    amg = fvx.Amg(op)
    u = inputs.normal(2, 0, op.F_b * op.k + op.n_b * op.k)
    D = op.div(op.to_rows(u[:op.F_b * op.k], rows=op.F_b), op.to_rows(u[op.F_b * op.k:]))
    for _ in range(2):
        _, st = op.solve(D, rtol=1e-8, amg=amg)
    torch.cuda.synchronize()
    log(f"amg profile run done: {st['iters']} iterations, {st['seconds']:.4f} s, levels {amg.levels()}")


def pcg_profile_mode(fvx, inputs, torch):
    """A short run for rocprofv3 kernel traces of the Chebyshev-preconditioned
    CG on the channel workload: one warm-up and one timed FP64 solve to 1e-8."""
    spec, mesh, op = build_case(fvx, inputs, K_MAIN)
    tune(op, fvx)
    tune_cg(op, fvx)
    u = inputs.normal(2, 0, op.F_b * op.k + op.n_b * op.k)
    D = op.div(op.to_rows(u[:op.F_b * op.k], rows=op.F_b), op.to_rows(u[op.F_b * op.k:]))
    for _ in range(2):
        _, st = op.solve(D, rtol=1e-8, precond=fvx.PRECOND_CHEBYSHEV)
    torch.cuda.synchronize()
    log(f"pcg profile run done: {st['iters']} iterations, {st['seconds']:.4f} s, "
        f"Chebyshev step bytes {5 * 8 * op.n_b * op.k + 16 * op.n_b} + matrix")


def large_sweep(fvx, inputs, torch, np):
    """Lap SpMM bandwidth on the convection-shaped 160 x 320 base at larger
    plane counts (FP64 and FP32, tuned tiles), beside a streaming copy of the
    same bytes per launch: how close the SpMM gets to the roofline once a
    launch moves hundreds of MB."""
    spec = inputs.convection_base(160, 320)
    mesh = fvx.Mesh.from_spec(spec)
    out = []
    for k in (16, 64, 256):
        op = fvx.Operator(mesh, k, math.pi / k, fvx.PERIODIC_Z, with_f32=True)
        for dt, name, v in ((fvx.F64, "f64", 8), (fvx.F32, "f32", 4)):
            tile = tune(op, fvx, dt)
            x = op.to_rows(inputs.uniform(0, 0, op.n_b * k), dtype=dt)
            per = 2 * op.n_b * op.ld * v
            R = max(3, math.ceil(COLD_BYTES / per))
            X = [x.clone() for _ in range(R)]
            Y = [torch.empty_like(x) for _ in range(R)]
            lap_sweep(op, X[:2], Y[:2], torch)
            t = lap_sweep(op, X, Y, torch, reps=2)
            Bk = spmm_bytes(op.nnz_b, op.n_b, k, v)
            nbytes = op.n_b * op.ld * v
            fvx.copy(Y[0], X[0], nbytes)
            tc = Timer(torch)
            with tc:
                for _ in range(2):
                    for xx, yy in zip(X, Y):
                        fvx.copy(yy, xx, nbytes)
            t_copy = tc.ms() / (2 * R)
            rec = {"k": k, "dtype": name, "tile": list(tile), "cells": op.n_b * k, "bytes_per_launch": Bk,
                   "spmm_us": t * 1e3, "spmm_GBs": Bk / (t * 1e-3) / 1e9,
                   "frac_hbm": Bk / (t * 1e-3) / 1e9 / HBM_PEAK_GBS,
                   "copy_GBs_same_size": 2 * nbytes / (t_copy * 1e-3) / 1e9,
                   "frac_of_copy": (Bk / t) / (2 * nbytes / t_copy)}
            out.append(rec)
            log(f"large k={k} {name}: {rec['spmm_GBs']:.0f} GB/s ({100 * rec['frac_hbm']:.0f}% of 8 TB/s), "
                f"copy {rec['copy_GBs_same_size']:.0f} GB/s")
            del X, Y, x
        del op
        torch.cuda.empty_cache()
    return out


def batch_leg(fvx, inputs, torch, np, rtol):
    """24 uneven problems (4 channel bases x k in {4..128}) solved together in
    mixed precision to rtol, against the same problems solved one by one and
    against plain FP64 SpMV-CG on their assembled matrices."""
    probs = inputs.batch_problems()
    ops, Bs, tiles = [], [], []
    for p in probs:
        mesh = fvx.Mesh.from_spec(p["base"])
        op = fvx.Operator(mesh, p["k"], p["dz"], fvx.PERIODIC_Z, with_f32=True)
        tiles.append((tune(op, fvx), tune(op, fvx, fvx.F32), tune_cg(op, fvx), tune_cg(op, fvx, fvx.F32)))
        Bs.append(op.to_rows(inputs.rhs_uniform(p["seed"], op.n_b * op.k)))
        ops.append((op, mesh))
    opl = [o for o, _ in ops]
    cells = sum(o.n_b * o.k for o in opl)
    log(f"batch: {len(opl)} problems, {cells} cells")
    fvx.solve_batch(opl, Bs, rtol=rtol, precision=fvx.MIXED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Xs, sts = fvx.solve_batch(opl, Bs, rtol=rtol, precision=fvx.MIXED)
    batch_s = time.perf_counter() - t0
    singles, csr = [], []
    for (op, mesh), B in zip(ops, Bs):
        op.solve(B, rtol=rtol, precision=fvx.MIXED)
        t0 = time.perf_counter()
        op.solve(B, rtol=rtol, precision=fvx.MIXED)
        singles.append(time.perf_counter() - t0)
        ptr, col, val = fvx.expand_csr(mesh, op.k, op.dz, fvx.PERIODIC_Z)
        A = fvx.CsrMatrix(ptr, col, val)
        b = torch.as_tensor(op.to_planes(B)).cuda()
        A.solve(b, rtol=rtol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = A.solve(b, rtol=rtol)
        csr.append(time.perf_counter() - t0)
        del A, b
    # The same batch with the Chebyshev preconditioner (degree 8 on [2/300, 2]).
    kwc = dict(rtol=rtol, precision=fvx.MIXED, precond=fvx.PRECOND_CHEBYSHEV)
    fvx.solve_batch(opl, Bs, **kwc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stc = fvx.solve_batch(opl, Bs, **kwc)
    batch_cheb_s = time.perf_counter() - t0
    out = {
        "batch_chebyshev_s": batch_cheb_s,
        "max_relres_true_chebyshev": max(s["relres_true"] for s in stc),
        "problems": [{"base": f"{p['base'].nx}x{p['base'].ny}", "k": p["k"], "cells": o.n_b * o.k,
                      "tile_f64": list(t[0]), "tile_f32": list(t[1]), "cg_tile_f64": list(t[2]),
                      "cg_tile_f32": list(t[3]), "inner_iters": s["iters"],
                      "outer": s["outer"], "relres_true": s["relres_true"], "single_s": ts, "csr3d_fp64_s": tc}
                     for p, o, t, s, ts, tc in zip(probs, opl, tiles, sts, singles, csr)],
        "cells": cells,
        "batch_s": batch_s,
        "sum_single_s": float(sum(singles)),
        "sum_csr3d_fp64_s": float(sum(csr)),
        "max_relres_true": max(s["relres_true"] for s in sts),
        "rtol": rtol,
    }
    log(f"batch {batch_s:.3f} s (Chebyshev {batch_cheb_s:.3f} s), singles {out['sum_single_s']:.3f} s, "
        f"csr3d {out['sum_csr3d_fp64_s']:.3f} s")
    return out


def airfoil_leg(fvx, inputs, torch, np):
    """Extruded NACA-0012 Delaunay mesh (k = 32): SpMM bandwidth in both
    precisions and the mixed-precision solve to 1e-10 against the FP64 solve
    and plain FP64 SpMV-CG."""
    rtol = 1e-10
    spec = inputs.naca_delaunay(seed=1)
    mesh = fvx.Mesh.from_spec(spec)
    k, dz = inputs.AIRFOIL_K, inputs.AIRFOIL_DZ
    op = fvx.Operator(mesh, k, dz, fvx.PERIODIC_Z, with_f32=True)
    res = {"cells_base": op.n_b, "k": k, "cells": op.n_b * k, "nnz_b": op.nnz_b}
    for dt, name, v in ((fvx.F64, "f64", 8), (fvx.F32, "f32", 4)):
        tile = tune(op, fvx, dt)
        x = op.to_rows(inputs.uniform(0, 0, op.n_b * k), dtype=dt)
        per = 2 * op.n_b * op.ld * v
        R = max(2, math.ceil(COLD_BYTES / per))
        X = [x.clone() for _ in range(R)]
        Y = [torch.empty_like(x) for _ in range(R)]
        lap_sweep(op, X[:2], Y[:2], torch)
        t = lap_sweep(op, X, Y, torch, reps=2)
        Bk = spmm_bytes(op.nnz_b, op.n_b, k, v)
        res[f"spmm_{name}"] = {"tile": list(tile), "us": t * 1e3, "GBs": Bk / (t * 1e-3) / 1e9,
                               "frac_hbm": Bk / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del X, Y
    res["cg_tile_f64"], res["cg_tile_f32"] = list(tune_cg(op, fvx)), list(tune_cg(op, fvx, fvx.F32))
    B = op.to_rows(inputs.rhs_uniform(3, op.n_b * k))
    cheb = fvx.PRECOND_CHEBYSHEV
    t0 = time.perf_counter()
    amg = fvx.Amg(op)
    res["amg_setup_s"] = time.perf_counter() - t0
    res["amg_levels"] = amg.levels()
    for prec, pre, name in ((fvx.MIXED, 0, "mixed"), (fvx.F64, 0, "f64"), (fvx.MIXED, cheb, "mixed_chebyshev"),
                            (fvx.F64, cheb, "f64_chebyshev"), (fvx.MIXED, amg, "mixed_amg"), (fvx.F64, amg, "f64_amg")):
        kw = dict(amg=pre) if isinstance(pre, fvx.Amg) else dict(precond=pre)
        op.solve(B, rtol=rtol, precision=prec, **kw)
        t0 = time.perf_counter()
        _, st = op.solve(B, rtol=rtol, precision=prec, **kw)
        res[f"solve_{name}"] = {"s": time.perf_counter() - t0, "iters": st["iters"], "outer": st["outer"],
                                "relres_true": st["relres_true"]}
    del amg
    ptr, col, val = fvx.expand_csr(mesh, k, dz, fvx.PERIODIC_Z)
    A = fvx.CsrMatrix(ptr, col, val)
    b = torch.as_tensor(op.to_planes(B)).cuda()
    A.solve(b, rtol=rtol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = A.solve(b, rtol=rtol)
    res["solve_csr3d_fp64"] = {"s": time.perf_counter() - t0, "iters": st["iters"],
                               "relres_true": st["relres_true"]}
    log(f"airfoil {op.n_b}x{k}: mixed {res['solve_mixed']['s']:.3f} s, f64 {res['solve_f64']['s']:.3f} s, "
        f"Chebyshev mixed {res['solve_mixed_chebyshev']['s']:.3f} s, f64 {res['solve_f64_chebyshev']['s']:.3f} s, "
        f"multigrid mixed {res['solve_mixed_amg']['s']:.3f} s, f64 {res['solve_f64_amg']['s']:.3f} s "
        f"(setup {res['amg_setup_s']:.2f} s), csr3d {res['solve_csr3d_fp64']['s']:.3f} s")
    return res


def guess_leg(fvx, inputs, torch, np, epochs, lr, rtol=1e-8):
    """Learned initial guess on the 64 x 64 x 8 channel: 2000 (rhs, solution)
    pairs from the library's own CG (20 trajectories of 100 steps of drifting
    Fourier modes, seed 4), Adam training, then 100 held-out pairs (seed 5,
    5 trajectories of 20 steps) solved to rtol from a zero guess, from the
    previous pressure, and from the network's guess."""
    cfg = inputs.SMALL_CHANNEL
    spec, k, dz = cfg["base"], cfg["k"], cfg["dz"]
    mesh = fvx.Mesh.from_spec(spec)
    op = fvx.Operator(mesh, k, dz, fvx.PERIODIC_Z, with_f32=False)
    tune(op, fvx)
    tune_cg(op, fvx)
    cx, cy = mesh.centroids()
    area = mesh.faces()[0]

    def pairs(seed, n_traj, n_steps):
        rhs = [[op.to_rows(inputs.integrated_rhs(m, cx, cy, area, k, dz))
                for m in inputs.guess_trajectory(seed, r, n_steps)] for r in range(n_traj)]
        flat = [b for tr in rhs for b in tr]
        sol = []
        for i in range(0, len(flat), 250):
            chunk = flat[i:i + 250]
            X, _ = fvx.solve_batch([op] * len(chunk), chunk, rtol=1e-10)
            sol += X
        it = iter(sol)
        return [[(b, next(it)) for b in tr] for tr in rhs]

    t0 = time.perf_counter()
    train = pairs(4, 20, 100)
    t_gen = time.perf_counter() - t0
    net = fvx.GuessNet(spec.nx, spec.ny, k, batch=16, params=inputs.net_init(6))
    n = sum(len(tr) for tr in train)
    inp = torch.empty((n, 2, k, spec.ny, spec.nx), dtype=torch.float32, device="cuda")
    tgt = torch.empty((n, 1, k, spec.ny, spec.nx), dtype=torch.float32, device="cuda")
    i = 0
    for tr in train:
        for t, (b, x) in enumerate(tr):
            net.prepare(op, b, tr[t - 1][1] if t > 0 else None, x, inp[i], tgt[i])
            i += 1
    del train
    torch.cuda.synchronize()
    log(f"guess: {n} training pairs in {t_gen:.1f} s")
    losses = []
    t0 = time.perf_counter()
    steps = 0
    for e in range(epochs):
        perm = torch.as_tensor(np.argsort(inputs.u64(4, 500 + e, n)), device="cuda")
        tot = 0.0
        for j in range(0, n - 15, 16):
            idx = perm[j:j + 16]
            tot += net.train_step(inp.index_select(0, idx), tgt.index_select(0, idx), lr)
            steps += 1
        losses.append(tot / (n // 16))
        log(f"guess: epoch {e + 1}/{epochs} loss {losses[-1]:.4e}")
    t_train = time.perf_counter() - t0
    del inp, tgt
    test = pairs(5, 5, 20)
    rec = {"zero": [], "prev": [], "net": []}
    used = {fvx.GUESS_NET: 0, fvx.GUESS_GIVEN: 0, fvx.GUESS_ZERO: 0}
    for tr in test:
        for t, (b, _) in enumerate(tr):
            prev = tr[t - 1][1] if t > 0 else None
            _, st = op.solve(b, rtol=rtol)
            rec["zero"].append((st["iters"], st["seconds"], st["relres_true"]))
            X = prev.clone() if prev is not None else op.zeros()
            _, st = op.solve(b, X, rtol=rtol, guess=fvx.GUESS_GIVEN)
            rec["prev"].append((st["iters"], st["seconds"], st["relres_true"]))
            _, st = net.solve(op, b, prev, rtol=rtol)
            rec["net"].append((st["iters"], st["seconds"], st["relres_true"]))
            used[st["source"]] += 1
    # inference alone
    b0, p0 = test[0][1][0], test[0][0][1]
    X0 = op.zeros()
    net.guess(op, b0, p0, X0)
    tm = Timer(torch)
    with tm:
        for _ in range(20):
            net.guess(op, b0, p0, X0)
    infer_ms = tm.ms() / 20
    summ = {m: {"mean_iters": float(np.mean([r[0] for r in v])),
                "mean_ms_to_1e-8": 1e3 * float(np.mean([r[1] for r in v])),
                "max_relres_true": float(max(r[2] for r in v))} for m, v in rec.items()}
    cells = op.n_b * k
    out = {"grid": f"{spec.nx}x{spec.ny}x{k}", "train_pairs": n, "epochs": epochs, "train_steps": steps,
           "batch": 16, "lr": lr, "pair_generation_s": t_gen, "train_s": t_train, "epoch_losses": losses,
           "train_ms_per_step": 1e3 * t_train / max(1, steps), "loss_first_epoch": losses[0] if losses else None,
           "loss_last_epoch": losses[-1] if losses else None, "eval_pairs": len(rec["net"]),
           "guess_chosen": {"net": used[fvx.GUESS_NET], "prev_pressure": used[fvx.GUESS_GIVEN],
                            "zero": used[fvx.GUESS_ZERO]}, "inference_ms": infer_ms,
           "inference_TFLOPs": 2 * cells * 27 * (2 * 32 + 32 * 32 * 2 + 32) / (infer_ms * 1e-3) / 1e12,
           "zero_guess": summ["zero"], "prev_pressure_guess": summ["prev"], "net_guess": summ["net"]}
    log(f"guess: iters zero {summ['zero']['mean_iters']:.0f}, prev {summ['prev']['mean_iters']:.0f}, "
        f"net {summ['net']['mean_iters']:.0f} (chosen {used}); infer {infer_ms:.3f} ms")
    return out


if __name__ == "__main__":
    main()
