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
# Tuned-tile database of the library on MI355X (gfx950): every tile the
# autotuner and the headline refinement chose for the operators this
# benchmark builds, keyed by (architecture, precision, k, ld, base rows, base
# nonzeros, stencil).  Runs start from it, so the timed and the profiled
# kernels are the same instances; --retune rebuilds it from scratch.
TILE_DB = os.path.join(ROOT, "paper_2508_06710_amd", "tiles_gfx950.json")


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


# Section 2's closed forms, as measurement bookkeeping (the tests pin the
# oracle's copy of them against independent values; the benchmark keeps its
# own so that no leg but the CPU baseline runs the oracle).
def ai_eq2(nnz, n_r, n_c, m):
    """Eq. 2: flops (2 nnz + 1) m over bytes 12 nnz + 4 (n_r + 1) + m (8 n_r + 8 n_c + 8)."""
    return (2 * nnz + 1) * m / (12 * nnz + 4 * (n_r + 1) + m * (8 * n_r + 8 * n_c + 8))


def p_ub_eq3a(nnz, n_r, n_c, m):
    """Eq. 3a (= I(m) / I(1) of Eq. 2)."""
    return m * (3 * (nnz + n_r + 1) + 2 * n_c) / (3 * nnz + (1 + 2 * m) * (n_r + 1) + 2 * m * n_c)


def p_lb_eq3b(nnz, n_r, m):
    """Eq. 3b (no reuse of the gathered input)."""
    return m * (5 * nnz + 3 * (n_r + 1)) / ((3 + 2 * m) * nnz + (1 + 2 * m) * (n_r + 1))


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


class Plug:
    """About 2 ms of streaming copies (6 x 1 GiB) put on the stream ahead of a
    timed sweep: the sweep's launches queue up behind it, so they run back to
    back on the GPU whatever the host's launch rate -- also under a kernel
    tracer, whose per-launch host overhead (about 13 us here) would
    otherwise leave each short kernel isolated with its own ramp and drain.
    The copies also flush the caches ahead of the sweep."""

    def __init__(self, fvx, torch):
        self.fvx = fvx
        self.a = torch.empty(2 ** 30 // 8, dtype=torch.float64, device="cuda")
        self.b = torch.empty_like(self.a)

    def __call__(self):
        for _ in range(6):
            self.fvx.copy(self.b, self.a)


def lap_sweep(op, X, Y, torch, reps=1, plug=None):
    """Mean time per lap SpMM over the rotating pairs (launched from C),
    HIP events around the sweep on the launch stream; with a plug, its
    copies run ahead of the first event.""" 
    if plug is not None:
        plug()
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


def setup_tile_cache(retune):
    """The run's tile cache: FVX_TUNE_CACHE if set, else
    gpurun_out/tiles_gfx950.json, seeded from the committed database unless
    retune (operators missing from it are tuned and added)."""
    import shutil
    path = os.environ.get("FVX_TUNE_CACHE") or os.path.join(ROOT, "gpurun_out", "tiles_gfx950.json")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    if retune:
        if os.path.exists(path):
            os.remove(path)
    elif not os.path.exists(path) and os.path.exists(TILE_DB):
        shutil.copyfile(TILE_DB, path)
    os.environ["FVX_TUNE_CACHE"] = path
    log(f"tile cache {path} ({'retune' if retune else 'from the database' if os.path.exists(path) else 'empty'})")


def lanczos_kappa(op, inputs, torch, m, seed=11):
    """kappa_est of the SPD operator A = -L on the complement of its null
    space: the ratio of the extreme Ritz values of m Lanczos steps (the
    tridiagonal that CG builds implicitly), started from a random vector;
    the Lanczos vectors are kept at zero mean (per column for independent
    planes) so that rounding does not bring the null space back.  Ritz
    values lie inside the spectrum, so this estimate is at most kappa."""
    import numpy as np
    from scipy.linalg import eigvalsh_tridiagonal
    k = op.k
    percol = op.coupling == 0 or k == 1

    def proj(v):
        if op.singular:
            vv = v[:, :k]
            vv -= vv.mean(dim=0, keepdim=True) if percol else vv.mean()

    def dot(a, b):
        return (a[:, :k] * b[:, :k]).sum()

    v = op.to_rows(inputs.uniform(seed, 0, op.n_b * k))
    proj(v)
    v /= torch.sqrt(dot(v, v))
    vp, w = torch.zeros_like(v), torch.empty_like(v)
    beta = torch.zeros((), dtype=torch.float64, device=v.device)
    al, be = [], []
    for _ in range(m):
        op.lap(v, w)
        w.neg_()
        a = dot(w, v)
        w -= a * v
        w -= beta * vp
        proj(w)
        beta = torch.sqrt(dot(w, w))
        al.append(a)
        be.append(beta)
        w /= beta
        vp, v, w = v, w, vp
    d = torch.stack(al).cpu().numpy()
    e = torch.stack(be).cpu().numpy()[:-1]
    lo = eigvalsh_tridiagonal(d, e, select="i", select_range=(0, 0))[0]
    hi = eigvalsh_tridiagonal(d, e, select="i", select_range=(m - 1, m - 1))[0]
    return float(hi / lo), float(lo), float(hi)


def rel_err(torch, op, X, Xs):
    k = op.k
    return float(torch.linalg.vector_norm(X[:, :k] - Xs[:, :k]) / torch.linalg.vector_norm(Xs[:, :k]))


def mixed_errors(fvx, inputs, torch, op, B, sols, rtol_star=1e-13, steps=None, star_kw=None):
    """Error of mixed-precision solutions against the FP64 solution x* to
    rtol_star (the library's FP64 CG, plain or with star_kw's
    preconditioner), per result, beside the a-posteriori bound
    kappa_est (relres + relres*): ||x - x_true|| <= ||r|| / lambda_min and
    ||x_true|| >= ||b|| / lambda_max.  kappa_est comes from `steps` Lanczos
    steps (default: the plain x* solve's iteration count, at most 3000).
    sols: {name: (X, stats)}.  Returns (record, x*)."""
    Xs, sts = op.solve(B, rtol=rtol_star, **(star_kw or {}))
    m = steps if steps else min(max(sts["iters"], 50), 3000)
    kap, lo, hi = lanczos_kappa(op, inputs, torch, m)
    out = {"x_star": {"rtol": rtol_star, "iters": sts["iters"], "relres_true": sts["relres_true"]},
           "kappa_est": kap, "lanczos_steps": m}
    for name, (X, st) in sols.items():
        err = rel_err(torch, op, X, Xs)
        bound = kap * (st["relres_true"] + sts["relres_true"])
        out[name] = {"rel_err_vs_fp64": err, "bound_kappa": bound, "relres_true": st["relres_true"]}
    return out, Xs


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
    # 24 iterations of the plain FP64 CG with the tuned CG tile, launched
    # phase by phase (the direction kernel kb_cg_a and the update kernel kb_cg_b)
    tune_cg(op, fvx)
    B = op.to_rows(inputs.rhs_uniform(3, op.n_b * op.k))
    op.solve(B, rtol=1e-300, max_iter=24, poll_every=24, launch=fvx.LAUNCH_PHASES, allow_not_converged=True)
    log("counters: 24 CG iterations")
    nbytes = 256 * 2 ** 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = [torch.empty_like(src) for _ in range(2)]
    for i in range(8):
        fvx.copy(dst[i % 2], src)
    torch.cuda.synchronize()
    log(f"counters run done: lap bytes/launch {spmm_bytes(op.nnz_b, op.n_b, op.k)}, copy bytes {nbytes}")


def summarize_counters(fetch_dir, write_dir, flops_dir, out=COUNTER_FILE):
    """Writes the counters file from three rocprofv3 --pmc runs of
    `bench.py --counters` (FETCH_SIZE; WRITE_SIZE; the FP64 VALU counters):
    per lap kernel instance the median FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) scaled by what the same counters read for the 256 MiB copy of
    the run, and the FP64 floating-point operations counted per dispatch.
    Runs on any host (CSV files only)."""
    import csv
    import glob
    import re
    import statistics

    def rows(d):
        out = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                out += list(csv.DictReader(fh))
        return out

    def short(n):
        n = n.replace("void ", "").replace("fvx::(anonymous namespace)::", "").replace("fvx::", "")
        return re.sub(r"\(.*", "", n).strip()

    def per_kernel(rs):
        acc = {}
        for r in rs:
            key = (short(r["Kernel_Name"]), int(r["Dispatch_Id"]))
            acc.setdefault(key, {})
            acc[key][r["Counter_Name"]] = acc[key].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        byk = {}
        for (name, _), cs in acc.items():
            byk.setdefault(name, []).append(cs)
        return byk

    fk, wk, pk = per_kernel(rows(fetch_dir)), per_kernel(rows(write_dir)), per_kernel(rows(flops_dir))
    med = lambda lst, c: statistics.median(x.get(c, 0.0) for x in lst)
    copy_bytes = 256 * 2 ** 20
    cf, cw = med(fk["k_copy"], "FETCH_SIZE"), med(wk["k_copy"], "WRITE_SIZE")
    fs, ws = copy_bytes / (cf * 1024), copy_bytes / (cw * 1024)
    nb, k = BASE[0] * BASE[1], K_MAIN
    nnz_b = nb + 2 * (BASE[0] * BASE[1] * 2 - BASE[0])  # periodic x faces + interior y faces, 5-point base
    alg = spmm_bytes(nnz_b, nb, k)
    # The CG kernels on the Cartesian base: per base row one 64-byte record
    # (meta_cart) and, per vector pass, k FP64 values; the direction kernel
    # reads r and p and writes p' (3 passes), the update kernel reads p', x and
    # r and writes x and r (5 passes).  Their five vectors (63 MB) fit in the
    # 256 MB Infinity Cache, so FETCH_SIZE counts reads from the fabric
    # (Infinity Cache hits included), not HBM reads alone.
    vec, rec_b = nb * k * 8, nb * 64
    cg_alg = {"kb_cg_a": 3 * vec + rec_b, "kb_cg_b": 5 * vec + rec_b}
    by_kernel = {}
    for name in fk:
        base = name.split("<")[0]
        if not (name.startswith("k_lap") or base in cg_alg):
            continue
        alg_n = cg_alg.get(base, alg)
        f = med(fk[name], "FETCH_SIZE") * 1024 * fs
        w = med(wk.get(name, [{}]), "WRITE_SIZE") * 1024 * ws
        e = {"kernel": name, "dispatches": len(fk[name]), "fetch_kib_per_dispatch": med(fk[name], "FETCH_SIZE"),
             "write_kib_per_dispatch": med(wk.get(name, [{}]), "WRITE_SIZE"), "fetch_bytes_per_launch": f,
             "write_bytes_per_launch": w, "algorithmic_bytes": alg_n, "traffic_over_algorithmic": (f + w) / alg_n}
        if name in pk:
            lst = pk[name]
            # the counter adds each FP64 VALU instruction's flops per lane (FMA 2,
            # ADD/MUL 1) once per wave instruction: times 64 lanes
            e["fp64_flops_counted"] = 64 * med(lst, "SQ_INSTS_VALU_FLOPS_FP64")
            e["fp64_flops_from_insts"] = 64 * (med(lst, "SQ_INSTS_VALU_ADD_F64") + med(lst, "SQ_INSTS_VALU_MUL_F64")
                                               + 2 * med(lst, "SQ_INSTS_VALU_FMA_F64"))
            if base not in cg_alg:
                e["fp64_flops_algorithmic"] = spmm_flops(nnz_b, nb, k)
        by_kernel[name] = e
    rec = {"workload": f"channel {BASE[0]}x{BASE[1]} base x {K_MAIN} periodic planes, FP64, cold (rotating buffers > 1 GiB)",
           "commands": ["rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_fetch -o fetch -- python3 bench.py --counters",
                        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_write -o write -- python3 bench.py --counters",
                        "rocprofv3 --pmc SQ_INSTS_VALU_FLOPS_FP64 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 "
                        "SQ_INSTS_VALU_FMA_F64 --output-format csv -d gpurun_out/pmc_flops -o flops -- python3 bench.py --counters",
                        "python bench.py --summarize-counters gpurun_out/pmc_fetch gpurun_out/pmc_write gpurun_out/pmc_flops"],
           "algorithmic_bytes_per_launch": alg,
           "copy_calibration": {"copy_bytes": copy_bytes, "fetch_kib": cf, "write_kib": cw, "fetch_scale": fs,
                                "write_scale": ws},
           "source_sha": kernel_source_sha(), "by_kernel": by_kernel}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"wrote {out}: " + ", ".join(f"{n}: {e['traffic_over_algorithmic']:.3f}x" for n, e in by_kernel.items()))


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
    (timed repeatedly) and its textbook CG to rtol on the same right-hand
    side, with all host threads; then on one thread the SpMV and a CG capped
    at 60 iterations, whose time per iteration is scaled to the all-thread
    run's iteration count (a bounded sample: about 10 s of one core)."""
    spec = inputs.channel_base(*BASE)
    g = oracle.geometry(spec)
    m3 = oracle.Mesh3D(g, k, math.pi / k, oracle.PERIODIC_Z)
    t0 = time.perf_counter()
    L = m3.lap()
    t_asm = time.perf_counter() - t0
    x = inputs.uniform(0, 0, m3.N)
    y = oracle.spmv(L, x)

    def time_spmv(max_reps, budget_s):
        ts = []
        while len(ts) < max_reps and sum(ts) < budget_s:
            t0 = time.perf_counter()
            oracle.spmv(L, x, out=y)
            ts.append(time.perf_counter() - t0)
        return float(sorted(ts)[len(ts) // 2]), len(ts)

    threads = oracle.threads()
    t_spmv, reps = time_spmv(20, 5.0)
    log(f"oracle spmv {t_spmv * 1e3:.2f} ms (median of {reps}, {threads} threads), assembly {t_asm:.1f} s")
    t0 = time.perf_counter()
    r = oracle.cg(m3, L, b_plane, rtol, max_iter=20000)
    t_cg = time.perf_counter() - t0
    log(f"oracle CG {r.iters[0]} iters {t_cg:.2f} s ({threads} threads)")
    oracle.set_threads(1)
    try:
        t_spmv1, reps1 = time_spmv(5, 3.0)
        cap = 60
        t0 = time.perf_counter()
        oracle.cg(m3, L, b_plane, rtol, max_iter=cap)
        t_it1 = (time.perf_counter() - t0) / cap
    finally:
        oracle.set_threads(threads)
    log(f"oracle 1 thread: spmv {t_spmv1 * 1e3:.2f} ms, CG {t_it1 * 1e3:.2f} ms per iteration")
    nb = g.n_cells
    nnz_b = nb + 2 * g.n_faces
    Bk = spmm_bytes(nnz_b, nb, k)
    return {
        "value": Bk / t_spmv / 1e9,
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle assembled-3D CSR SpMV on the {BASE[0]}x{BASE[1]}x{k} channel (median of {reps}), "
                   f"GB/s counted with the SpMM's algorithmic bytes (the same product); one oracle CG to {rtol:g} "
                   f"on the projection right-hand side; 1 thread: SpMV median of {reps1} and a 60-iteration CG "
                   f"scaled to the full iteration count"),
        "value_1thread": Bk / t_spmv1 / 1e9,
        "csr_own_GBs": csr3d_bytes(L.nnz, m3.N) / t_spmv / 1e9,
        "spmv_ms": t_spmv * 1e3,
        "spmv_ms_1thread": t_spmv1 * 1e3,
        "poisson_s_to_1e-8": t_cg,
        "poisson_s_to_1e-8_1thread": t_it1 * r.iters[0],
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
    ap.add_argument("--launch-only", action="store_true",
                    help="only the launch-mode comparison (phase by phase vs graph replay) of the solves")
    ap.add_argument("--guess-epochs", type=int, default=20)
    ap.add_argument("--guess-lr", type=float, default=1e-4)
    ap.add_argument("--retune", action="store_true",
                    help="ignore the tile database and tune every operator again")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "FLOPS_DIR"),
                    help="write the counters file from rocprofv3 --pmc output of --counters runs (no GPU needed)")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
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
    setup_tile_cache(args.retune)
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
    plug = Plug(fvx, torch)
    log(f"{N} cells, {len(X)} rotating lap buffer pairs ({len(X) * 2 * n_b * op.ld * 8 / 2**30:.2f} GiB)")
    if args.launch_only:
        op.div(U0, W0, D)
        rec = {"launch_modes": launch_leg(fvx, torch, op, D, rtol)}
        rec["launch_modes"]["batch_mixed"] = batch_leg(fvx, inputs, torch, np, rtol, launch_only=True)
        path = os.path.join(ROOT, "gpurun_out", "bench_launch.json")
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        log(f"wrote {path}")
        return

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
        t_lap = lap_sweep(op, X, Y, torch, plug=plug)
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

    # Headline: per step, the mean launch time of the lap SpMM over one sweep
    # of the rotating buffers (HIP events around the sweep on the launch
    # stream); the median over the timed steps.
    laps = sorted(r["lap_ms"] for r in recs)
    lap_ms = float(np.median(laps))
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
    flops_counted = None
    if cnt:  # counters of this very kernel instance
        hit = [e for e in cnt.get("by_kernel", {}).values() if norm(e.get("kernel", "")) == norm(lap_kernel_name(tile, k))]
        if hit:
            traffic = hit[0]["fetch_bytes_per_launch"] + hit[0]["write_bytes_per_launch"]
            flops_counted = hit[0].get("fp64_flops_counted")
    full = {
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
                     "launch_us": lap_ms * 1e3, "launch_us_min": laps[0] * 1e3, "launch_us_max": laps[-1] * 1e3,
                     "sweep_launches": len(X), "fp64_tflops": Fk / (lap_ms * 1e-3) / 1e12,
                     "fp64_tflops_counted": None if flops_counted is None else flops_counted / (lap_ms * 1e-3) / 1e12,
                     "fp64_peak_tflops": FP64_PEAK_TFLOPS, "intensity_flop_per_byte": Fk / Bk,
                     "source_sha": sha},
        "poisson": {"s_to_1e-8": solve_s, "iters": st["iters"], "relres_true": st["relres_true"], "cg_tiles": cg_tiles,
                    "ms_per_iter": solve_s * 1e3 / max(1, st["iters"]),
                    "div_after_over_before": div_ratio},
        "phases_ms": {p: float(np.mean([r[p] for r in recs])) for p in ("div_ms", "solve_ms", "grad_ms", "lap_ms")},
    }

    legs = {}
    if not args.no_sweep:
        legs.update(extra_measurements(fvx, inputs, torch, np, op, mesh, rtol, D))
        same = [c for c in legs["copy_ceiling"] if c["size"] == "headline_traffic"]
        if same:
            full["roofline"]["copy_same_bytes_GBs"] = same[0]["GBs"]
            full["roofline"]["frac_of_copy"] = achieved / same[0]["GBs"]

    if not args.no_stencil:
        legs["stencils"] = stencil_leg(fvx, inputs, torch, np)
        torch.cuda.empty_cache()
        legs["refine_mapping"] = refine_leg(fvx, inputs, torch, np)
        torch.cuda.empty_cache()
        legs["generic_spmm"] = generic_leg(fvx, inputs, torch, np)
        torch.cuda.empty_cache()
    if not args.no_ns:
        legs["ns_step"] = ns_leg(fvx, inputs, torch, np)
        torch.cuda.empty_cache()
    if not args.no_batch:
        legs["batched"] = batch_leg(fvx, inputs, torch, np, rtol)
        torch.cuda.empty_cache()
    if not args.no_airfoil:
        legs["airfoil"] = airfoil_leg(fvx, inputs, torch, np)
        torch.cuda.empty_cache()
    if not args.no_guess:
        legs["learned_guess"] = guess_leg(fvx, inputs, torch, np, args.guess_epochs, args.guess_lr, rtol)
        torch.cuda.empty_cache()

    if not args.no_cpu:
        log("timing the CPU oracle")
        b_plane = op.to_planes(D)
        full["cpu_baseline"] = cpu_baseline(inputs, __import__("oracle"), b_plane, k, rtol)
    full.update(legs)
    path = os.path.join(ROOT, "gpurun_out", "bench_profile.json" if args.profile else "bench_full.json")
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as fh:
            json.dump(full, fh, indent=1)
        log(f"every leg written to {path}")
    except OSError as e:
        log(f"could not write {path}: {e}")
    line = json.dumps(compact_line(full, legs))
    print(line, flush=True)


def compact_line(full, legs):
    """The one JSON line of the contract: the headline, its roofline, the
    Poisson times and the CPU baseline, each leg reduced to its key figures
    (the full record goes to gpurun_out/bench_full.json), under 4 KB."""
    r = lambda v, n=4: None if v is None else float(f"{v:.{n}g}")
    keys = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
            "vs_baseline", "dtype", "data")
    out = {k: full[k] for k in keys}
    out["value"] = r(out["value"], 5)
    out["ms_per_step"] = r(out["ms_per_step"], 5)
    c = full["config"]
    out["config"] = {"workload": c["workload"], "base": c["base"], "k": c["k"], "cells": c["cells"]}
    rf = full["roofline"]
    out["roofline"] = {q: (r(rf[q]) if isinstance(rf.get(q), float) else rf.get(q))
                       for q in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel", "launch_us",
                                 "launch_us_min", "launch_us_max", "bytes_per_launch", "fp64_tflops",
                                 "fp64_tflops_counted",
                                 "copy_same_bytes_GBs", "frac_of_copy") if q in rf}
    p = full["poisson"]
    out["poisson"] = {"s_to_1e-8": r(p["s_to_1e-8"]), "iters": p["iters"], "relres_true": r(p["relres_true"], 3),
                      "ms_per_iter": r(p["ms_per_iter"])}
    if "csr3d_cg" in legs:
        out["poisson"]["csr3d_spmv_cg_s"] = r(legs["csr3d_cg"]["s_to_1e-8"])
    if "mixed_cg" in legs:
        m = legs["mixed_cg"]
        out["poisson"]["mixed"] = {"s": r(m["s_to_1e-8"]), "rel_err_vs_fp64": r(m["rel_err_vs_fp64"], 3),
                                   "bound": r(m["bound_kappa"], 3), "kappa_est": r(m["kappa_est"], 3)}
    if "poisson_pcg" in legs:
        out["poisson"]["chebyshev_s"] = r(legs["poisson_pcg"]["chebyshev"]["s_to_1e-8"])
    if "poisson_amg" in legs:
        out["poisson"]["multigrid_s"] = r(legs["poisson_amg"]["f64"]["s_to_1e-8"])
        out["poisson"]["multigrid_iters"] = legs["poisson_amg"]["f64"]["iters"]
    if "k_sweep" in legs:
        out["k_sweep"] = [{"k": e["k"], "GBs": r(e["spmm_GBs"]), "P_k": r(e["P_k"], 3),
                           "vs_csr3d": r(e["speedup_vs_csr3d"], 3)} for e in legs["k_sweep"]]
    if "copy_ceiling" in legs:
        out["copy_GBs"] = {e["size"]: r(e["GBs"]) for e in legs["copy_ceiling"]}
    if "stencils" in legs:
        out["stencil_k64_f64_GBs"] = {str(e["stencil"]): r(e["spmm_GBs"]) for e in legs["stencils"]
                                      if e["k"] == 64 and e["dtype"] == "f64"}
    if "batched" in legs:
        b = legs["batched"]
        out["batched"] = {"s": r(b["batch_s"]), "singles_s": r(b["sum_single_s"]), "csr3d_s": r(b["sum_csr3d_fp64_s"]),
                          "max_rel_err_vs_fp64": r(b["max_rel_err_vs_fp64"], 3),
                          "max_err_over_bound": r(b["max_err_over_bound"], 3)}
    if "airfoil" in legs:
        a = legs["airfoil"]
        out["airfoil"] = {"spmm_f64_GBs": r(a["spmm_f64"]["GBs"]), "spmm_f32_GBs": r(a["spmm_f32"]["GBs"]),
                          "cell_order": a["cell_order"],
                          "spmm_f64_GBs_generator_order": r(a["as_generated_order"]["spmm_f64"]["GBs"]),
                          "mixed_s": r(a["solve_mixed"]["s"]), "f64_s": r(a["solve_f64"]["s"]),
                          "mixed_multigrid_s": r(a["solve_mixed_amg"]["s"]),
                          "csr3d_s": r(a["solve_csr3d_fp64"]["s"]),
                          "mixed_rel_err_vs_fp64": r(a["solve_mixed"]["rel_err_vs_fp64"], 3),
                          "mixed_bound": r(a["solve_mixed"]["bound_kappa"], 3)}
    if "learned_guess" in legs:
        g = legs["learned_guess"]
        out["learned_guess"] = {"iters_zero": r(g["zero_guess"]["mean_iters"]),
                                "iters_prev": r(g["prev_pressure_guess"]["mean_iters"]),
                                "iters_net": r(g["net_guess"]["mean_iters"]),
                                "ms_zero": r(g["zero_guess"]["mean_ms_to_1e-8"]),
                                "ms_net": r(g["net_guess"]["mean_ms_to_1e-8"]),
                                "net_chosen": g["guess_chosen"]["net"], "eval_pairs": g["eval_pairs"]}
    if "cpu_baseline" in full:
        cb = full["cpu_baseline"]
        out["cpu_baseline"] = {"value": r(cb["value"]), "unit": cb["unit"], "cores": cb["cores"], "kind": cb["kind"],
                               "sample": cb["sample"], "value_1thread": r(cb["value_1thread"]),
                               "poisson_s_to_1e-8": r(cb["poisson_s_to_1e-8"]),
                               "poisson_s_to_1e-8_1thread": r(cb["poisson_s_to_1e-8_1thread"]),
                               "nproc": cb["nproc"], "cpu_model": cb["cpu_model"]}
    out["legs_file"] = "gpurun_out/bench_full.json"
    while len(json.dumps(out)) > 4000:  # keep the line short enough for any capture
        for q in ("stencil_k64_f64_GBs", "copy_GBs", "k_sweep", "learned_guess", "airfoil", "batched"):
            if q in out:
                del out[q]
                break
        else:
            break
    return out


def extra_measurements(fvx, inputs, torch, np, op, mesh, rtol, D):
    """k sweep (SpMM vs k single-column products and vs the assembled 3D CSR
    SpMV), the copy ceiling, the assembled-CSR CG comparator and the mixed
    precision solve.  Measured outside the timed steps."""
    res = {"copy_ceiling": copy_leg(fvx, torch, spmm_bytes(op.nnz_b, op.n_b, op.k))}
    res["copy_ceiling_GBs"] = max(c["GBs"] for c in res["copy_ceiling"])

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
               "P_ub_eq3a": p_ub_eq3a(opk.nnz_b, opk.n_b, opk.n_b, k)}
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
    # Mixed precision solve to 1e-8 on the SpMM operator, and its error
    # against the FP64 solution to 1e-13 beside the kappa bound.
    op.solve(D, rtol=rtol, precision=fvx.MIXED)
    tm = Timer(torch)
    with tm:
        Xm, stm = op.solve(D, rtol=rtol, precision=fvx.MIXED, inner_rtol=1e-4)
    Xf, stf = op.solve(D, rtol=rtol)
    errs, Xstar = mixed_errors(fvx, inputs, torch, op, D, {"mixed": (Xm, stm), "fp64": (Xf, stf)})
    res["mixed_cg"] = {"s_to_1e-8": tm.ms() / 1e3, "inner_iters": stm["iters"], "outer": stm["outer"],
                       "relres_true": stm["relres_true"], "rel_err_vs_fp64": errs["mixed"]["rel_err_vs_fp64"],
                       "bound_kappa": errs["mixed"]["bound_kappa"], "kappa_est": errs["kappa_est"],
                       "fp64_rtol_rel_err": errs["fp64"]["rel_err_vs_fp64"], "x_star": errs["x_star"]}
    log(f"mixed vs FP64 x*: rel err {errs['mixed']['rel_err_vs_fp64']:.2e} (bound {errs['mixed']['bound_kappa']:.2e},"
        f" kappa_est {errs['kappa_est']:.3e}); FP64 at rtol: {errs['fp64']['rel_err_vs_fp64']:.2e}")
    kap = errs["kappa_est"]
    star_res = errs["x_star"]["relres_true"]

    def err_of(X, st):
        return {"rel_err_vs_fp64": rel_err(torch, op, X, Xstar), "bound_kappa": kap * (st["relres_true"] + star_res)}

    res["poisson_pcg"] = pcg_leg(fvx, torch, op, D, rtol, err_of)
    res["poisson_amg"] = amg_leg(fvx, torch, inputs, op, D, rtol, err_of)
    res["launch_modes"] = launch_leg(fvx, torch, op, D, rtol)
    log(f"csr3d CG {res['csr3d_cg']['s_to_1e-8']:.3f} s, mixed {res['mixed_cg']['s_to_1e-8']:.3f} s")
    return res


def launch_modes(fvx, torch, solve, reps=3):
    """One solve configuration launched phase by phase and replayed from HIP
    graphs: per mode the first solve (in graph mode it captures the graphs)
    and the best of `reps` later ones.  solve(launch) returns (X, stats) or
    (Xs, [stats])."""
    rec = {}
    for mode, lm in (("phases", fvx.LAUNCH_PHASES), ("graph", fvx.LAUNCH_GRAPH)):
        times = []
        for _ in range(reps + 1):
            tm = Timer(torch)
            with tm:
                _, st = solve(lm)
            times.append(tm.ms() / 1e3)
        sts = st if isinstance(st, list) else [st]
        rec[mode] = {"first_s": times[0], "s": min(times[1:]), "iters": max(x["iters"] for x in sts)}
    rec["graph_speedup"] = rec["phases"]["s"] / rec["graph"]["s"]
    return rec


def launch_leg(fvx, torch, op, D, rtol):
    """The CG iterations of the benchmark's solves launched kernel by kernel
    and replayed from HIP graphs: plain, Chebyshev and multigrid CG in FP64,
    multigrid and plain CG in mixed precision (default options otherwise)."""
    amg = fvx.Amg(op)
    cases = {"plain": {}, "chebyshev": dict(precond=fvx.PRECOND_CHEBYSHEV), "mixed": dict(precision=fvx.MIXED),
             "multigrid": dict(amg=amg), "multigrid_mixed": dict(amg=amg, precision=fvx.MIXED)}
    out = {}
    for name, kw in cases.items():
        out[name] = launch_modes(fvx, torch, lambda lm: op.solve(D, rtol=rtol, launch=lm, **kw))
        r = out[name]
        log(f"launch {name}: phases {r['phases']['s'] * 1e3:.2f} ms, graph {r['graph']['s'] * 1e3:.2f} ms "
            f"(first {r['graph']['first_s'] * 1e3:.2f} ms), {r['phases']['iters']} iterations")
    return out


def copy_leg(fvx, torch, headline_bytes):
    """Achievable-bandwidth reference: the library's streaming copy (fvx_copy)
    over rotating buffer pairs totalling more than 1 GiB (cold Infinity
    Cache), at the headline launch's traffic (a copy of half its algorithmic
    bytes), at buffers of 16.8, 26.9, 56.1 and 213 MB, and at 1 GiB.  Time
    per launch: the median over 3 back-to-back sweeps of the mean per launch
    (HIP events on the launch stream); GB/s counts the bytes read and
    written."""
    out = []
    sizes = [("headline_traffic", headline_bytes / 2)] + [(f"{mb:g}MB", mb * 1e6) for mb in (16.8, 26.9, 56.1, 213.0)] \
        + [("1GiB", float(2 ** 30))]
    for label, size in sizes:
        nbytes = int(size) // 4096 * 4096
        R = max(2, math.ceil(COLD_BYTES / (2 * nbytes)))
        src = [torch.ones(nbytes // 8, dtype=torch.float64, device="cuda") for _ in range(R)]
        dst = [torch.empty_like(src[0]) for _ in range(R)]
        fvx.copy_many(dst, src)
        ts = []
        for _ in range(3):
            tm = Timer(torch)
            with tm:
                fvx.copy_many(dst, src)
            ts.append(tm.ms() / R)
        t = sorted(ts)[1]
        rec = {"size": label, "bytes_per_launch": 2 * nbytes, "us": t * 1e3, "GBs": 2 * nbytes / (t * 1e-3) / 1e9}
        rec["frac_hbm"] = rec["GBs"] / HBM_PEAK_GBS
        out.append(rec)
        log(f"copy {label} ({2 * nbytes / 1e6:.1f} MB moved): {rec['us']:.2f} us, {rec['GBs']:.0f} GB/s "
            f"({100 * rec['frac_hbm']:.1f}% of 8 TB/s)")
        del src, dst
        torch.cuda.empty_cache()
    return out


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
                rec.update({"P_k": k * t1[name] / t, "P_ub_eq3a": p_ub_eq3a(nnz, n_r, n_c, k)})
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
                   "P_ub_eq3a": p_ub_eq3a(nnz, n, n, m), "P_lb_eq3b": p_lb_eq3b(nnz, n, m)}
            out.append(rec)
            log(f"generic SpMM {points} nnz/row m={m}: {rec['spmm_us']:.1f} us ({rec['spmm_GBs']:.0f} GB/s), "
                f"P_m {rec['P_m']:.2f} (bounds {rec['P_lb_eq3b']:.2f}..{rec['P_ub_eq3a']:.2f}; "
                f"vs the CSR-vector SpMV {rec['P_m_vs_csr_spmv']:.2f})")
            torch.cuda.empty_cache()
        del M, A
    return out


def pcg_leg(fvx, torch, op, D, rtol, err_of=None):
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
                X, st = op.solve(D, rtol=rtol, **kw)
            best = tm.ms() if best is None else min(best, tm.ms())
        o = op.solve_opts(**kw)
        out[name] = {"s_to_1e-8": best / 1e3, "iters": st["iters"], "outer": st["outer"],
                     "relres_true": st["relres_true"], "cheb_degree": int(o.cheb_degree),
                     "cheb_ratio": float(o.cheb_ratio)}
        if err_of is not None and kw.get("precision") == fvx.MIXED:
            out[name].update(err_of(X, st))
        log(f"pcg {name}: {best:.2f} ms, {st['iters']} iterations, true residual {st['relres_true']:.2e}")
    return out


def amg_leg(fvx, torch, inputs, op, D, rtol, err_of=None):
    """CG preconditioned by one V-cycle of the aggregation multigrid (default
    options: Chebyshev degree 2 on [2/8, 2], pairwise aggregation with beta
    0.75, plane merging when the plane coupling dominates, coarsest level at
    most 2048 unknowns, or solved per plane mode at the first level whose
    modes hold at most 2^23 terms) on the benchmark's projection right-hand side, FP64 and
    mixed precision, the best of 3 timed solves each; the time of one V-cycle
    and, per level, the level's SpMM (its operator on the level's k planes;
    graph-timed, inputs warm in the caches) -- the per-level SpMM table of the
    paper's multigrid appendix."""
    t0 = time.perf_counter()
    amg = fvx.Amg(op)
    out = {"setup_s": time.perf_counter() - t0, "levels": [], "coarsest_modes": amg.coarsest_modes}
    for name, kw in (("f64", {}), ("mixed", dict(precision=fvx.MIXED))):
        op.solve(D, rtol=rtol, amg=amg, **kw)
        best, st = None, None
        for _ in range(3):
            tm = Timer(torch)
            with tm:
                X, st = op.solve(D, rtol=rtol, amg=amg, **kw)
            best = tm.ms() if best is None else min(best, tm.ms())
        out[name] = {"s_to_1e-8": best / 1e3, "iters": st["iters"], "outer": st["outer"],
                     "relres_true": st["relres_true"]}
        if err_of is not None and name == "mixed":
            out[name].update(err_of(X, st))
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
    out["app_a"] = app_a_accounting(out["levels"], out["f64"]["iters"], amg.degree if hasattr(amg, "degree") else 2)
    a = out["app_a"]
    log(f"App. A: weighted Eq. 3a bound {a['P_ub_weighted']:.2f} over {len(a['products'])} product kinds, "
        f"pi_SpMM {a['pi_spmm_gflops']:.0f} GFLOP/s over the timed square products")
    return out


def app_a_accounting(levels, cg_iters, degree=2):
    """The accounting of the paper's Appendix A for this multigrid: every
    sparse product of one preconditioned-CG solve with its shape (rows,
    columns, nonzeros of the base block, right-hand sides m = planes) and
    call count, the weight w_i = calls_i / all calls, the weighted upper bound
    sum_i w_i P_ub(nnz_i, n_r,i, n_c,i, m_i) (Eq. 3a per product), the weighted
    Eq. 2 intensity, and pi_SpMM = sum_i w_i OC_i / t_i with OC_i = (2 nnz_i +
    1) m_i over the products timed one by one (the square level products; the
    restrictions and prolongations are fused into level kernels and carry no
    time of their own, so pi's weights are renormalised over the timed ones).
    Per CG iteration: two level-0 products (direction and update kernels)
    and one V-cycle, which on every level but the coarsest applies the level
    operator 2 * degree times (degree - 1 pre-smoothing products, the
    residual before the restriction, degree post-smoothing products), one
    restriction and one prolongation; the coarsest level is a dense product
    with its pseudo-inverse."""
    prods = []

    def add(kind, lvl, n_r, n_c, nnz, m, calls, t_us=None):
        prods.append({"kind": kind, "level": lvl, "n_r": n_r, "n_c": n_c, "nnz": nnz, "m": m, "calls": calls,
                      "t_us": t_us})

    L = levels
    add("cg level 0", 0, L[0]["n_b"], L[0]["n_b"], L[0]["nnz_b"], L[0]["k"], 2 * cg_iters, L[0]["spmm_us"])
    for l, lv in enumerate(L):
        n, k, nnz = lv["n_b"], lv["k"], lv["nnz_b"]
        if lv["next"] == "coarsest":
            nd = n * k
            add("coarsest dense", l, nd, nd, nd * nd, 1, cg_iters)
            break
        add("level operator", l, n, n, nnz, k, 2 * degree * cg_iters, lv["spmm_us"])
        nxt = L[l + 1]
        if lv["next"] == "base":   # aggregates of base cells: one entry per fine row
            add("restriction", l, nxt["n_b"], n, n, k, cg_iters)
            add("prolongation", l, n, nxt["n_b"], n, k, cg_iters)
        else:                      # plane pairs merged: one entry per fine row and plane pair
            add("restriction (planes)", l, n, n, n, nxt["k"], cg_iters)
            add("prolongation (planes)", l, n, n, n, nxt["k"], cg_iters)
    total = sum(p["calls"] for p in prods)
    for p in prods:
        p["weight"] = p["calls"] / total
        p["P_ub_eq3a"] = p_ub_eq3a(p["nnz"], p["n_r"], p["n_c"], p["m"])
        p["intensity_eq2"] = ai_eq2(p["nnz"], p["n_r"], p["n_c"], p["m"])
        p["oc"] = (2 * p["nnz"] + 1) * p["m"]
    timed = [p for p in prods if p["t_us"]]
    wt = sum(p["weight"] for p in timed)
    return {"products": prods,
            "P_ub_weighted": sum(p["weight"] * p["P_ub_eq3a"] for p in prods),
            "intensity_weighted": sum(p["weight"] * p["intensity_eq2"] for p in prods),
            "pi_spmm_gflops": sum(p["weight"] / wt * p["oc"] / (p["t_us"] * 1e-6) for p in timed) / 1e9,
            "timed_weight": wt}


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
            fvx.copy_many(Y, X, nbytes)
            tc = Timer(torch)
            with tc:
                for _ in range(2):
                    fvx.copy_many(Y, X, nbytes)
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


def batch_leg(fvx, inputs, torch, np, rtol, launch_only=False):
    """24 uneven problems (4 channel bases x k in {4..128}) solved together in
    mixed precision to rtol, against the same problems solved one by one and
    against plain FP64 SpMV-CG on their assembled matrices; the batch launched
    phase by phase and replayed from graphs (launch_only: that comparison
    alone)."""
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
    modes = launch_modes(fvx, torch, lambda lm: fvx.solve_batch(opl, Bs, rtol=rtol, precision=fvx.MIXED, launch=lm))
    log(f"batch launch modes: phases {modes['phases']['s']:.3f} s, graph {modes['graph']['s']:.3f} s "
        f"(first {modes['graph']['first_s']:.3f} s)")
    if launch_only:
        return modes
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
    # Error of every mixed result against its FP64 solution to 1e-13 (the
    # batched FP64 CG), beside kappa_est (relres + relres*).
    Xstar, sstar = fvx.solve_batch(opl, Bs, rtol=1e-13)
    perr = []
    for op, X, st, Xs, ss in zip(opl, Xs, sts, Xstar, sstar):
        m = min(max(ss["iters"], 50), 2000)
        kap = lanczos_kappa(op, inputs, torch, m)[0]
        perr.append({"rel_err_vs_fp64": rel_err(torch, op, X, Xs), "kappa_est": kap, "lanczos_steps": m,
                     "bound_kappa": kap * (st["relres_true"] + ss["relres_true"])})
    log("batch mixed vs FP64 x*: max rel err {:.2e}, max err/bound {:.3f}".format(
        max(e["rel_err_vs_fp64"] for e in perr), max(e["rel_err_vs_fp64"] / e["bound_kappa"] for e in perr)))
    # The same batch with the Chebyshev preconditioner (degree 8 on [2/300, 2]).
    kwc = dict(rtol=rtol, precision=fvx.MIXED, precond=fvx.PRECOND_CHEBYSHEV)
    fvx.solve_batch(opl, Bs, **kwc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stc = fvx.solve_batch(opl, Bs, **kwc)
    batch_cheb_s = time.perf_counter() - t0
    out = {
        "batch_chebyshev_s": batch_cheb_s,
        "launch_modes": modes,
        "max_relres_true_chebyshev": max(s["relres_true"] for s in stc),
        "problems": [{"base": f"{p['base'].nx}x{p['base'].ny}", "k": p["k"], "cells": o.n_b * o.k,
                      "tile_f64": list(t[0]), "tile_f32": list(t[1]), "cg_tile_f64": list(t[2]),
                      "cg_tile_f32": list(t[3]), "inner_iters": s["iters"],
                      "outer": s["outer"], "relres_true": s["relres_true"], "single_s": ts, "csr3d_fp64_s": tc,
                      **e}
                     for p, o, t, s, ts, tc, e in zip(probs, opl, tiles, sts, singles, csr, perr)],
        "max_rel_err_vs_fp64": max(e["rel_err_vs_fp64"] for e in perr),
        "max_err_over_bound": max(e["rel_err_vs_fp64"] / e["bound_kappa"] for e in perr),
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
    k, dz = inputs.AIRFOIL_K, inputs.AIRFOIL_DZ

    def spmm(op):
        out = {}
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
            out[f"spmm_{name}"] = {"tile": list(tile), "us": t * 1e3, "GBs": Bk / (t * 1e-3) / 1e9,
                                   "frac_hbm": Bk / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}
            del X, Y
        return out

    # The triangles in the generator's (Qhull's) order, then renumbered along
    # a Hilbert curve of their centroids (the layout the solves use).
    op = fvx.Operator(fvx.Mesh.from_spec(spec), k, dz, fvx.PERIODIC_Z, with_f32=True)
    as_generated = spmm(op)
    del op
    torch.cuda.empty_cache()
    mesh = fvx.Mesh.from_spec(spec, order="hilbert")
    op = fvx.Operator(mesh, k, dz, fvx.PERIODIC_Z, with_f32=True)
    res = {"cells_base": op.n_b, "k": k, "cells": op.n_b * k, "nnz_b": op.nnz_b, "cell_order": "hilbert"}
    res.update(spmm(op))
    res["as_generated_order"] = as_generated
    log(f"airfoil SpMM FP64: {res['spmm_f64']['us']:.2f} us in Hilbert order, "
        f"{as_generated['spmm_f64']['us']:.2f} us in the generator's order")
    res["cg_tile_f64"], res["cg_tile_f32"] = list(tune_cg(op, fvx)), list(tune_cg(op, fvx, fvx.F32))
    B = op.to_rows(inputs.rhs_uniform(3, op.n_b * k))
    cheb = fvx.PRECOND_CHEBYSHEV
    t0 = time.perf_counter()
    amg = fvx.Amg(op)
    res["amg_setup_s"] = time.perf_counter() - t0
    res["amg_levels"] = amg.levels()
    res["amg_coarsest_modes"] = amg.coarsest_modes
    mixed = {}
    for prec, pre, name in ((fvx.MIXED, 0, "mixed"), (fvx.F64, 0, "f64"), (fvx.MIXED, cheb, "mixed_chebyshev"),
                            (fvx.F64, cheb, "f64_chebyshev"), (fvx.MIXED, amg, "mixed_amg"), (fvx.F64, amg, "f64_amg")):
        kw = dict(amg=pre) if isinstance(pre, fvx.Amg) else dict(precond=pre)
        op.solve(B, rtol=rtol, precision=prec, **kw)
        t0 = time.perf_counter()
        X, st = op.solve(B, rtol=rtol, precision=prec, **kw)
        res[f"solve_{name}"] = {"s": time.perf_counter() - t0, "iters": st["iters"], "outer": st["outer"],
                                "relres_true": st["relres_true"]}
        if prec == fvx.MIXED:
            mixed[name] = (X, st)
    # error of each mixed solve against the FP64 solution to 1e-13 (multigrid PCG)
    errs, _ = mixed_errors(fvx, inputs, torch, op, B, mixed, steps=3000, star_kw=dict(amg=amg))
    for name in mixed:
        res[f"solve_{name}"].update(errs[name])
    res["kappa_est"], res["lanczos_steps"], res["x_star"] = errs["kappa_est"], errs["lanczos_steps"], errs["x_star"]
    log(f"airfoil mixed vs FP64 x*: " + ", ".join(f"{n} {errs[n]['rel_err_vs_fp64']:.2e} (bound "
                                                  f"{errs[n]['bound_kappa']:.2e})" for n in mixed))
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
