// Autotuner for the SpMM launch tile: times candidate tiles of the Laplacian
// SpMM on the device (HIP events around a sweep over rotating input/output
// pairs) and keeps the fastest, in two stages: the row mapping first, then
// the launch options around it.  All candidates compute the same product;
// the choice only affects speed.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace fvx {
namespace {

// Stage 1: the row mapping (vector width, lanes per row, block size) with
// the launch options at their defaults.
std::vector<fvx_tile> shape_candidates(const fvx_op *op, int dtype) {
    std::vector<fvx_tile> out;
    const int vmax = dtype == FVX_F32 ? 4 : 2;
    for (int vec = vmax; vec >= 1; vec >>= 1) {
        if (op->ld % vec) continue;
        if (op->stencil != 7 && op->k % vec) continue;
        const int base = std::min(64, next_pow2(int(ceil_div(op->k, vec))));
        for (int lpr = base; lpr >= 1 && lpr >= base / 4; lpr >>= 1)
            for (int block : {64, 128, 256, 512}) {
                if (block < lpr) continue;
                if (op->stencil != 7) {  // structured: one pass, or exactly 2 or 4
                    const int span = lpr * vec;
                    if (!(span >= op->k || (span >= 2 && (op->k == 2 * span || op->k == 4 * span)))) continue;
                }
                out.push_back(fvx_tile{vec, lpr, block, 1, 0, 0, 0});
            }
    }
    return out;
}

// Stage 2: the launch options (grid cap, XCD remap, LDS staging of the row
// metadata, non-temporal stores) around the best row mapping.
std::vector<fvx_tile> option_candidates(const fvx_op *op, const fvx_tile &b) {
    std::vector<fvx_tile> out;
    for (int cap : {0, 1024, 2048})
        for (int remap : {1, 0})
            for (int stage : {0, 1}) {
                if (stage && (b.block / b.lanes_per_row > kMaxStageRows || op->stencil != 7)) continue;
                for (int nt : {0, 1}) {
                    if (cap == 0 && remap == 1 && stage == 0 && nt == 0) continue;  // timed in stage 1
                    out.push_back(fvx_tile{b.vec, b.lanes_per_row, b.block, remap, cap, stage, nt});
                }
            }
    // A Cartesian base whose k columns one row group covers: the cap sets the
    // grid lines per row group, whose best workgroup differs from the
    // one-line kernel's (few workgroups of 64 threads leave a capped grid
    // unbalanced), so the caps are also timed at the other workgroup sizes.
    if (op->d64.cart && b.lanes_per_row * b.vec == op->k && b.lanes_per_row >= 8)
        for (int block : {128, 256, 512}) {
            if (block == b.block || block < b.lanes_per_row) continue;
            for (int cap : {1024, 2048})
                for (int remap : {1, 0})
                    for (int nt : {0, 1}) out.push_back(fvx_tile{b.vec, b.lanes_per_row, block, remap, cap, 0, nt});
        }
    return out;
}

// Structured operators stored in direction order: the line tiles (64 lanes
// over k = 64 vec in one pass, a workgroup cap selecting 2, 4 or 8 grid lines
// per wavefront) at every workgroup size, whatever the best row mapping of
// stage 1.
std::vector<fvx_tile> stencil_line_candidates(const fvx_op *op, int dtype) {
    std::vector<fvx_tile> out;
    const int vec = op->k / 64;
    const int vmax = dtype == FVX_F32 ? 4 : 2;
    if (!op->stencil_dir || op->k % 64 || vec < 1 || vec > vmax || (vec & (vec - 1)) || op->ld % vec) return out;
    for (int block : {64, 128, 256, 512})
        for (int cap : {256, 512, 1024, 2048})
            for (int remap : {1, 0})
                for (int nt : {0, 1}) out.push_back(fvx_tile{vec, 64, block, remap, cap, 0, nt});
    return out;
}

template <typename T>
double time_tile(fvx_op *op, int dtype, const fvx_tile &t, T *buf, int pairs, size_t nv, int reps, hipStream_t s,
                 hipEvent_t e0, hipEvent_t e1) {
    op->tile[dtype] = t;
    auto sweep = [&] {
        for (int i = 0; i < pairs; ++i) launch_lap<T>(op, buf + 2 * i * nv, buf + (2 * i + 1) * nv, nullptr, s);
    };
    sweep();  // warm-up: code object load, first-touch
    FVX_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) sweep();
    FVX_HIP(hipEventRecord(e1, s));
    FVX_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    FVX_HIP(hipEventElapsedTime(&ms, e0, e1));
    return 1e3 * double(ms) / double(reps * pairs);
}

}  // namespace
}  // namespace fvx

extern "C" int fvx_tune(fvx_op *op, int dtype, void *scratch, size_t scratch_bytes, int reps, void *stream,
                        fvx_tune_result *results, int max_results, int *n_results) {
    return fvx::guard([&] {
        FVX_REQUIRE(op && scratch, FVX_E_ARG, "NULL op or scratch");
        FVX_REQUIRE(dtype == FVX_F64 || (dtype == FVX_F32 && op->has_f32), FVX_E_ARG, "bad dtype for this op");
        FVX_REQUIRE(reinterpret_cast<uintptr_t>(scratch) % 16 == 0, FVX_E_ARG, "scratch must be 16-byte aligned");
        const size_t es = dtype == FVX_F64 ? 8 : 4;
        const size_t nv = size_t(op->n_b) * op->ld;
        const size_t pair_bytes = 2 * nv * es;
        FVX_REQUIRE(scratch_bytes >= pair_bytes, FVX_E_NOMEM, "scratch holds no input/output pair");
        // Enough pairs that a sweep streams from HBM for large operators; a
        // few hundred launches for small ones (whose data stay in cache in use).
        const int pairs = int(std::min<size_t>(scratch_bytes / pair_bytes, 512));
        reps = std::max(1, reps);
        hipStream_t s = fvx::as_stream(stream);
        // Inputs: zero-filled scratch is a valid, finite multivector.
        FVX_HIP(hipMemsetAsync(scratch, 0, size_t(pairs) * pair_bytes, s));
        hipEvent_t e0, e1;
        FVX_HIP(hipEventCreate(&e0));
        FVX_HIP(hipEventCreate(&e1));
        const fvx_tile keep = op->tile[dtype];
        fvx_tile best = keep;
        double best_us = 1e30;
        int n = 0;
        auto try_all = [&](const std::vector<fvx_tile> &cands) {
            for (const fvx_tile &t : cands) {
                const double us = dtype == FVX_F64
                                      ? fvx::time_tile<double>(op, dtype, t, static_cast<double *>(scratch), pairs, nv,
                                                               reps, s, e0, e1)
                                      : fvx::time_tile<float>(op, dtype, t, static_cast<float *>(scratch), pairs, nv,
                                                              reps, s, e0, e1);
                if (results && n < max_results) results[n] = fvx_tune_result{t, us};
                ++n;
                if (us < best_us) {
                    best_us = us;
                    best = t;
                }
            }
        };
        try {
            try_all(fvx::shape_candidates(op, dtype));
            try_all(fvx::option_candidates(op, best));
            try_all(fvx::stencil_line_candidates(op, dtype));
        } catch (...) {
            op->tile[dtype] = keep;
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            throw;
        }
        op->tile[dtype] = best;
        if (n_results) *n_results = n;
        FVX_HIP(hipEventDestroy(e0));
        FVX_HIP(hipEventDestroy(e1));
        return FVX_OK;
    });
}
