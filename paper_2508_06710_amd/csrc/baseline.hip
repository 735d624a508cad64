// Comparators for measurement: the assembled 3D CSR SpMV (no block reuse;
// a group of lanes per row sized to the mean row length) and the textbook FP64 SpMV-CG built from it
// with separate SpMV, dot, axpy and xpay kernels; plus a streaming copy
// kernel that measures the achievable HBM bandwidth.
#include <chrono>
#include <cmath>

#include "cg_common.h"

namespace fvx {
namespace {

constexpr int kFlatBlock = 256;
constexpr int kFlatMaxBlocks = 1024;

struct Flat {
    int64_t n, per_block;
};

Flat flat(int64_t n) {
    const int64_t nb = std::min<int64_t>(kFlatMaxBlocks, std::max<int64_t>(1, ceil_div(n, kFlatBlock * 4)));
    Flat f;
    f.n = n;
    f.per_block = ceil_div(n, nb);
    return f;
}

int flat_blocks(const Flat &f) { return int(ceil_div(f.n, f.per_block)); }

#define FLAT_RANGE                                                  \
    const int64_t i0 = int64_t(blockIdx.x) * f.per_block;           \
    const int64_t i1 = min(f.n, i0 + f.per_block);

__global__ __launch_bounds__(kFlatBlock) void k_csr_spmv(int64_t n, const int32_t *__restrict__ ptr,
                                                         const int32_t *__restrict__ col,
                                                         const double *__restrict__ val,
                                                         const double *__restrict__ x, double *__restrict__ y,
                                                         const int32_t *__restrict__ done) {
    if (done && *done) return;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        double s = 0.0;
        for (int32_t j = ptr[i]; j < ptr[i + 1]; ++j) s += val[j] * x[col[j]];
        y[i] = s;
    }
}

// CSR-vector SpMV: G lanes per row stride over its nonzeros and reduce by
// shuffles (G about the mean row length), so that the loads of one row are
// contiguous across lanes.
template <int G>
__global__ __launch_bounds__(kFlatBlock) void k_csr_spmv_vec(int64_t n, const int32_t *__restrict__ ptr,
                                                             const int32_t *__restrict__ col,
                                                             const double *__restrict__ val,
                                                             const double *__restrict__ x, double *__restrict__ y,
                                                             const int32_t *__restrict__ done) {
    if (done && *done) return;
    const int lane = threadIdx.x & (G - 1);
    const int64_t per_block = kFlatBlock / G;
    for (int64_t i = blockIdx.x * per_block + threadIdx.x / G; i < n; i += int64_t(gridDim.x) * per_block) {
        double s = 0.0;
        const int32_t j1 = ptr[i + 1];
        for (int32_t j = ptr[i] + lane; j < j1; j += G) s += val[j] * x[col[j]];
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
        if (lane == 0) y[i] = s;
    }
}

// The comparator keeps the textbook structure: each dot product is its own
// kernel writing per-block partials, and the kernel that needs the scalar sums
// them in its prologue (every block, fixed order).  rho is double-buffered by
// iteration parity as in the SpMM solver.
__device__ inline void flat_partial(double v, Flat f, double *part, double *lds) {
    (void)f;
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int w = 0; w < int(blockDim.x) / 64; ++w) a += lds[w];
        part[blockIdx.x] = a;
    }
}

__global__ __launch_bounds__(kFlatBlock) void k_b_dot(Flat f, CgDev d, const double *__restrict__ u,
                                                      const double *__restrict__ v, double *__restrict__ part) {
    if (d.st->done) return;
    __shared__ double lds[4];
    FLAT_RANGE
    double c = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) c += u[i] * v[i];
    flat_partial(c, f, part, lds);
}

// y += alpha x with alpha = rho / (-p.q) from the p.q partials; `sign`
// selects x (alpha) or r (alpha, q = L p = -A p).
__global__ __launch_bounds__(kFlatBlock) void k_b_axpy(Flat f, CgDev d, int it, int nblk, double *__restrict__ y,
                                                       const double *__restrict__ x, int first) {
    if (d.st->done) return;
    __shared__ double lds[4];
    __shared__ double tot[1];
    sum_partials(d.part_a, nblk, 1, lds, tot);
    const int slot = (it + 1) & 1;
    const double pap = -tot[0];
    if (!(pap > 0.0) || !isfinite(pap)) {
        if (first && blockIdx.x == 0 && threadIdx.x == 0) {
            d.st->done = 1;
            d.st->status = isfinite(pap) ? FVX_E_BREAKDOWN : FVX_E_NONFINITE;
        }
        return;
    }
    const double a = d.rho[slot] / pap;
    if (first && blockIdx.x == 0 && threadIdx.x == 0) d.alpha[0] = a;
    FLAT_RANGE
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) y[i] += a * x[i];
}

// rho' from the r.r partials; convergence; p = r + beta p.
__global__ __launch_bounds__(kFlatBlock) void k_b_xpay(Flat f, CgDev d, int it, int nblk, double *__restrict__ p,
                                                       const double *__restrict__ r) {
    if (d.st->done) return;
    __shared__ double lds[4];
    __shared__ double tot[1];
    sum_partials(d.part_b, nblk, 1, lds, tot);
    const double rn = tot[0], ro = d.rho[(it + 1) & 1];
    const bool conv = rn <= d.rtol2 * d.bnorm2[0];
    const bool cap = it + 1 >= d.st->max_iter;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        d.rho[it & 1] = rn;
        d.rho_last[0] = rn;
        d.iters[0] = it + 1;
        d.st->iter = it + 1;
        if (!isfinite(rn)) {
            d.st->done = 1;
            d.st->status = FVX_E_NONFINITE;
        } else if (conv) {
            d.st->done = 1;
        } else if (cap) {
            d.st->done = 1;
            d.st->status = FVX_NOT_CONVERGED;
        }
    }
    if (conv || cap || !isfinite(rn)) return;
    const double b = rn / ro;
    FLAT_RANGE
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) p[i] = r[i] + b * p[i];
}

__global__ __launch_bounds__(kFlatBlock) void k_b_sum(Flat f, CgDev d, const double *__restrict__ v,
                                                      double *__restrict__ part) {
    __shared__ double lds[4];
    FLAT_RANGE
    double c = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) c += v[i];
    flat_partial(c, f, part, lds);
}

__global__ __launch_bounds__(kFlatBlock) void k_b_init(Flat f, CgDev d, int nblk, int singular,
                                                       const double *__restrict__ b, double *__restrict__ bp,
                                                       double *__restrict__ x, double *__restrict__ r,
                                                       double *__restrict__ p, const double *__restrict__ q,
                                                       int given) {
    __shared__ double lds[4];
    __shared__ double tot[1];
    double m = 0.0;
    if (singular) {
        sum_partials(d.part_a, nblk, 1, lds, tot);
        m = tot[0] / double(f.n);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (!isfinite(m)) {
                d.st->status = FVX_E_NONFINITE;
                d.st->done = 1;
            }
            if (m != 0.0) d.st->rhs_projected = 1;
        }
    }
    FLAT_RANGE
    double c0 = 0.0, c1 = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const double bv = b[i] - m;
        const double rv = given ? q[i] - bv : -bv;
        bp[i] = bv;
        r[i] = rv;
        p[i] = rv;
        if (!given) x[i] = 0.0;
        c0 += rv * rv;
        c1 += bv * bv;
    }
    flat_partial(c0, f, d.part_b, lds);
    __syncthreads();
    flat_partial(c1, f, d.part_b + nblk, lds);
}

// One block: rho_0, ||b||^2 and the initial convergence test.
__global__ __launch_bounds__(kFlatBlock) void k_b_check0(CgDev d, int nblk) {
    __shared__ double lds[4];
    __shared__ double tot[1];
    __shared__ double tb[1];
    sum_partials(d.part_b, nblk, 1, lds, tot);
    sum_partials(d.part_b + nblk, nblk, 1, lds, tb);
    if (threadIdx.x == 0) {
        const double rr = tot[0], bb = tb[0];
        d.rho[1] = rr;
        d.r0[0] = rr;
        d.rho_last[0] = rr;
        d.bnorm2[0] = bb;
        d.iters[0] = 0;
        if (!isfinite(rr) || !isfinite(bb)) {
            d.st->status = FVX_E_NONFINITE;
            d.st->done = 1;
        } else if (!(bb > 0.0 && rr > d.rtol2 * bb)) {
            d.st->done = 1;
        }
    }
}

__global__ __launch_bounds__(kFlatBlock) void k_b_fix_x(Flat f, CgDev d, int nblk, double *__restrict__ x,
                                                        int project) {
    __shared__ double lds[4];
    __shared__ double tot[1];
    double m = 0.0;
    if (project) {
        sum_partials(d.part_a, nblk, 1, lds, tot);
        m = tot[0] / double(f.n);
    }
    const bool zero = d.bnorm2[0] == 0.0;
    FLAT_RANGE
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) x[i] = zero ? 0.0 : x[i] - m;
}

__global__ __launch_bounds__(kFlatBlock) void k_b_resid(Flat f, CgDev d, const double *__restrict__ bp,
                                                        const double *__restrict__ q) {
    __shared__ double lds[4];
    FLAT_RANGE
    double c = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const double e = bp[i] - q[i];
        c += e * e;
    }
    flat_partial(c, f, d.part_b, lds);
}

// Streaming copy: per trip a block moves one contiguous chunk of
// kCopyUnroll * kFlatBlock 16-byte words (16 KiB), each lane holding
// kCopyUnroll independent non-temporal loads in flight before its stores;
// chunks are dealt to blocks in a grid-stride loop.  Contiguous chunks per
// block keep the DRAM pages each block opens local, which measured faster on
// gfx950 than spreading a block's loads over the whole buffer (grid-stride
// per lane) at every size from 17 MB to 1 GiB.
constexpr int kCopyUnroll = 4;
using u32x4 = uint32_t __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kFlatBlock) void k_copy(int64_t n16, const u32x4 *__restrict__ src,
                                                     u32x4 *__restrict__ dst) {
    constexpr int64_t chunk = int64_t(kCopyUnroll) * kFlatBlock;
    for (int64_t c = int64_t(blockIdx.x) * chunk; c < n16; c += int64_t(gridDim.x) * chunk) {
        if (c + chunk <= n16) {
            u32x4 v[kCopyUnroll];
#pragma unroll
            for (int u = 0; u < kCopyUnroll; ++u)
                v[u] = __builtin_nontemporal_load(src + c + u * kFlatBlock + threadIdx.x);
#pragma unroll
            for (int u = 0; u < kCopyUnroll; ++u)
                __builtin_nontemporal_store(v[u], dst + c + u * kFlatBlock + threadIdx.x);
        } else {
            for (int64_t i = c + threadIdx.x; i < n16; i += kFlatBlock) dst[i] = src[i];
        }
    }
}

struct CsrWs {
    CgDev d;
    double *bp, *r, *p, *q;
    size_t bytes;
};

template <typename T>
T *take(char *base, size_t &off, size_t n) {
    T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
    off += (sizeof(T) * n + 255) / 256 * 256;
    return p;
}

CsrWs carve_csr(void *ws, int64_t n) {
    char *b = static_cast<char *>(ws);
    size_t off = 0;
    CsrWs w{};
    w.d.st = take<CgState>(b, off, 1);
    w.d.rho = take<double>(b, off, 2);
    w.d.active = take<int32_t>(b, off, 2);
    w.d.alpha = take<double>(b, off, 1);
    w.d.bnorm2 = take<double>(b, off, 1);
    w.d.r0 = take<double>(b, off, 1);
    w.d.rho_last = take<double>(b, off, 1);
    w.d.iters = take<int32_t>(b, off, 1);
    w.d.part_a = take<double>(b, off, 2 * kFlatMaxBlocks);
    w.d.part_b = take<double>(b, off, 2 * kFlatMaxBlocks);
    w.d.tot = take<double>(b, off, 4);
    w.d.mean = take<double>(b, off, 1);
    w.d.G = 1;
    w.d.percol = 0;
    w.d.count = n;
    w.bp = take<double>(b, off, n);
    w.r = take<double>(b, off, n);
    w.p = take<double>(b, off, n);
    w.q = take<double>(b, off, n);
    w.bytes = off;
    return w;
}

int spmv_blocks(int64_t n) { return int(std::min<int64_t>(65536, std::max<int64_t>(1, ceil_div(n, kFlatBlock)))); }

// Lanes per row of the CSR SpMV: the mean row length rounded up to a power of
// two (1 = the row-per-thread kernel).
int csr_lanes(int64_t n, int64_t nnz) {
    const int64_t mean = n > 0 ? ceil_div(std::max<int64_t>(nnz, 1), n) : 1;
    int g = 1;
    while (g < mean && g < 64) g <<= 1;
    return g <= 2 ? 1 : g;
}

void launch_csr_spmv(int g, int64_t n, const int32_t *ptr, const int32_t *col, const double *val, const double *x,
                     double *y, const int32_t *done, hipStream_t s) {
    const dim3 block(kFlatBlock);
    auto go = [&](auto Gt) {
        constexpr int G = decltype(Gt)::value;
        const int64_t nb = std::min<int64_t>(1 << 20, std::max<int64_t>(1, ceil_div(n * G, kFlatBlock)));
        hipLaunchKernelGGL(k_csr_spmv_vec<G>, dim3(int(nb)), block, 0, s, n, ptr, col, val, x, y, done);
    };
    switch (g) {
    case 4: go(std::integral_constant<int, 4>{}); break;
    case 8: go(std::integral_constant<int, 8>{}); break;
    case 16: go(std::integral_constant<int, 16>{}); break;
    case 32: go(std::integral_constant<int, 32>{}); break;
    case 64: go(std::integral_constant<int, 64>{}); break;
    default: hipLaunchKernelGGL(k_csr_spmv, dim3(spmv_blocks(n)), block, 0, s, n, ptr, col, val, x, y, done);
    }
}

}  // namespace
}  // namespace fvx

using fvx::guard;

extern "C" {

int fvx_csr_spmv(int64_t n_rows, int64_t nnz, const int32_t *ptr, const int32_t *col, const double *val,
                 const double *x, double *y, void *stream) {
    return guard([&] {
        FVX_REQUIRE(n_rows >= 0 && nnz >= 0 && ptr && col && val && x && y, FVX_E_ARG, "NULL argument");
        if (n_rows == 0) return FVX_OK;
        fvx::launch_csr_spmv(fvx::csr_lanes(n_rows, nnz), n_rows, ptr, col, val, x, y, nullptr,
                             fvx::as_stream(stream));
        FVX_HIP(hipGetLastError());
        return FVX_OK;
    });
}

int fvx_csr_solve_bytes(int64_t n_rows, size_t *bytes) {
    return guard([&] {
        FVX_REQUIRE(n_rows >= 1 && bytes, FVX_E_ARG, "bad argument");
        *bytes = fvx::carve_csr(nullptr, n_rows).bytes;
        return FVX_OK;
    });
}

int fvx_csr_poisson_solve(int64_t n, int64_t nnz, const int32_t *ptr, const int32_t *col, const double *val,
                          const double *B, double *X, int singular, const fvx_solve_opts *o, void *ws,
                          size_t ws_bytes, fvx_solve_stats *stats, void *stream) {
    return guard([&] {
        using namespace fvx;
        const auto t_start = std::chrono::steady_clock::now();
        FVX_REQUIRE(n >= 1 && nnz >= 0 && ptr && col && val && B && X && ws && o, FVX_E_ARG, "NULL argument");
        const int g = csr_lanes(n, nnz);
        FVX_REQUIRE(o->rtol > 0 && o->rtol < 1 && o->max_iter >= 1 && o->poll_every >= 1, FVX_E_ARG, "bad options");
        FVX_REQUIRE(o->precision == FVX_F64, FVX_E_UNSUPPORTED, "the assembled-matrix comparator is FP64 only");
        FVX_REQUIRE(reinterpret_cast<uintptr_t>(ws) % 256 == 0, FVX_E_ARG, "ws must be 256-byte aligned");
        CsrWs w = carve_csr(ws, n);
        FVX_REQUIRE(ws_bytes >= w.bytes, FVX_E_NOMEM, "workspace too small: need " + std::to_string(w.bytes));
        hipStream_t s = as_stream(stream);
        CgDev d = w.d;
        d.rtol2 = o->rtol * o->rtol;
        CgState st0{};
        st0.max_iter = o->max_iter;
        FVX_HIP(hipMemcpyAsync(d.st, &st0, sizeof(CgState), hipMemcpyHostToDevice, s));
        const Flat f = flat(n);
        const int nblk = flat_blocks(f);
        const dim3 grid(nblk), block(kFlatBlock);
        const bool given = o->guess == FVX_GUESS_GIVEN;
        if (singular) hipLaunchKernelGGL(k_b_sum, grid, block, 0, s, f, d, B, d.part_a);
        if (given) launch_csr_spmv(g, n, ptr, col, val, X, w.q, nullptr, s);
        hipLaunchKernelGGL(k_b_init, grid, block, 0, s, f, d, nblk, singular, B, w.bp, X, w.r, w.p, w.q, int(given));
        hipLaunchKernelGGL(k_b_check0, dim3(1), block, 0, s, d, nblk);
        FVX_HIP(hipGetLastError());
        int it = 0;
        int32_t done = 0;
        while (true) {
            const int batch = std::min(o->poll_every, std::max(1, o->max_iter - it));
            for (int i = 0; i < batch; ++i, ++it) {
                launch_csr_spmv(g, n, ptr, col, val, w.p, w.q, &d.st->done, s);
                hipLaunchKernelGGL(k_b_dot, grid, block, 0, s, f, d, w.p, w.q, d.part_a);
                hipLaunchKernelGGL(k_b_axpy, grid, block, 0, s, f, d, it, nblk, X, w.p, 1);
                hipLaunchKernelGGL(k_b_axpy, grid, block, 0, s, f, d, it, nblk, w.r, w.q, 0);
                hipLaunchKernelGGL(k_b_dot, grid, block, 0, s, f, d, w.r, w.r, d.part_b);
                hipLaunchKernelGGL(k_b_xpay, grid, block, 0, s, f, d, it, nblk, w.p, w.r);
            }
            FVX_HIP(hipGetLastError());
            FVX_HIP(hipMemcpyAsync(&done, &d.st->done, 4, hipMemcpyDeviceToHost, s));
            FVX_HIP(hipStreamSynchronize(s));
            if (done || it >= o->max_iter + 1) break;
        }
        CgState st;
        double rho = 0, r0 = 0, bb = 0;
        int32_t its = 0;
        FVX_HIP(hipMemcpyAsync(&st, d.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        FVX_HIP(hipMemcpyAsync(&rho, d.rho_last, 8, hipMemcpyDeviceToHost, s));
        FVX_HIP(hipMemcpyAsync(&r0, d.r0, 8, hipMemcpyDeviceToHost, s));
        FVX_HIP(hipMemcpyAsync(&bb, d.bnorm2, 8, hipMemcpyDeviceToHost, s));
        FVX_HIP(hipMemcpyAsync(&its, d.iters, 4, hipMemcpyDeviceToHost, s));
        if (singular) hipLaunchKernelGGL(k_b_sum, grid, block, 0, s, f, d, X, d.part_a);
        hipLaunchKernelGGL(k_b_fix_x, grid, block, 0, s, f, d, nblk, X, singular);
        launch_csr_spmv(g, n, ptr, col, val, X, w.q, nullptr, s);
        hipLaunchKernelGGL(k_b_resid, grid, block, 0, s, f, d, w.bp, w.q);
        FVX_HIP(hipGetLastError());
        std::vector<double> part(nblk);
        FVX_HIP(hipMemcpyAsync(part.data(), d.part_b, 8 * nblk, hipMemcpyDeviceToHost, s));
        FVX_HIP(hipStreamSynchronize(s));
        double res2 = 0.0;
        for (double v : part) res2 += v;
        const int status = st.status;
        if (stats) {
            *stats = fvx_solve_stats{};
            stats->status = status;
            stats->iters = its;
            stats->rhs_projected = st.rhs_projected;
            stats->relres_rec = bb > 0 ? std::sqrt(rho / bb) : 0.0;
            stats->relres_true = bb > 0 ? std::sqrt(res2 / bb) : 0.0;
            stats->r0_over_b = bb > 0 ? std::sqrt(r0 / bb) : 0.0;
            stats->bnorm = std::sqrt(bb);
            stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        }
        if (status < 0) throw Error(status, fvx_status_str(status));
        return status;
    });
}

int fvx_copy(void *dst, const void *src, size_t bytes, void *stream) {
    return guard([&] {
        FVX_REQUIRE(dst && src, FVX_E_ARG, "NULL buffer");
        FVX_REQUIRE(bytes % 16 == 0 && reinterpret_cast<uintptr_t>(dst) % 16 == 0 &&
                        reinterpret_cast<uintptr_t>(src) % 16 == 0,
                    FVX_E_ARG, "copy needs 16-byte aligned buffers and sizes");
        const int64_t n16 = int64_t(bytes / 16);
        if (n16 == 0) return FVX_OK;
        // one chunk per block up to 8192 blocks (32 per CU), then grid-stride
        const int64_t nb = std::min<int64_t>(8192, fvx::ceil_div(n16, int64_t(fvx::kCopyUnroll) * fvx::kFlatBlock));
        hipLaunchKernelGGL(fvx::k_copy, dim3(int(nb)), dim3(fvx::kFlatBlock), 0, fvx::as_stream(stream), n16,
                           static_cast<const fvx::u32x4 *>(src), static_cast<fvx::u32x4 *>(dst));
        FVX_HIP(hipGetLastError());
        return FVX_OK;
    });
}

int fvx_copy_many(int n, void *const *dst, const void *const *src, size_t bytes, void *stream) {
    return guard([&]() -> int {
        FVX_REQUIRE(n >= 0 && (n == 0 || (dst && src)), FVX_E_ARG, "bad pointer arrays");
        for (int i = 0; i < n; ++i) {
            const int rc = fvx_copy(dst[i], src[i], bytes, stream);
            if (rc != FVX_OK) return rc;
        }
        return FVX_OK;
    });
}

}  // extern "C"
