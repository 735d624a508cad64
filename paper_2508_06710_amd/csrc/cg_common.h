// Device-side CG state and the deterministic reductions shared by the
// SpMM-based solver and the assembled-matrix comparator.
//
// No kernel waits on another block of the same grid: a kernel writes one
// partial sum per block (and per group), and the NEXT kernel on the stream
// reduces those partials in its prologue -- every block redundantly, in the
// same fixed order, so every block obtains bit-identical scalars.  Kernel
// boundaries make the partials visible across the XCDs' separate L2 caches
// without grid-wide fences (which on gfx950 write back and invalidate L2).
#pragma once

#include "kernels.h"

namespace fvx {

constexpr int kMaxCgBlock = 512;     // launch bound of the CG kernels
constexpr int kMaxPercolBlock = 256;  // independent planes: per-column partials staged in LDS
constexpr int kMaxV = 4;
constexpr int kMaxGroups = 256;

// iter: the iteration the direction kernel last started (written by its block
// 0, read by the update kernel that follows); next_it: the iteration the next
// direction kernel runs (written by block 0 of the update kernel, 0 after
// reset).  Each is read by a kernel in which no block writes it, so the
// iteration kernels take no iteration argument and every iteration launches
// the same kernels with the same arguments.
struct CgState {
    int32_t done, status, rhs_projected, iter;
    int32_t max_iter, next_it;
    int32_t pad[2];
};

// Per-group scalars.  rho/active are double-buffered by iteration parity: the
// search-direction kernel of iteration `it` reads slot (it-1)&1 (written by
// block 0 of the previous iteration's kernel) and block 0 writes slot it&1.
struct CgDev {
    CgState *st;
    double *rho;       // [2][G]
    int32_t *active;   // [2][G]
    double *alpha;     // [G]  (last alpha, for inspection)
    double *bnorm2;    // [G]
    double *r0;        // [G]
    double *rho_last;  // [G]  residual norm^2 at the last check
    int32_t *iters;    // [G]
    double *part_a;    // [maxb][G]  p.q partials
    double *part_b;    // [2][maxb][G]  r.r (and b.b at start) partials
    double *tot;       // [4][G]  folded totals (independent columns)
    double *mean;      // [G]
    int G;
    int percol;
    double rtol2;
    int64_t count;     // entries per group (for means)
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Writes this block's partial sums of NV quantities: part[q][blk][g].
// c[q][t] is the thread's contribution to quantity q in column c0 + t (one
// pass of the row group covers all columns when percol).
template <int NV, int V>
__device__ void write_partials(const double (&c)[NV][V], int sub, int lpr, int G, int percol, double *part,
                               int64_t blk, int nblk, double *lds) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int q = 0; q < NV; ++q) {
        double *pq = part + int64_t(q) * nblk * G;
        if (percol) {
            const int grp = tid / lpr, wdt = lpr * V, ngrp = nthr / lpr;
#pragma unroll
            for (int t = 0; t < V; ++t) lds[grp * wdt + sub * V + t] = c[q][t];
            __syncthreads();
            for (int g = tid; g < G; g += nthr) {
                double s = 0.0;
                for (int r = 0; r < ngrp; ++r) s += lds[r * wdt + g];
                pq[blk * G + g] = s;
            }
            __syncthreads();
        } else {
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < V; ++t) s += c[q][t];
            s = wave_sum(s);
            if ((tid & 63) == 0) lds[tid >> 6] = s;
            __syncthreads();
            if (tid == 0) {
                double a = 0.0;
                for (int w = 0; w < nthr / 64; ++w) a += lds[w];
                pq[blk] = a;
            }
            __syncthreads();
        }
    }
}

// Sum over n partial rows part[b*G + g] (b = 0..n-1, fixed order) for every
// group; every thread of the block returns with tot[g] filled.
__device__ inline void sum_partials(const double *__restrict__ part, int n, int G, double *lds, double *tot) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    if (G == 1) {
        double a = 0.0;
        for (int b = tid; b < n; b += nthr) a += part[b];
        a = wave_sum(a);
        if ((tid & 63) == 0) lds[tid >> 6] = a;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < nthr / 64; ++w) s += lds[w];
            tot[0] = s;
        }
    } else {
        for (int g = tid; g < G; g += nthr) {
            double s = 0.0;
            for (int b = 0; b < n; ++b) s += part[int64_t(b) * G + g];
            tot[g] = s;
        }
    }
    __syncthreads();
}

// Folds partials [NV][n][G] into totals [NV][G]: block (q, g) sums one column
// of partials in a fixed order (used when the groups are independent columns).
static __global__ __launch_bounds__(256) void k_fold(const double *__restrict__ part, int n, int G,
                                                     double *__restrict__ out) {
    __shared__ double lds[4];
    const int q = blockIdx.x / G, g = blockIdx.x % G;
    const double *p = part + int64_t(q) * n * G;
    double a = 0.0;
    for (int b = threadIdx.x; b < n; b += blockDim.x) a += p[int64_t(b) * G + g];
    a = wave_sum(a);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < int(blockDim.x) / 64; ++w) s += lds[w];
        out[q * G + g] = s;
    }
}

__device__ __forceinline__ int group_of(const CgDev &d, int col) { return d.percol ? col : 0; }

}  // namespace fvx
