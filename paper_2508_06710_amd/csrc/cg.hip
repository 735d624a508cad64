// Conjugate-gradient Poisson solve on the repeated-block Laplacian.
//
// CG runs on the SPD operator A = -L with right-hand side -b.  Each iteration
// is three kernels on the caller's stream:
//   1. q = L p (the SpMM) fused with the partial dot products p.q, finished by
//      the last block to arrive, which forms alpha = rho / (p.Ap);
//   2. x += alpha p, r -= alpha Ap, fused with r.r, finished into beta and
//      the convergence flag;
//   3. p = r + beta p.
// All scalars stay on the device.  Dot products are deterministic: each block
// reduces its rows in a fixed order, writes one partial per group, and the
// last block (ticket counter) adds the partials in block order.  Groups are
// the columns when the planes are independent systems (each column its own
// CG, frozen once converged) or one global group when they are coupled.
// The host polls the device "done" flag every poll_every iterations; kernels
// launched after convergence return at once.
#include <chrono>
#include <cmath>

#include "kernels.h"

namespace fvx {
namespace {

constexpr int kMaxCgBlock = 256;
constexpr int kMaxV = 4;

struct CgState {
    int32_t iter, done, status, rhs_projected;
    uint32_t ticket;
    int32_t max_iter;
    int32_t pad[2];
};

// Per-group scalars plus the reduction partials of one CG instance.
struct CgDev {
    CgState *st;
    double *rho, *alpha, *beta, *bnorm2, *r0, *mean, *relres, *aux;
    int32_t *active, *iters;
    double *part;   // [2][max_blocks][G]
    int G;          // groups: k (independent columns) or 1
    int percol;
    double rtol2;
    int64_t count;  // entries per group (for means)
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-level then grid-level deterministic reduction of NV quantities.
// c[q][t] is this thread's contribution to quantity q in column c0 + t.
// Returns true in the last block to finish, whose shared `tot[q*G + g]` then
// holds the totals.
template <int NV, int V>
__device__ bool reduce_grid(const double (&c)[NV][V], int sub, int lpr, const CgDev &d, int64_t blk,
                            double *lds, double *tot) {
    const int tid = threadIdx.x, nthr = blockDim.x, nblk = gridDim.x;
    const int G = d.G;
    for (int q = 0; q < NV; ++q) {
        double *part = d.part + int64_t(q) * nblk * G;
        if (d.percol) {
            const int grp = tid / lpr, wdt = lpr * V, ngrp = nthr / lpr;
#pragma unroll
            for (int t = 0; t < V; ++t) lds[grp * wdt + sub * V + t] = c[q][t];
            __syncthreads();
            for (int g = tid; g < G; g += nthr) {
                double s = 0.0;
                for (int r = 0; r < ngrp; ++r) s += lds[r * wdt + g];
                part[blk * G + g] = s;
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
                part[blk] = a;
            }
            __syncthreads();
        }
    }
    __shared__ int s_last;
    __threadfence();
    if (tid == 0) s_last = atomicAdd(&d.st->ticket, 1u) == unsigned(nblk - 1);
    __syncthreads();
    if (!s_last) return false;
    __threadfence();
    for (int q = 0; q < NV; ++q) {
        const double *part = d.part + int64_t(q) * nblk * G;
        if (d.percol) {
            for (int g0 = 0; g0 < G; g0 += nthr) {
                const int gc = min(nthr, G - g0);
                const int S = nthr / gc;
                const int g = g0 + tid % gc, s = tid / gc;
                if (s < S) {
                    double a = 0.0;
                    for (int b = s; b < nblk; b += S) a += part[int64_t(b) * G + g];
                    lds[s * gc + tid % gc] = a;
                }
                __syncthreads();
                if (tid < gc) {
                    double a = 0.0;
                    for (int r = 0; r < S; ++r) a += lds[r * gc + tid];
                    tot[q * G + g0 + tid] = a;
                }
                __syncthreads();
            }
        } else {
            double a = 0.0;
            for (int b = tid; b < nblk; b += nthr) a += part[b];
            a = wave_sum(a);
            if ((tid & 63) == 0) lds[tid >> 6] = a;
            __syncthreads();
            if (tid == 0) {
                double s = 0.0;
                for (int w = 0; w < nthr / 64; ++w) s += lds[w];
                tot[q] = s;
            }
            __syncthreads();
        }
    }
    if (tid == 0) atomicExch(&d.st->ticket, 0u);
    return true;
}

__device__ __forceinline__ int group_of(const CgDev &d, int col) { return d.percol ? col : 0; }

// Finishing logic after the p.Lp reduction: alpha per active group.
__device__ void finish_alpha(const CgDev &d, const double *tot) {
    for (int g = threadIdx.x; g < d.G; g += blockDim.x) {
        if (!d.active[g]) {
            d.alpha[g] = 0.0;
            continue;
        }
        const double pap = -tot[g];
        if (!(pap > 0.0) || !isfinite(pap)) {
            d.alpha[g] = 0.0;
            d.active[g] = 0;
            atomicExch(&d.st->status, isfinite(pap) ? int(FVX_E_BREAKDOWN) : int(FVX_E_NONFINITE));
            atomicExch(&d.st->done, 1);
        } else {
            d.alpha[g] = d.rho[g] / pap;
        }
    }
}

// Finishing logic after the r.r reduction: convergence, beta, counters.
__device__ void finish_beta(const CgDev &d, const double *tot) {
    __shared__ int s_any;
    if (threadIdx.x == 0) s_any = 0;
    __syncthreads();
    for (int g = threadIdx.x; g < d.G; g += blockDim.x) {
        if (!d.active[g]) continue;
        const double rn = tot[g];
        d.iters[g] += 1;
        if (!isfinite(rn)) {
            d.active[g] = 0;
            atomicExch(&d.st->status, int(FVX_E_NONFINITE));
            atomicExch(&d.st->done, 1);
            continue;
        }
        d.beta[g] = rn / d.rho[g];
        d.rho[g] = rn;
        if (rn <= d.rtol2 * d.bnorm2[g])
            d.active[g] = 0;
        else
            atomicOr(&s_any, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int it = d.st->iter + 1;
        d.st->iter = it;
        if (!s_any) {
            d.st->done = 1;
        } else if (it >= d.st->max_iter) {
            d.st->done = 1;
            if (d.st->status == 0) d.st->status = FVX_NOT_CONVERGED;
        }
    }
}

#define CG_PROLOGUE                                                         \
    const int lpr = a.lpr;                                                  \
    const int sub = threadIdx.x & (lpr - 1);                                \
    const int grp = threadIdx.x / lpr;                                      \
    const int64_t blk = logical_block(a.remap);                             \
    const int64_t t0 = blk * a.tiles_per_block;                             \
    __shared__ double lds[kMaxCgBlock * kMaxV];                             \
    __shared__ double tot[2 * 256];

// 1. q = L p, partial p.q
template <typename T, int V, bool Z>
__global__ __launch_bounds__(kMaxCgBlock) void k_cg_spmm(RowArgs<T> a, CgDev d, const T *__restrict__ p,
                                                         T *__restrict__ q) {
    if (d.st->done) return;
    CG_PROLOGUE
    const bool single = lpr * V >= a.k;
    double c[1][V] = {};
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
            vec_t<T, V> po;
            const vec_t<T, V> acc = lap_row<T, V, Z>(a.A, p, a.n_b, a.k, a.ld, a.W, row, c0, sub, lpr, single, po);
            stv_masked<T, V>(q + row * a.ld + c0, acc, a.k - c0);
#pragma unroll
            for (int u = 0; u < V; ++u)
                if (c0 + u < a.k) c[0][u] += double(po[u]) * double(acc[u]);
        }
    }
    if (reduce_grid<1, V>(c, sub, lpr, d, blk, lds, tot)) finish_alpha(d, tot);
}

// 2. x += alpha p; r += alpha q (q = L p = -A p); partial r.r
template <typename T, int V>
__global__ __launch_bounds__(kMaxCgBlock) void k_cg_update(RowArgs<T> a, CgDev d, T *__restrict__ x,
                                                           T *__restrict__ r, const T *__restrict__ p,
                                                           const T *__restrict__ q) {
    if (d.st->done) return;
    CG_PROLOGUE
    double c[1][V] = {};
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
            const int64_t o = row * a.ld + c0;
            vec_t<T, V> xv = ldv<T, V>(x + o), rv = ldv<T, V>(r + o);
            const vec_t<T, V> pv = ldv<T, V>(p + o), qv = ldv<T, V>(q + o);
#pragma unroll
            for (int u = 0; u < V; ++u) {
                if (c0 + u >= a.k) continue;
                const T al = T(d.alpha[group_of(d, c0 + u)]);
                xv[u] += al * pv[u];
                rv[u] += al * qv[u];
                c[0][u] += double(rv[u]) * double(rv[u]);
            }
            stv_masked<T, V>(x + o, xv, a.k - c0);
            stv_masked<T, V>(r + o, rv, a.k - c0);
        }
    }
    if (reduce_grid<1, V>(c, sub, lpr, d, blk, lds, tot)) finish_beta(d, tot);
}

// 3. p = r + beta p for groups still iterating
template <typename T, int V>
__global__ __launch_bounds__(kMaxCgBlock) void k_cg_p(RowArgs<T> a, CgDev d, const T *__restrict__ r,
                                                      T *__restrict__ p) {
    if (d.st->done) return;
    CG_PROLOGUE
    (void)lds;
    (void)tot;
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
            const int64_t o = row * a.ld + c0;
            const vec_t<T, V> rv = ldv<T, V>(r + o);
            vec_t<T, V> pv = ldv<T, V>(p + o);
#pragma unroll
            for (int u = 0; u < V; ++u) {
                if (c0 + u >= a.k) continue;
                const int g = group_of(d, c0 + u);
                if (d.active[g]) pv[u] = rv[u] + T(d.beta[g]) * pv[u];
            }
            stv_masked<T, V>(p + o, pv, a.k - c0);
        }
    }
}

// Plain mean per group of a vector (used for zero-mean projections); also
// flags non-finite input.  Result in d.mean (or d.aux when to_aux).
template <typename T, int V>
__global__ __launch_bounds__(kMaxCgBlock) void k_mean(RowArgs<T> a, CgDev d, const T *__restrict__ v,
                                                      int to_aux, int flag_input) {
    CG_PROLOGUE
    double c[1][V] = {};
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
            const vec_t<T, V> vv = ldv<T, V>(v + row * a.ld + c0);
#pragma unroll
            for (int u = 0; u < V; ++u)
                if (c0 + u < a.k) c[0][u] += double(vv[u]);
        }
    }
    if (reduce_grid<1, V>(c, sub, lpr, d, blk, lds, tot)) {
        for (int g = threadIdx.x; g < d.G; g += blockDim.x) {
            const double m = tot[g] / double(d.count);
            (to_aux ? d.aux : d.mean)[g] = m;
            if (flag_input) {
                if (!isfinite(m)) {
                    atomicExch(&d.st->status, int(FVX_E_NONFINITE));
                    atomicExch(&d.st->done, 1);
                }
                if (m != 0.0) atomicExch(&d.st->rhs_projected, 1);
            }
        }
    }
}

// Start of CG: bp = b - mean; r = L x0 - bp (given guess, Lx0 in q) or -bp;
// p = r; x = 0 for the zero guess; reductions bp.bp and r.r.
template <typename T, int V>
__global__ __launch_bounds__(kMaxCgBlock) void k_cg_init(RowArgs<T> a, CgDev d, const T *__restrict__ b,
                                                         T *__restrict__ bp, T *__restrict__ x,
                                                         T *__restrict__ r, T *__restrict__ p,
                                                         const T *__restrict__ q, int given) {
    CG_PROLOGUE
    double c[2][V] = {};
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
            const int64_t o = row * a.ld + c0;
            vec_t<T, V> bv = ldv<T, V>(b + o), rv;
            const vec_t<T, V> qv = given ? ldv<T, V>(q + o) : vec_t<T, V>(0);
#pragma unroll
            for (int u = 0; u < V; ++u) {
                if (c0 + u >= a.k) continue;
                bv[u] = T(double(bv[u]) - d.mean[group_of(d, c0 + u)]);
                rv[u] = given ? qv[u] - bv[u] : -bv[u];
                c[0][u] += double(bv[u]) * double(bv[u]);
                c[1][u] += double(rv[u]) * double(rv[u]);
            }
            stv_masked<T, V>(bp + o, bv, a.k - c0);
            stv_masked<T, V>(r + o, rv, a.k - c0);
            stv_masked<T, V>(p + o, rv, a.k - c0);
            if (!given) stv_masked<T, V>(x + o, vec_t<T, V>(0), a.k - c0);
        }
    }
    if (reduce_grid<2, V>(c, sub, lpr, d, blk, lds, tot)) {
        __shared__ int s_any;
        if (threadIdx.x == 0) s_any = 0;
        __syncthreads();
        for (int g = threadIdx.x; g < d.G; g += blockDim.x) {
            const double bb = tot[g], rr = tot[d.G + g];
            d.bnorm2[g] = bb;
            d.rho[g] = rr;
            d.r0[g] = rr;
            d.iters[g] = 0;
            d.beta[g] = 0.0;
            d.alpha[g] = 0.0;
            if (!isfinite(bb) || !isfinite(rr)) {
                d.active[g] = 0;
                atomicExch(&d.st->status, int(FVX_E_NONFINITE));
                atomicExch(&d.st->done, 1);
            } else {
                const int act = bb > 0.0 && rr > d.rtol2 * bb;
                d.active[g] = act;
                if (act) atomicOr(&s_any, 1);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0 && !s_any) d.st->done = 1;
    }
}

// End of CG: x -= mean(x) (singular L), x = 0 where b vanished.
template <typename T, int V>
__global__ __launch_bounds__(kMaxCgBlock) void k_fix_x(RowArgs<T> a, CgDev d, T *__restrict__ x, int project) {
    CG_PROLOGUE
    (void)lds;
    (void)tot;
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
            vec_t<T, V> xv = ldv<T, V>(x + row * a.ld + c0);
#pragma unroll
            for (int u = 0; u < V; ++u) {
                if (c0 + u >= a.k) continue;
                const int g = group_of(d, c0 + u);
                xv[u] = d.bnorm2[g] == 0.0 ? T(0) : (project ? T(double(xv[u]) - d.aux[g]) : xv[u]);
            }
            stv_masked<T, V>(x + row * a.ld + c0, xv, a.k - c0);
        }
    }
}

// ||bp - q||^2 per group into d.relres (as a relative residual), and
// optionally r = bp - q (the FP64 outer residual of the mixed solve).
template <typename T, int V>
__global__ __launch_bounds__(kMaxCgBlock) void k_resid(RowArgs<T> a, CgDev d, const T *__restrict__ bp,
                                                       const T *__restrict__ q, T *__restrict__ r) {
    CG_PROLOGUE
    double c[1][V] = {};
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
            const int64_t o = row * a.ld + c0;
            const vec_t<T, V> bv = ldv<T, V>(bp + o), qv = ldv<T, V>(q + o);
            const vec_t<T, V> rv = bv - qv;
#pragma unroll
            for (int u = 0; u < V; ++u)
                if (c0 + u < a.k) c[0][u] += double(rv[u]) * double(rv[u]);
            if (r) stv_masked<T, V>(r + o, rv, a.k - c0);
        }
    }
    if (reduce_grid<1, V>(c, sub, lpr, d, blk, lds, tot)) {
        __shared__ int s_any;
        if (threadIdx.x == 0) s_any = 0;
        __syncthreads();
        for (int g = threadIdx.x; g < d.G; g += blockDim.x) {
            const double bb = d.bnorm2[g];
            d.relres[g] = bb > 0.0 ? sqrt(tot[g] / bb) : 0.0;
            d.aux[g] = tot[g];
            if (bb > 0.0 && !(tot[g] <= d.rtol2 * bb)) atomicOr(&s_any, 1);
            if (!isfinite(tot[g])) atomicExch(&d.st->status, int(FVX_E_NONFINITE));
        }
        __syncthreads();
        if (threadIdx.x == 0) d.st->done = !s_any;
    }
}

// Mixed precision: rhs of the inner FP32 solve, b32 = r64 - mean(r64) for
// groups not yet converged (zero for converged ones).
template <int V>
__global__ __launch_bounds__(kMaxCgBlock) void k_to_inner(RowArgs<double> a, CgDev d, const double *__restrict__ r,
                                                          float *__restrict__ b32, int project) {
    CG_PROLOGUE
    (void)lds;
    (void)tot;
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
            const vec_t<double, V> rv = ldv<double, V>(r + row * a.ld + c0);
            vec_t<float, V> o;
#pragma unroll
            for (int u = 0; u < V; ++u) {
                const int g = group_of(d, c0 + u < a.k ? c0 + u : 0);
                const bool conv = d.bnorm2[g] == 0.0 || d.aux[g] <= d.rtol2 * d.bnorm2[g];
                o[u] = conv ? 0.0f : float(project ? rv[u] - d.mean[g] : rv[u]);
            }
            stv_masked<float, V>(b32 + row * a.ld + c0, o, a.k - c0);
        }
    }
}

// Mixed precision: x += d32 in FP64.
template <int V>
__global__ __launch_bounds__(kMaxCgBlock) void k_add_inner(RowArgs<double> a, double *__restrict__ x,
                                                           const float *__restrict__ d32) {
    const int lpr = a.lpr;
    const int sub = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const int64_t t0 = logical_block(a.remap) * a.tiles_per_block;
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
            const int64_t o = row * a.ld + c0;
            vec_t<double, V> xv = ldv<double, V>(x + o);
            const vec_t<float, V> dv = ldv<float, V>(d32 + o);
#pragma unroll
            for (int u = 0; u < V; ++u) xv[u] += double(dv[u]);
            stv_masked<double, V>(x + o, xv, a.k - c0);
        }
    }
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------

struct Carve {
    char *base;
    size_t off = 0, cap;
    template <typename T>
    T *take(size_t n) {
        T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
        off += (sizeof(T) * n + 255) / 256 * 256;
        return p;
    }
};

int groups_of(const fvx_op *op) { return op->percol ? op->k : 1; }

// CG launch tile for precision T: the op's tile, widened so that one pass of
// a row group covers all k columns (per-column reductions need it), with at
// most kMaxCgBlock threads.
template <typename T>
fvx_tile cg_tile(const fvx_op *op) {
    fvx_tile t = op->tile[dtype_of<T>()];
    if (t.lanes_per_row * t.vec < op->k)
        t.lanes_per_row = std::min(64, next_pow2(int(ceil_div(op->k, t.vec))));
    if (op->percol && t.lanes_per_row * t.vec < op->k) {
        const fvx_tile d = default_tile(op, dtype_of<T>());
        t.vec = d.vec;
        t.lanes_per_row = d.lanes_per_row;
    }
    FVX_REQUIRE(!op->percol || t.lanes_per_row * t.vec >= op->k, FVX_E_UNSUPPORTED,
                "independent-plane solve: k exceeds one pass of a row group");
    t.block = std::max(std::min(t.block, kMaxCgBlock), t.lanes_per_row);
    return t;
}

int max_blocks_for(const fvx_op *op) { return op->percol ? 256 : 1024; }

CgDev carve_cg(Carve &c, const fvx_op *op) {
    CgDev d{};
    const int G = groups_of(op);
    d.st = c.take<CgState>(1);
    d.rho = c.take<double>(G);
    d.alpha = c.take<double>(G);
    d.beta = c.take<double>(G);
    d.bnorm2 = c.take<double>(G);
    d.r0 = c.take<double>(G);
    d.mean = c.take<double>(G);
    d.relres = c.take<double>(G);
    d.aux = c.take<double>(G);
    d.active = c.take<int32_t>(G);
    d.iters = c.take<int32_t>(G);
    d.part = c.take<double>(size_t(2) * max_blocks_for(op) * G);
    d.G = G;
    d.percol = op->percol ? 1 : 0;
    d.count = op->percol ? op->n_b : op->n_b * int64_t(op->k);
    return d;
}

struct Workspace {
    CgDev outer, inner;
    double *bp, *r, *p, *q;       // FP64 solve vectors (bp, r also used by the outer loop)
    float *b32, *x32, *bp32, *r32, *p32, *q32;
    size_t bytes;
};

Workspace carve(void *ws, const fvx_op *op, bool mixed) {
    Carve c{static_cast<char *>(ws), 0, 0};
    Workspace w{};
    const size_t nv = size_t(op->n_b) * op->ld;
    w.outer = carve_cg(c, op);
    w.bp = c.take<double>(nv);
    w.r = c.take<double>(nv);
    w.p = c.take<double>(nv);
    w.q = c.take<double>(nv);
    if (mixed) {
        w.inner = carve_cg(c, op);
        w.b32 = c.take<float>(nv);
        w.x32 = c.take<float>(nv);
        w.bp32 = c.take<float>(nv);
        w.r32 = c.take<float>(nv);
        w.p32 = c.take<float>(nv);
        w.q32 = c.take<float>(nv);
    }
    w.bytes = c.off;
    return w;
}

template <typename T, typename F>
void by_v(int vec, F &&f) {
    switch (vec) {
        case 1: f(std::integral_constant<int, 1>{}); break;
        case 2: f(std::integral_constant<int, 2>{}); break;
        case 4:
            if constexpr (sizeof(T) <= 4) {
                f(std::integral_constant<int, 4>{});
                break;
            }
            [[fallthrough]];
        default: throw Error(FVX_E_ARG, "bad vector width");
    }
}

struct HostScalars {
    CgState st;
    std::vector<double> rho, bnorm2, r0, relres, aux;
    std::vector<int32_t> iters;
};

HostScalars read_state(const CgDev &d, hipStream_t s) {
    HostScalars h;
    h.rho.resize(d.G);
    h.bnorm2.resize(d.G);
    h.r0.resize(d.G);
    h.relres.resize(d.G);
    h.aux.resize(d.G);
    h.iters.resize(d.G);
    FVX_HIP(hipMemcpyAsync(&h.st, d.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    FVX_HIP(hipMemcpyAsync(h.rho.data(), d.rho, 8 * d.G, hipMemcpyDeviceToHost, s));
    FVX_HIP(hipMemcpyAsync(h.bnorm2.data(), d.bnorm2, 8 * d.G, hipMemcpyDeviceToHost, s));
    FVX_HIP(hipMemcpyAsync(h.r0.data(), d.r0, 8 * d.G, hipMemcpyDeviceToHost, s));
    FVX_HIP(hipMemcpyAsync(h.relres.data(), d.relres, 8 * d.G, hipMemcpyDeviceToHost, s));
    FVX_HIP(hipMemcpyAsync(h.aux.data(), d.aux, 8 * d.G, hipMemcpyDeviceToHost, s));
    FVX_HIP(hipMemcpyAsync(h.iters.data(), d.iters, 4 * d.G, hipMemcpyDeviceToHost, s));
    FVX_HIP(hipStreamSynchronize(s));
    return h;
}

int32_t read_done(const CgDev &d, hipStream_t s) {
    int32_t v = 0;
    FVX_HIP(hipMemcpyAsync(&v, &d.st->done, 4, hipMemcpyDeviceToHost, s));
    FVX_HIP(hipStreamSynchronize(s));
    return v;
}

void reset_state(const CgDev &d, int max_iter, hipStream_t s) {
    CgState st{};
    st.max_iter = max_iter;
    FVX_HIP(hipMemcpyAsync(d.st, &st, sizeof(CgState), hipMemcpyHostToDevice, s));
}

// One CG solve in precision T on the op's Laplacian.  b, x, bp, r, p, q are
// [n_b][ld] arrays of T; x holds the guess when `given`.  Returns after the
// device flag says done; the caller reads the state.
template <typename T>
void run_cg(const fvx_op *op, CgDev d, const T *b, T *x, T *bp, T *r, T *p, T *q, bool given, double rtol,
            int max_iter, int poll, hipStream_t s) {
    const fvx_tile t = cg_tile<T>(op);
    RowGrid g;
    auto a = row_args<T>(op, op->n_b, g, t, max_blocks_for(op));
    d.rtol2 = rtol * rtol;
    reset_state(d, max_iter, s);
    const dim3 grid(g.n_blocks), block(t.block);
    by_v<T>(t.vec, [&](auto Vt) {
        constexpr int V = decltype(Vt)::value;
        if (op->singular) {
            hipLaunchKernelGGL((k_mean<T, V>), grid, block, 0, s, a, d, b, 0, 1);
        } else {
            FVX_HIP(hipMemsetAsync(d.mean, 0, 8 * d.G, s));
        }
        if (given) launch_lap<T>(op, x, q, nullptr, s);
        hipLaunchKernelGGL((k_cg_init<T, V>), grid, block, 0, s, a, d, b, bp, x, r, p, q, int(given));
        FVX_HIP(hipGetLastError());
        int launched = 0;
        while (true) {
            const int batch = std::min(poll, std::max(1, max_iter - launched));
            for (int i = 0; i < batch; ++i) {
                if (op->zfaces)
                    hipLaunchKernelGGL((k_cg_spmm<T, V, true>), grid, block, 0, s, a, d, p, q);
                else
                    hipLaunchKernelGGL((k_cg_spmm<T, V, false>), grid, block, 0, s, a, d, p, q);
                hipLaunchKernelGGL((k_cg_update<T, V>), grid, block, 0, s, a, d, x, r, p, q);
                hipLaunchKernelGGL((k_cg_p<T, V>), grid, block, 0, s, a, d, r, p);
            }
            FVX_HIP(hipGetLastError());
            launched += batch;
            if (read_done(d, s)) break;
            if (launched >= max_iter + 1) break;  // the device flag is set by then
        }
    });
}

// x projection and the true residual in FP64 (relres per group).
void finish_f64(const fvx_op *op, CgDev d, double *x, const double *bp, double *q, hipStream_t s) {
    const fvx_tile t = cg_tile<double>(op);
    RowGrid g;
    auto a = row_args<double>(op, op->n_b, g, t, max_blocks_for(op));
    const dim3 grid(g.n_blocks), block(t.block);
    by_v<double>(t.vec, [&](auto Vt) {
        constexpr int V = decltype(Vt)::value;
        if (op->singular) hipLaunchKernelGGL((k_mean<double, V>), grid, block, 0, s, a, d, x, 1, 0);
        hipLaunchKernelGGL((k_fix_x<double, V>), grid, block, 0, s, a, d, x, int(op->singular));
        launch_lap<double>(op, x, q, nullptr, s);
        hipLaunchKernelGGL((k_resid<double, V>), grid, block, 0, s, a, d, bp, q, (double *)nullptr);
        FVX_HIP(hipGetLastError());
    });
}

void fill_stats(fvx_solve_stats *st, const HostScalars &h, int status) {
    if (!st) return;
    st->status = status;
    st->iters = 0;
    st->relres_rec = st->relres_true = st->r0_over_b = st->bnorm = 0.0;
    for (size_t g = 0; g < h.rho.size(); ++g) {
        st->iters = std::max(st->iters, h.iters[g]);
        const double bb = h.bnorm2[g];
        if (bb > 0.0) {
            st->relres_rec = std::max(st->relres_rec, std::sqrt(h.rho[g] / bb));
            st->r0_over_b = std::max(st->r0_over_b, std::sqrt(h.r0[g] / bb));
        }
        st->relres_true = std::max(st->relres_true, h.relres[g]);
        st->bnorm = std::max(st->bnorm, std::sqrt(bb));
    }
    st->rhs_projected = h.st.rhs_projected;
}

void check_opts(const fvx_op *op, const fvx_solve_opts *o) {
    FVX_REQUIRE(op && o, FVX_E_ARG, "NULL op or options");
    FVX_REQUIRE(o->rtol > 0 && o->rtol < 1, FVX_E_ARG, "rtol must be in (0, 1)");
    FVX_REQUIRE(o->max_iter >= 1, FVX_E_ARG, "max_iter must be >= 1");
    FVX_REQUIRE(o->precision == FVX_F64 || o->precision == FVX_MIXED, FVX_E_ARG,
                "precision must be FVX_F64 or FVX_MIXED");
    FVX_REQUIRE(o->guess == FVX_GUESS_ZERO || o->guess == FVX_GUESS_GIVEN, FVX_E_ARG, "bad guess mode");
    FVX_REQUIRE(o->poll_every >= 1, FVX_E_ARG, "poll_every must be >= 1");
    if (o->precision == FVX_MIXED) {
        FVX_REQUIRE(op->has_f32, FVX_E_ARG, "mixed precision needs an operator built with FP32 copies");
        FVX_REQUIRE(o->inner_rtol > 0 && o->inner_rtol < 1 && o->max_outer >= 1, FVX_E_ARG,
                    "bad inner_rtol or max_outer");
    }
    if (op->percol)
        FVX_REQUIRE(op->k <= 64 * (o->precision == FVX_MIXED ? 2 : 2), FVX_E_UNSUPPORTED,
                    "independent-plane solves support k <= 128");
}

int solve_f64(const fvx_op *op, const double *B, double *X, const fvx_solve_opts *o, Workspace &w,
              fvx_solve_stats *stats, hipStream_t s) {
    run_cg<double>(op, w.outer, B, X, w.bp, w.r, w.p, w.q, o->guess == FVX_GUESS_GIVEN, o->rtol, o->max_iter,
                   o->poll_every, s);
    auto h0 = read_state(w.outer, s);
    finish_f64(op, w.outer, X, w.bp, w.q, s);
    auto h = read_state(w.outer, s);
    h.r0 = h0.r0;
    h.rho = h0.rho;
    h.iters = h0.iters;
    int status = h0.st.status;
    fill_stats(stats, h, status);
    if (stats) stats->outer = 0;
    return status;
}

int solve_mixed(const fvx_op *op, const double *B, double *X, const fvx_solve_opts *o, Workspace &w,
                fvx_solve_stats *stats, hipStream_t s) {
    CgDev D = w.outer;
    D.rtol2 = o->rtol * o->rtol;
    const fvx_tile t = cg_tile<double>(op);
    RowGrid g;
    auto a = row_args<double>(op, op->n_b, g, t, max_blocks_for(op));
    const dim3 grid(g.n_blocks), block(t.block);
    reset_state(D, o->max_iter, s);
    int total_inner = 0, outer = 0, status = FVX_OK;
    std::vector<double> r0;
    by_v<double>(t.vec, [&](auto Vt) {
        constexpr int V = decltype(Vt)::value;
        // bp = B - mean(B), bnorm2; x = x0 or 0.  The init kernel also sets
        // r and p, unused here.
        if (op->singular)
            hipLaunchKernelGGL((k_mean<double, V>), grid, block, 0, s, a, D, B, 0, 1);
        else
            FVX_HIP(hipMemsetAsync(D.mean, 0, 8 * D.G, s));
        const bool given = o->guess == FVX_GUESS_GIVEN;
        if (given) launch_lap<double>(op, X, w.q, nullptr, s);
        hipLaunchKernelGGL((k_cg_init<double, V>), grid, block, 0, s, a, D, B, w.bp, X, w.r, w.p, w.q,
                           int(given));
        FVX_HIP(hipGetLastError());
        auto h = read_state(D, s);
        r0 = h.r0;
        if (h.st.status < 0) {
            status = h.st.status;
            return;
        }
        for (outer = 0;; ++outer) {
            // FP64 outer residual r = bp - L x and its norm per group.
            launch_lap<double>(op, X, w.q, nullptr, s);
            hipLaunchKernelGGL((k_resid<double, V>), grid, block, 0, s, a, D, w.bp, w.q, w.r);
            FVX_HIP(hipGetLastError());
            if (read_done(D, s)) break;  // every group meets rtol
            if (outer >= o->max_outer || total_inner >= o->max_iter) {
                status = FVX_NOT_CONVERGED;
                break;
            }
            // Inner rhs: zero-mean FP32 copy of r for unconverged groups.
            if (op->singular) hipLaunchKernelGGL((k_mean<double, V>), grid, block, 0, s, a, D, w.r, 0, 0);
            hipLaunchKernelGGL((k_to_inner<V>), grid, block, 0, s, a, D, w.r, w.b32, int(op->singular));
            FVX_HIP(hipGetLastError());
            const int budget = std::max(1, o->max_iter - total_inner);
            run_cg<float>(op, w.inner, w.b32, w.x32, w.bp32, w.r32, w.p32, w.q32, false, o->inner_rtol, budget,
                          o->poll_every, s);
            auto hi = read_state(w.inner, s);
            int it = 0;
            for (auto v : hi.iters) it = std::max(it, v);
            total_inner += it;
            if (hi.st.status < 0) {
                status = hi.st.status;
                break;
            }
            {
                const fvx_tile t32 = cg_tile<double>(op);
                RowGrid g2;
                auto a2 = row_args<double>(op, op->n_b, g2, t32, max_blocks_for(op));
                hipLaunchKernelGGL((k_add_inner<V>), dim3(g2.n_blocks), dim3(t32.block), 0, s, a2, X, w.x32);
                FVX_HIP(hipGetLastError());
            }
        }
    });
    // Projection and true residual (recomputed in FP64).
    finish_f64(op, D, X, w.bp, w.q, s);
    auto h = read_state(D, s);
    h.r0 = r0;
    if (status == FVX_OK && h.st.status < 0) status = h.st.status;
    fill_stats(stats, h, status);
    if (stats) {
        stats->iters = total_inner;
        stats->outer = outer;
        stats->relres_rec = stats->relres_true;
    }
    return status;
}

}  // namespace
}  // namespace fvx

using fvx::guard;

extern "C" {

int fvx_solve_opts_default(fvx_solve_opts *o) {
    if (!o) return FVX_E_ARG;
    *o = fvx_solve_opts{};
    o->rtol = 1e-8;
    o->max_iter = 100000;
    o->precision = FVX_F64;
    o->inner_rtol = 1e-4;
    o->max_outer = 50;
    o->guess = FVX_GUESS_ZERO;
    o->poll_every = 64;
    return FVX_OK;
}

int fvx_solve_bytes(const fvx_op *op, const fvx_solve_opts *o, size_t *bytes) {
    return guard([&] {
        fvx::check_opts(op, o);
        FVX_REQUIRE(bytes, FVX_E_ARG, "bytes is NULL");
        *bytes = fvx::carve(nullptr, op, o->precision == FVX_MIXED).bytes;
        return FVX_OK;
    });
}

int fvx_poisson_solve(const fvx_op *op, const double *B, double *X, const fvx_solve_opts *o, void *ws,
                      size_t ws_bytes, fvx_solve_stats *stats, void *stream) {
    return guard([&] {
        const auto t0 = std::chrono::steady_clock::now();
        fvx::check_opts(op, o);
        FVX_REQUIRE(B && X && ws, FVX_E_ARG, "NULL B, X or workspace");
        FVX_REQUIRE(reinterpret_cast<uintptr_t>(B) % 16 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0 &&
                        reinterpret_cast<uintptr_t>(ws) % 256 == 0,
                    FVX_E_ARG, "B and X must be 16-byte aligned and ws 256-byte aligned");
        const bool mixed = o->precision == FVX_MIXED;
        auto w = fvx::carve(ws, op, mixed);
        FVX_REQUIRE(ws_bytes >= w.bytes, FVX_E_NOMEM, "workspace too small: need " + std::to_string(w.bytes));
        hipStream_t s = fvx::as_stream(stream);
        const int rc = mixed ? fvx::solve_mixed(op, B, X, o, w, stats, s) : fvx::solve_f64(op, B, X, o, w, stats, s);
        if (stats)
            stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (rc < 0) throw fvx::Error(rc, fvx_status_str(rc));
        return rc;
    });
}

}  // extern "C"
