// Conjugate-gradient Poisson solve on the repeated-block Laplacian.
//
// CG runs on the SPD operator A = -L with right-hand side -b.  One iteration
// is two kernels on the caller's stream:
//   A (direction + SpMM):  prologue sums the r.r partials of the previous
//      iteration (every block, fixed order) into rho, beta and the
//      convergence test; the body forms p' = r + beta p on the fly for every
//      row it gathers, stores p' for its own rows (p is double-buffered), and
//      computes q = L p' for the partial dot products p'.q -- q itself is not
//      stored;
//   B (update):  prologue sums the p'.q partials into alpha; the body forms
//      q = L p' again from the stored p' (gathering p' as A gathered r and
//      p, with the same operations, so it is A's q bit for bit) and updates
//      x += alpha p', r -= alpha A p' (= r + alpha q) with partial r.r.
// Recomputing q instead of storing and re-reading it moves 8 vectors per
// iteration instead of 10 (A: r, p read, p' written; B: p', x, r read, x, r
// written); the SpMM's arithmetic is far below the bandwidth roofline.
// All scalars stay on the device; every block derives them from the same
// partials in the same order, so results are deterministic and no kernel
// waits on another block of its own grid.  Groups are the k columns when the
// planes are independent systems (each column its own CG, frozen once
// converged; per-column partials are folded by a small kernel between the
// two) or one global group when the planes are coupled.  The host reads the
// device "done" flag every poll_every iterations; kernels launched after
// convergence return at once.
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>

#include "amg.h"

namespace fvx {
namespace {


// Where a kernel finds the partials it has to sum: n rows of G values.
struct Src {
    const double *p;
    int n;
};

// Partial sums of a vector per group (for plain means).
template <typename T, int V>
__device__ void b_sum(const RowArgs<T> &a, const CgDev &d, VB vb, const T *__restrict__ v, double *__restrict__ part) {
    __shared__ double lds[kMaxPercolBlock * kMaxV];
    ROW_PROLOGUE
    double c[1][V] = {};
    FOR_ROWS {
        const vec_t<T, V> vv = ldv<T, V>(v + row * a.ld + c0);
#pragma unroll
        for (int u = 0; u < V; ++u)
            if (c0 + u < a.k) c[0][u] += double(vv[u]);
    }
    END_ROWS
    write_partials<1, V>(c, sub, lpr, d.G, d.percol, part, blk, vb.nblk, lds);
}

template <typename T, int V>
__global__ __launch_bounds__(kMaxCgBlock) void k_sum(RowArgs<T> a, CgDev d, const T *__restrict__ v,
                                                     double *__restrict__ part) {
    b_sum<T, V>(a, d, vb_single(a.remap), v, part);
}

// Start: mean (if singular) from partials; bp = b - mean; r = L x0 - bp (x0
// given, L x0 in q) or -bp; x = 0 for the zero guess; partials of r.r and
// b.b into part_b.
template <typename T, int V, int PRE>
__device__ void b_cg_init(const RowArgs<T> &a, const CgDev &d, VB vb, Src mean_src, int singular,
                          const T *__restrict__ b, T *__restrict__ bp, T *__restrict__ x, T *__restrict__ r,
                          const T *__restrict__ q, int given) {
    __shared__ double lds[kMaxPercolBlock * kMaxV];
    __shared__ double tot[kMaxGroups];
    ROW_PROLOGUE
    const int G = d.G;
    if (singular) {
        sum_partials(mean_src.p, mean_src.n, G, lds, tot);
        for (int g = threadIdx.x; g < G; g += blockDim.x) {
            const double m = tot[g] / double(d.count);
            tot[g] = m;
            if (blk == 0) {
                d.mean[g] = m;
                if (!isfinite(m)) {
                    d.st->status = FVX_E_NONFINITE;
                    d.st->done = 1;
                }
                if (m != 0.0) d.st->rhs_projected = 1;
            }
        }
    } else {
        for (int g = threadIdx.x; g < G; g += blockDim.x) tot[g] = 0.0;
    }
    __syncthreads();
    double c[2][V] = {}, cz[1][V] = {};
    FOR_ROWS {
        const int64_t o = row * a.ld + c0;
        vec_t<T, V> bv = ldv<T, V>(b + o), rv;
        const vec_t<T, V> qv = given ? ldv<T, V>(q + o) : vec_t<T, V>(0);
        const double di = PRE == 1 ? double(a.A.dinv[row]) : 0.0;
#pragma unroll
        for (int u = 0; u < V; ++u) {
            if (c0 + u >= a.k) continue;
            bv[u] = T(double(bv[u]) - tot[group_of(d, c0 + u)]);
            rv[u] = given ? qv[u] - bv[u] : -bv[u];
            c[0][u] += double(rv[u]) * double(rv[u]);
            c[1][u] += double(bv[u]) * double(bv[u]);
            if constexpr (PRE == 1) cz[0][u] += double(rv[u]) * (di * double(rv[u]));
        }
        stv_masked<T, V>(bp + o, bv, a.k - c0);
        stv_masked<T, V>(r + o, rv, a.k - c0);
        if (!given) stv_masked<T, V>(x + o, vec_t<T, V>(0), a.k - c0);
    }
    END_ROWS
    write_partials<2, V>(c, sub, lpr, G, d.percol, d.part_b, blk, vb.nblk, lds);
    if constexpr (PRE == 1) {
        __syncthreads();
        write_partials<1, V>(cz, sub, lpr, G, d.percol, d.part_b + 2 * int64_t(vb.nblk) * G, blk, vb.nblk, lds);
    }
}

template <typename T, int V, int PRE>
__global__ __launch_bounds__(kMaxCgBlock) void k_cg_init(RowArgs<T> a, CgDev d, Src mean_src, int singular,
                                                         const T *__restrict__ b, T *__restrict__ bp,
                                                         T *__restrict__ x, T *__restrict__ r,
                                                         const T *__restrict__ q, int given) {
    b_cg_init<T, V, PRE>(a, d, vb_single(a.remap), mean_src, singular, b, bp, x, r, q, given);
}

// A: direction update fused with the SpMM.  rr: partial sums of r.r after the
// previous iteration (or after init, with bb the b.b sums, when it == 0).
// Preconditioned (PRE = 1 Jacobi, 2 Chebyshev): rz holds the partials of r.z,
// which replaces r.r in rho = r.z and beta; the stopping test stays on r.r.
// The direction is p' = z + beta p: z = D^-1 r on the fly for Jacobi, the
// stored Chebyshev output (passed as r) otherwise.
template <typename T, int V, bool Z, int WT, int PRE, bool LN>
__device__ void b_cg_a(const RowArgs<T> &a, const CgDev &d, VB vb, int it, Src rr, Src bb, Src rz,
                       const T *__restrict__ r, const T *__restrict__ p_old, T *__restrict__ p_new) {
    if (d.st->done) return;
    __shared__ double lds[kMaxPercolBlock * kMaxV];
    __shared__ double tot[kMaxGroups];
    __shared__ double tbb[kMaxGroups];
    __shared__ double trz[kMaxGroups];
    __shared__ double s_beta[kMaxGroups];
    __shared__ int s_any, s_bad;
    ROW_PROLOGUE
    const int G = d.G;
    sum_partials(rr.p, rr.n, G, lds, tot);
    if (it == 0) sum_partials(bb.p, bb.n, G, lds, tbb);
    if (PRE) sum_partials(rz.p, rz.n, G, lds, trz);
    if (threadIdx.x == 0) s_any = s_bad = 0;
    __syncthreads();
    const int prev = (it + 1) & 1, cur = it & 1;
    for (int g = threadIdx.x; g < G; g += blockDim.x) {
        const double rn = tot[g];
        const double rzn = PRE ? trz[g] : rn;
        double beta = 0.0, rho = rzn;
        int act;
        if (it == 0) {
            const double b2 = tbb[g];
            const bool bad = !isfinite(rn) || !isfinite(b2) || !isfinite(rzn);
            if (bad) atomicOr(&s_bad, 1);
            act = !bad && b2 > 0.0 && rn > d.rtol2 * b2;
            if (blk == 0) {
                d.bnorm2[g] = b2;
                d.r0[g] = rn;
                d.iters[g] = 0;
                d.rho_last[g] = rn;
            }
        } else if (d.active[prev * G + g]) {
            if (!isfinite(rn) || !isfinite(rzn)) {
                atomicOr(&s_bad, 1);
                act = 0;
            } else {
                beta = rzn / d.rho[prev * G + g];
                act = rn > d.rtol2 * d.bnorm2[g];
            }
            if (blk == 0) {
                d.rho_last[g] = rn;
                d.iters[g] = it;
            }
        } else {
            rho = d.rho[prev * G + g];
            act = 0;
        }
        s_beta[g] = act ? beta : 0.0;
        if (act) atomicOr(&s_any, 1);
        if (blk == 0) {
            d.rho[cur * G + g] = rho;
            d.active[cur * G + g] = act;
        }
    }
    __syncthreads();
    if (s_bad || !s_any || it >= d.st->max_iter) {
        if (blk == 0 && threadIdx.x == 0) {
            d.st->done = 1;
            d.st->iter = it;
            if (s_bad)
                d.st->status = FVX_E_NONFINITE;
            else if (s_any && d.st->status == 0)
                d.st->status = FVX_NOT_CONVERGED;
        }
        return;
    }
    if (blk == 0 && threadIdx.x == 0) d.st->iter = it;
    const bool single = lpr * V >= a.k;
    double c[1][V] = {};
    using Load = std::conditional_t<PRE == 1, DirLoadJ<T, V>, DirLoad<T, V>>;
    auto loader = [&](int c0) {
        Load in;
        if constexpr (PRE == 1)
            in = Load{r, p_old, a.A.dinv, a.ld, vec_t<T, V>(0)};
        else
            in = Load{r, p_old, a.ld, vec_t<T, V>(0)};
#pragma unroll
        for (int u = 0; u < V; ++u) in.beta[u] = T(s_beta[d.percol ? (c0 + u < a.k ? c0 + u : 0) : 0]);
        return in;
    };
    auto emit = [&](int64_t row, int c0, const vec_t<T, V> &pn, const vec_t<T, V> &acc) {
        stv_masked<T, V>(p_new + row * a.ld + c0, pn, a.k - c0);
#pragma unroll
        for (int u = 0; u < V; ++u)
            if (c0 + u < a.k) c[0][u] += double(pn[u]) * double(acc[u]);
    };
    if constexpr (LN) {
        FOR_LINE_TILES {
            vec_t<T, V> acc[kCgLines], pn[kCgLines];
            int64_t rows[kCgLines];
            bool ok[kCgLines];
            cart_lines<T, V, Z>(a, loader(sub * V), uint32_t(t), uint32_t(grp), sub, lpr, acc, pn, rows, ok);
#pragma unroll
            for (int q = 0; q < kCgLines; ++q)
                if (ok[q]) emit(rows[q], sub * V, pn[q], acc[q]);
        }
    } else {
        FOR_ROWS {
            vec_t<T, V> pn;
            const vec_t<T, V> acc =
                lap_row_ld<T, V, Z, WT>(a.A, loader(c0), a.n_b, a.k, a.W, row, c0, sub, lpr, single, pn);
            emit(row, c0, pn, acc);
        }
        END_ROWS
    }
    write_partials<1, V>(c, sub, lpr, G, d.percol, d.part_a, blk, vb.nblk, lds);
}

// B: alpha from the p.q partials; q = L p from the stored p (gathered);
// x += alpha p; r += alpha q; partial r.r (and, with the Jacobi
// preconditioner, r.z with z = D^-1 r).
template <typename T, int V, bool Z, int WT, int PRE, bool LN>
__device__ void b_cg_b(const RowArgs<T> &a, const CgDev &d, VB vb, int it, Src pq, T *__restrict__ x,
                       T *__restrict__ r, const T *__restrict__ p) {
    if (d.st->done) return;
    __shared__ double lds[kMaxPercolBlock * kMaxV];
    __shared__ double tot[kMaxGroups];
    __shared__ int s_bad;
    ROW_PROLOGUE
    const int G = d.G;
    if (blk == 0 && threadIdx.x == 0) d.st->next_it = it + 1;
    sum_partials(pq.p, pq.n, G, lds, tot);
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const int cur = it & 1;
    for (int g = threadIdx.x; g < G; g += blockDim.x) {
        double alpha = 0.0;
        if (d.active[cur * G + g]) {
            const double pap = -tot[g];
            if (!(pap > 0.0) || !isfinite(pap))
                atomicOr(&s_bad, isfinite(pap) ? 1 : 2);
            else
                alpha = d.rho[cur * G + g] / pap;
        }
        tot[g] = alpha;
        if (blk == 0) d.alpha[g] = alpha;
    }
    __syncthreads();
    if (s_bad) {
        if (blk == 0 && threadIdx.x == 0) {
            d.st->done = 1;
            d.st->status = (s_bad & 2) ? FVX_E_NONFINITE : FVX_E_BREAKDOWN;
        }
        return;
    }
    const bool single = lpr * V >= a.k;
    double c[1][V] = {}, cz[1][V] = {};
    auto update = [&](int64_t row, int c0, const vec_t<T, V> &pv, const vec_t<T, V> &qv, vec_t<T, V> xv,
                      vec_t<T, V> rv) {
        const int64_t o = row * a.ld + c0;
        const double di = PRE == 1 ? double(a.A.dinv[row]) : 0.0;
#pragma unroll
        for (int u = 0; u < V; ++u) {
            if (c0 + u >= a.k) continue;
            const T al = T(tot[group_of(d, c0 + u)]);
            xv[u] += al * pv[u];
            rv[u] += al * qv[u];
            c[0][u] += double(rv[u]) * double(rv[u]);
            if constexpr (PRE == 1) cz[0][u] += double(rv[u]) * (di * double(rv[u]));
        }
        stv_masked<T, V>(x + o, xv, a.k - c0);
        stv_masked<T, V>(r + o, rv, a.k - c0);
    };
    if constexpr (LN) {
        FOR_LINE_TILES {
            vec_t<T, V> qv[kCgLines], pv[kCgLines], xv[kCgLines], rv[kCgLines];
            int64_t rows[kCgLines];
            bool ok[kCgLines];
            cart_lines<T, V, Z>(a, PlainLoad<T, V>{p, a.ld}, uint32_t(t), uint32_t(grp), sub, lpr, qv, pv, rows, ok);
#pragma unroll
            for (int q = 0; q < kCgLines; ++q) {
                xv[q] = ldv<T, V>(x + rows[q] * a.ld + sub * V);
                rv[q] = ldv<T, V>(r + rows[q] * a.ld + sub * V);
            }
#pragma unroll
            for (int q = 0; q < kCgLines; ++q)
                if (ok[q]) update(rows[q], sub * V, pv[q], qv[q], xv[q], rv[q]);
        }
    } else {
        FOR_ROWS {
            const int64_t o = row * a.ld + c0;
            vec_t<T, V> pv;
            const vec_t<T, V> qv = lap_row<T, V, Z, WT>(a.A, p, a.n_b, a.k, a.ld, a.W, row, c0, sub, lpr, single, pv);
            update(row, c0, pv, qv, ldv<T, V>(x + o), ldv<T, V>(r + o));
        }
        END_ROWS
    }
    write_partials<1, V>(c, sub, lpr, G, d.percol, d.part_b, blk, vb.nblk, lds);
    if constexpr (PRE == 1) {
        __syncthreads();
        write_partials<1, V>(cz, sub, lpr, G, d.percol, d.part_b + 2 * int64_t(vb.nblk) * G, blk, vb.nblk, lds);
    }
}

// End: x -= mean(x) (singular L; mean from partials), x = 0 where b vanished.
template <typename T, int V>
__global__ __launch_bounds__(kMaxCgBlock) void k_fix_x(RowArgs<T> a, CgDev d, Src mean_src, int project,
                                                       T *__restrict__ x) {
    __shared__ double lds[kMaxPercolBlock * kMaxV];
    __shared__ double tot[kMaxGroups];
    const VB vb = vb_single(a.remap);
    ROW_PROLOGUE
    const int G = d.G;
    if (project) {
        sum_partials(mean_src.p, mean_src.n, G, lds, tot);
    } else {
        for (int g = threadIdx.x; g < G; g += blockDim.x) tot[g] = 0.0;
        __syncthreads();
    }
    FOR_ROWS {
        vec_t<T, V> xv = ldv<T, V>(x + row * a.ld + c0);
#pragma unroll
        for (int u = 0; u < V; ++u) {
            if (c0 + u >= a.k) continue;
            const int g = group_of(d, c0 + u);
            xv[u] = d.bnorm2[g] == 0.0 ? T(0) : T(double(xv[u]) - tot[g] / double(d.count));
        }
        stv_masked<T, V>(x + row * a.ld + c0, xv, a.k - c0);
    }
    END_ROWS
}

// r = bp - q (optional) with partial sums of r.r and of r.
template <typename T, int V>
__global__ __launch_bounds__(kMaxCgBlock) void k_resid(RowArgs<T> a, CgDev d, const T *__restrict__ bp,
                                                       const T *__restrict__ q, T *__restrict__ r,
                                                       double *__restrict__ part) {
    __shared__ double lds[kMaxPercolBlock * kMaxV];
    const VB vb = vb_single(a.remap);
    ROW_PROLOGUE
    double c[2][V] = {};
    FOR_ROWS {
        const int64_t o = row * a.ld + c0;
        const vec_t<T, V> rv = ldv<T, V>(bp + o) - ldv<T, V>(q + o);
#pragma unroll
        for (int u = 0; u < V; ++u)
            if (c0 + u < a.k) {
                c[0][u] += double(rv[u]) * double(rv[u]);
                c[1][u] += double(rv[u]);
            }
        if (r) stv_masked<T, V>(r + o, rv, a.k - c0);
    }
    END_ROWS
    write_partials<2, V>(c, sub, lpr, d.G, d.percol, part, blk, vb.nblk, lds);
}

// Mixed precision: inner right-hand side b32 = r - mean_g for groups still
// iterating (zero for converged groups).  gmean/gact: host-computed [G].
template <int V>
__global__ __launch_bounds__(kMaxCgBlock) void k_to_inner(RowArgs<double> a, CgDev d, const double *__restrict__ r,
                                                          const double *__restrict__ gmean,
                                                          const double *__restrict__ gact, float *__restrict__ b32) {
    const VB vb = vb_single(a.remap);
    ROW_PROLOGUE
    (void)blk;
    FOR_ROWS {
        const vec_t<double, V> rv = ldv<double, V>(r + row * a.ld + c0);
        vec_t<float, V> o;
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const int g = group_of(d, c0 + u < a.k ? c0 + u : 0);
            o[u] = gact[g] != 0.0 ? float(rv[u] - gmean[g]) : 0.0f;
        }
        stv_masked<float, V>(b32 + row * a.ld + c0, o, a.k - c0);
    }
    END_ROWS
}

// Mixed precision: x += d32 in FP64.
template <int V>
__global__ __launch_bounds__(kMaxCgBlock) void k_add_inner(RowArgs<double> a, double *__restrict__ x,
                                                           const float *__restrict__ d32) {
    const VB vb = vb_single(a.remap);
    ROW_PROLOGUE
    (void)blk;
    FOR_ROWS {
        const int64_t o = row * a.ld + c0;
        vec_t<double, V> xv = ldv<double, V>(x + o);
        const vec_t<float, V> dv = ldv<float, V>(d32 + o);
#pragma unroll
        for (int u = 0; u < V; ++u) xv[u] += double(dv[u]);
        stv_masked<double, V>(x + o, xv, a.k - c0);
    }
    END_ROWS
}

// ---------------------------------------------------------------------------
// Batched launches: one grid covers several problems.  Each problem owns a
// contiguous range of hardware blocks starting at a multiple of 8 (so the
// XCD-aware order holds inside the range) and runs exactly the virtual blocks
// of its single-problem grid.  Blocks past a problem's range (alignment
// padding) return at once.
// ---------------------------------------------------------------------------

template <typename T>
struct BItem {
    RowArgs<T> a;
    CgDev d;
    const T *b;
    T *x, *bp, *r, *p0, *p1, *q;
    T *z[2], *zf;  // Chebyshev: the two z buffers and the one holding the final z
    Src rr, bb, pq, rz;
    int nblk, first;
};

// The item whose block range holds this block: the last one with first <=
// blockIdx.x (items ascend by first, items[0].first = 0).
template <typename T>
__device__ __forceinline__ int find_item(const BItem<T> *items, int n) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (items[mid].first <= int(blockIdx.x))
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// p' of iteration it: p0 on even iterations, p1 on odd ones; the previous
// direction is r at it = 0 (p' = r + 0 r) and the other buffer afterwards.
// The iteration number comes from the item's state (next_it here, iter in
// the update kernel), so the kernels take the same arguments on every
// iteration.
template <typename T, int V, bool Z, int WT, int PRE, bool LN>
__global__ __launch_bounds__(kMaxCgBlock) void kb_cg_a(const BItem<T> *__restrict__ items, int n) {
    const BItem<T> &I = items[find_item(items, n)];
    const int local = int(blockIdx.x) - I.first;
    if (local >= I.nblk) return;
    const RowArgs<T> a = I.a;
    const CgDev d = I.d;
    const int it = d.st->next_it;
    const VB vb{logical_block_of(local, I.nblk, a.remap), I.nblk};
    T *src = PRE == 2 ? I.zf : I.r;
    T *pold = it == 0 ? src : ((it & 1) ? I.p0 : I.p1);
    T *pnew = (it & 1) ? I.p1 : I.p0;
    b_cg_a<T, V, Z, WT, PRE, LN>(a, d, vb, it, I.rr, I.bb, I.rz, src, pold, pnew);
}

template <typename T, int V, bool Z, int WT, int PRE, bool LN>
__global__ __launch_bounds__(kMaxCgBlock) void kb_cg_b(const BItem<T> *__restrict__ items, int n) {
    const BItem<T> &I = items[find_item(items, n)];
    const int local = int(blockIdx.x) - I.first;
    if (local >= I.nblk) return;
    const RowArgs<T> a = I.a;
    const CgDev d = I.d;
    const int it = d.st->iter;
    const VB vb{logical_block_of(local, I.nblk, a.remap), I.nblk};
    T *pnew = (it & 1) ? I.p1 : I.p0;
    b_cg_b<T, V, Z, WT, PRE, LN>(a, d, vb, it, I.pq, I.x, I.r, pnew);
}

// Chebyshev step j >= 1 for every item: gathers z_j from buffer (j - 2) & 1
// (r when j == 1) and writes z_{j+1} over z_{j-1} in buffer (j - 1) & 1.
template <typename T, int V, bool Z, int WT, int MODE, bool LAST>
__global__ __launch_bounds__(kMaxCgBlock) void kb_cheb(const BItem<T> *__restrict__ items, int n, int j, T c1, T c2,
                                                       T inv_theta) {
    const BItem<T> &I = items[find_item(items, n)];
    const int local = int(blockIdx.x) - I.first;
    if (local >= I.nblk) return;
    const RowArgs<T> a = I.a;
    const CgDev d = I.d;
    const VB vb{logical_block_of(local, I.nblk, a.remap), I.nblk};
    b_cheb<T, V, Z, WT, MODE, LAST>(a, d, vb, I.r, I.z[j & 1], I.z[(j - 1) & 1], c1, c2, inv_theta);
}

// A fixed, nonzero right-hand side for timing CG tiles: a hash of the index
// in [-0.5, 0.5) (its mean is projected away like any other).
__global__ __launch_bounds__(256) void k_fill_pattern(double *__restrict__ b, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        b[i] = double((uint64_t(i) * 2654435761ull) % 1000ull) / 1000.0 - 0.5;
}

// What the host reads at a poll, per item: its CG's done flag and the
// largest ||r||^2 / ||b||^2 over its groups still iterating (one read back
// per poll for the batch).
struct PollRec {
    int32_t done, pad;
    double r2;
};

template <typename T>
__global__ __launch_bounds__(256) void kb_done(const BItem<T> *__restrict__ items, int n, PollRec *__restrict__ out) {
    for (int i = int(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const CgDev &d = items[i].d;
        double r2 = 0.0;
        for (int g = 0; g < d.G; ++g)
            if (d.bnorm2[g] > 0.0) r2 = fmax(r2, d.rho_last[g] / d.bnorm2[g]);
        out[i].done = d.st->done;
        out[i].r2 = r2;
    }
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------

struct Carve {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t n) {
        T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
        off += (sizeof(T) * n + 255) / 256 * 256;
        return p;
    }
};

int groups_of(const fvx_op *op) { return op->percol ? op->k : 1; }
int max_blocks_for(const fvx_op *) { return 2048; }

// CG launch tile for precision T: the tile set by the CG autotuner, else a
// default (the SpMM tile's vector width, 256 threads, XCD remap, a grid of at
// most 1024 blocks); lanes per row widened so that one pass of a row group
// covers all k columns, at most kMaxCgBlock threads (kMaxPercolBlock for
// independent planes).
template <typename T>
fvx_tile cg_tile(const fvx_op *op) {
    const int dt = dtype_of<T>();
    fvx_tile t = op->cg_tile[dt];
    if (t.block <= 0) {
        t = op->tile[dt];
        t.block = 256;
        t.xcd_remap = 1;
        t.max_blocks = 1024;
        t.stage_lds = 0;
        t.nt_store = 0;
    }
    if (t.lanes_per_row * t.vec < op->k) t.lanes_per_row = std::min(64, next_pow2(int(ceil_div(op->k, t.vec))));
    if (op->percol && t.lanes_per_row * t.vec < op->k) {
        const fvx_tile d = default_tile(op, dt);
        t.vec = d.vec;
        t.lanes_per_row = d.lanes_per_row;
    }
    FVX_REQUIRE(!op->percol || t.lanes_per_row * t.vec >= op->k, FVX_E_UNSUPPORTED,
                "independent-plane solve: k exceeds one pass of a row group");
    t.block = std::max(std::min(t.block, op->percol ? kMaxPercolBlock : kMaxCgBlock), t.lanes_per_row);
    return t;
}

// Line tiles (stage_lds of a CG tile) apply on a Cartesian 5-point base
// with its coefficient record, when one pass of a row group covers the k
// columns and the grid has at least kCgLines lines; elsewhere the tile's
// row mapping is used.
template <typename T>
bool cg_lines_ok(const fvx_op *op, const fvx_tile &t) {
    return op->stencil == 7 && dev<T>(op).cart != nullptr && op->W == 4 && op->grid_nx > 0 &&
           op->grid_ny >= kCgLines && t.lanes_per_row * t.vec >= op->k;
}

CgDev carve_cg(Carve &c, const fvx_op *op) {
    CgDev d{};
    const int G = groups_of(op);
    const size_t mb = size_t(max_blocks_for(op));
    d.st = c.take<CgState>(1);
    d.rho = c.take<double>(2 * G);
    d.active = c.take<int32_t>(2 * G);
    d.alpha = c.take<double>(G);
    d.bnorm2 = c.take<double>(G);
    d.r0 = c.take<double>(G);
    d.rho_last = c.take<double>(G);
    d.iters = c.take<int32_t>(G);
    d.part_a = c.take<double>(2 * mb * G);
    d.part_b = c.take<double>(3 * mb * G);
    d.tot = c.take<double>(6 * G);
    d.mean = c.take<double>(G);
    d.G = G;
    d.percol = op->percol ? 1 : 0;
    d.count = op->percol ? op->n_b : op->n_b * int64_t(op->k);
    return d;
}

struct Workspace {
    CgDev outer, inner;
    double *bp, *r, *p0, *p1, *q;
    double *z[2];          // Chebyshev preconditioner buffers (FP64 CG)
    double *gmean, *gact;  // [G] host-filled per-group arrays (mixed outer loop)
    float *b32, *x32, *bp32, *r32, *p32a, *p32b, *q32;
    float *z32[2];         // Chebyshev preconditioner buffers (FP32 inner CG)
    AmgWork<double> amg64;  // multigrid vectors (FP64 CG)
    AmgWork<float> amg32;   // multigrid vectors (FP32 inner CG)
    size_t bytes;
};

Workspace carve(void *ws, const fvx_op *op, bool mixed, bool cheb, const fvx_amg *amg = nullptr) {
    Carve c{static_cast<char *>(ws), 0};
    Workspace w{};
    const size_t nv = size_t(op->n_b) * op->ld;
    w.outer = carve_cg(c, op);
    w.bp = c.take<double>(nv);
    w.r = c.take<double>(nv);
    w.p0 = c.take<double>(nv);
    w.p1 = c.take<double>(nv);
    w.q = c.take<double>(nv);
    if (cheb && !mixed) {
        w.z[0] = c.take<double>(nv);
        w.z[1] = c.take<double>(nv);
    }
    if (mixed) {
        w.inner = carve_cg(c, op);
        w.gmean = c.take<double>(groups_of(op));
        w.gact = c.take<double>(groups_of(op));
        w.b32 = c.take<float>(nv);
        w.x32 = c.take<float>(nv);
        w.bp32 = c.take<float>(nv);
        w.r32 = c.take<float>(nv);
        w.p32a = c.take<float>(nv);
        w.p32b = c.take<float>(nv);
        w.q32 = c.take<float>(nv);
        if (cheb) {
            w.z32[0] = c.take<float>(nv);
            w.z32[1] = c.take<float>(nv);
        }
    }
    if (amg) {
        if (mixed)
            w.amg32 = amg_carve<float>(amg, c.take<char>(amg_work_bytes(amg, FVX_F32)));
        else
            w.amg64 = amg_carve<double>(amg, c.take<char>(amg_work_bytes(amg, FVX_F64)));
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
    std::vector<double> bnorm2, r0, rho_last;
    std::vector<int32_t> iters;
};

HostScalars read_state(const CgDev &d, hipStream_t s) {
    HostScalars h;
    h.bnorm2.resize(d.G);
    h.r0.resize(d.G);
    h.rho_last.resize(d.G);
    h.iters.resize(d.G);
    FVX_HIP(hipMemcpyAsync(&h.st, d.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    FVX_HIP(hipMemcpyAsync(h.bnorm2.data(), d.bnorm2, 8 * d.G, hipMemcpyDeviceToHost, s));
    FVX_HIP(hipMemcpyAsync(h.r0.data(), d.r0, 8 * d.G, hipMemcpyDeviceToHost, s));
    FVX_HIP(hipMemcpyAsync(h.rho_last.data(), d.rho_last, 8 * d.G, hipMemcpyDeviceToHost, s));
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

// Launch context of the row-tiled CG kernels for precision T.
template <typename T>
struct Ctx {
    fvx_tile t;
    RowGrid g;
    RowArgs<T> a;
    dim3 grid, block;
    explicit Ctx(const fvx_op *op) {
        t = cg_tile<T>(op);
        a = row_args<T>(op, op->n_b, g, t, max_blocks_for(op));
        if (t.stage_lds && cg_lines_ok<T>(op, t)) {
            // the iteration kernels take line tiles; the other kernels of the
            // solve keep the row tiles (same blocks, same partials layout)
            a.lines = kCgLines;
            a.n_xtiles = uint32_t(ceil_div(op->grid_nx, a.rows_per_tile));
            a.n_ltiles = a.n_xtiles * uint32_t(ceil_div(op->grid_ny, kCgLines));
            a.ltiles_per_block = ceil_div(int64_t(a.n_ltiles), int64_t(g.n_blocks));
        }
        grid = dim3(g.n_blocks);
        block = dim3(t.block);
    }
};

// Where the consumer of partials [nq][n_blocks][G] finds quantity q_index:
// the partials themselves (one global group, summed in the consumer's
// prologue) or, for per-column groups, totals folded by a small kernel.
Src fold_or_direct(const CgDev &d, const double *part, int nq, int n_blocks, int q_index, double *tot_out,
                   hipStream_t s) {
    if (!d.percol) return Src{part + size_t(q_index) * n_blocks * d.G, n_blocks};
    hipLaunchKernelGGL(k_fold, dim3(nq * d.G), dim3(256), 0, s, part, n_blocks, d.G, tot_out);
    return Src{tot_out + size_t(q_index) * d.G, 1};
}

// Totals per group of a reduction that the host needs.
std::vector<double> host_totals(const CgDev &d, const double *part, int nq, int n_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_fold, dim3(nq * d.G), dim3(256), 0, s, part, n_blocks, d.G, d.tot);
    FVX_HIP(hipGetLastError());
    std::vector<double> h(size_t(nq) * d.G);
    FVX_HIP(hipMemcpyAsync(h.data(), d.tot, 8 * h.size(), hipMemcpyDeviceToHost, s));
    FVX_HIP(hipStreamSynchronize(s));
    return h;
}

// One CG of a batch: the problem's operator, its CG state and its vectors.
template <typename T>
struct CgJob {
    const fvx_op *op;
    CgDev d;
    const T *b;
    T *x, *bp, *r, *p0, *p1, *q;
    bool given;
    double rtol;
    int max_iter;
    T *z0 = nullptr, *z1 = nullptr;  // Chebyshev buffers
    const AmgWork<T> *amgw = nullptr;  // multigrid vectors
};

// Preconditioner of a batch (the same for all its problems): kind 0 none,
// 1 Jacobi, 2 Chebyshev with `degree` >= 2 steps (degree 1 is Jacobi up to a
// constant factor, which CG does not see, so it runs as kind 1).  The step
// coefficients follow Saad's Algorithm 12.1 on [2 / ratio, 2].
struct Precond {
    int kind = 0, degree = 1;  // kind 3: one V-cycle of the multigrid amg
    const fvx_amg *amg = nullptr;
    double inv_theta = 1.0;
    std::vector<double> c1, c2;  // [degree]: step j uses c1[j], c2[j] (j >= 1)
};

Precond make_precond(const fvx_solve_opts *o) {
    Precond pc;
    if (o->precond == FVX_PRECOND_JACOBI || (o->precond == FVX_PRECOND_CHEBYSHEV && o->cheb_degree == 1)) {
        pc.kind = 1;
    } else if (o->precond == FVX_PRECOND_AMG) {
        pc.kind = 3;
        pc.amg = o->amg;
    } else if (o->precond == FVX_PRECOND_CHEBYSHEV) {
        pc.kind = 2;
        pc.degree = o->cheb_degree;
        const double b = 2.0, a = b / o->cheb_ratio;
        const double theta = 0.5 * (b + a), delta = 0.5 * (b - a), sigma = theta / delta;
        pc.inv_theta = 1.0 / theta;
        pc.c1.assign(pc.degree, 0.0);
        pc.c2.assign(pc.degree, 0.0);
        double rho = 1.0 / sigma;
        for (int j = 1; j < pc.degree; ++j) {
            const double rn = 1.0 / (2.0 * sigma - rho);
            pc.c1[j] = rn * rho;
            pc.c2[j] = 2.0 * rn / delta;
            rho = rn;
        }
    }
    return pc;
}

// The CG kernels' view of the preconditioner: 1 Jacobi (formed on the fly),
// 2 a stored z (Chebyshev or multigrid output), 0 none.
template <typename F>
void by_pre(int kind, F &&f) {
    if (kind == 1)
        f(std::integral_constant<int, 1>{});
    else if (kind == 2 || kind == 3)
        f(std::integral_constant<int, 2>{});
    else
        f(std::integral_constant<int, 0>{});
}

// Batched launches group jobs whose kernels share one instance: block size,
// vector width, plane coupling and ELL width.
struct GroupKey {
    int block, vec, z, w, lines;
    bool operator==(const GroupKey &o) const {
        return block == o.block && vec == o.vec && z == o.z && w == o.w && lines == o.lines;
    }
};

// ---------------------------------------------------------------------------
// Launch graphs of the CG iteration (FVX_LAUNCH_GRAPH)
// ---------------------------------------------------------------------------
// The iterations between two polls can be replayed from HIP graphs instead of
// being launched kernel by kernel: graphs of 1, 2, 4, ..., 64 iterations,
// captured on first use and kept in a process-wide cache under a key that
// holds everything a captured launch depends on (device, precision,
// workspace and descriptor addresses, each operator's serial and tiles, the
// preconditioner with its hierarchy's serial, the launch groups).  A later
// solve with the same key replays the cached graphs.  The captured kernels,
// arguments and order are those of the launches they replace, so the
// iterates are bitwise the same either way.
constexpr int kGraphSizes = 7;     // graphs of 2^0 .. 2^6 iterations
constexpr size_t kGraphSets = 16;  // cached keys; the least recently used is dropped first
constexpr int kGraphDevices = 64;

struct GraphSet {
    std::vector<uint64_t> key;
    int device = 0;  // the device the graphs were instantiated on
    hipGraphExec_t ex[kGraphSizes] = {};
    uint64_t used = 0;
};

struct GraphCache {
    std::mutex mu;
    std::vector<std::unique_ptr<GraphSet>> sets;
    hipStream_t cap[kGraphDevices] = {};  // per device: the stream graphs are captured on
    uint64_t clock = 0;
};

// Never destroyed: graph objects are not released during the runtime's own
// teardown at process exit.
GraphCache &graph_cache() {
    static GraphCache *c = new GraphCache;
    return *c;
}

struct KeyBuf {
    std::vector<uint64_t> v;
    void u(int64_t x) { v.push_back(uint64_t(x)); }
    void p(const void *x) { v.push_back(uint64_t(reinterpret_cast<uintptr_t>(x))); }
    void d(double x) {
        uint64_t b;
        std::memcpy(&b, &x, sizeof b);
        v.push_back(b);
    }
    void tile(const fvx_tile &t) {
        for (int x : {t.vec, t.lanes_per_row, t.block, t.xcd_remap, t.max_blocks, t.stage_lds, t.nt_store}) u(x);
    }
};

// The cached set for `key` on `device` (created empty when absent).
// Dropping a set first waits for its device: one of its graphs may still be
// running on another stream.  Caller holds the cache's mutex.
GraphSet &graph_set(GraphCache &c, const std::vector<uint64_t> &key, int device) {
    for (auto &g : c.sets)
        if (g->key == key) {
            g->used = ++c.clock;
            return *g;
        }
    if (c.sets.size() >= kGraphSets) {
        size_t old = 0;
        for (size_t i = 1; i < c.sets.size(); ++i)
            if (c.sets[i]->used < c.sets[old]->used) old = i;
        const int gone = c.sets[old]->device;
        FVX_HIP(hipSetDevice(gone));
        const hipError_t rc = hipDeviceSynchronize();
        for (hipGraphExec_t e : c.sets[old]->ex)
            if (e) (void)hipGraphExecDestroy(e);
        c.sets.erase(c.sets.begin() + long(old));
        FVX_HIP(hipSetDevice(device));
        FVX_HIP(rc);
    }
    c.sets.push_back(std::make_unique<GraphSet>());
    c.sets.back()->key = key;
    c.sets.back()->device = device;
    c.sets.back()->used = ++c.clock;
    return *c.sets.back();
}

// Captures `launch` (which launches on the stream variable `s`) into a graph
// on the device's capture stream and instantiates it.  `s` is pointed at the
// capture stream meanwhile and restored afterwards, also when a launch throws
// (the capture is then ended and its graph dropped).
hipGraphExec_t capture_graph(GraphCache &c, hipStream_t &s, const std::function<void()> &launch) {
    int dev = 0;
    FVX_HIP(hipGetDevice(&dev));
    FVX_REQUIRE(dev >= 0 && dev < kGraphDevices, FVX_E_UNSUPPORTED, "device index beyond the graph cache");
    if (!c.cap[dev]) FVX_HIP(hipStreamCreateWithFlags(&c.cap[dev], hipStreamNonBlocking));
    const hipStream_t user = s, cap = c.cap[dev];
    struct Restore {
        hipStream_t &s, user, cap;
        bool open = true;
        ~Restore() {
            s = user;
            if (open) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(cap, &g);
                if (g) (void)hipGraphDestroy(g);
            }
        }
    } restore{s, user, cap};
    FVX_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    s = cap;
    launch();
    hipGraph_t g = nullptr;
    restore.open = false;
    FVX_HIP(hipStreamEndCapture(cap, &g));
    hipGraphExec_t e = nullptr;
    const hipError_t rc = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    FVX_HIP(rc);
    return e;
}

// Runs the CGs of all jobs.  Each job starts exactly as a single solve would
// (its own launches), then every iteration is one batched launch per phase and
// group.  items_dev: device array for the launch descriptors (>= jobs.size()).
// launch_mode FVX_LAUNCH_GRAPH: the iterations after the first poll are
// replayed from cached graphs (above); the launches, hence the iterates, are
// those of FVX_LAUNCH_PHASES.
template <typename T>
void run_cg_batch(std::vector<CgJob<T>> &jobs, BItem<T> *items_dev, PollRec *flags_dev, int poll, const Precond &pc,
                  int launch_mode, hipStream_t s) {
    if (jobs.empty()) return;
    std::vector<BItem<T>> items(jobs.size());
    std::vector<GroupKey> keys(jobs.size());
    int max_iter = 0;
    for (size_t j = 0; j < jobs.size(); ++j) {
        CgJob<T> &J = jobs[j];
        Ctx<T> c(J.op);
        J.d.rtol2 = J.rtol * J.rtol;
        reset_state(J.d, J.max_iter, s);
        max_iter = std::max(max_iter, J.max_iter);
        const CgDev &d = J.d;
        const int nb = c.g.n_blocks;
        BItem<T> &I = items[j];
        by_v<T>(c.t.vec, [&](auto Vt) {
            constexpr int V = decltype(Vt)::value;
            Src mean{nullptr, 0};
            if (J.op->singular) {
                hipLaunchKernelGGL((k_sum<T, V>), c.grid, c.block, 0, s, c.a, d, J.b, d.part_a);
                mean = fold_or_direct(d, d.part_a, 1, nb, 0, d.tot + 3 * d.G, s);
            }
            if (J.given) launch_lap<T>(J.op, J.x, J.q, nullptr, s);
            if (pc.kind == 1)
                hipLaunchKernelGGL((k_cg_init<T, V, 1>), c.grid, c.block, 0, s, c.a, d, mean, int(J.op->singular),
                                   J.b, J.bp, J.x, J.r, J.q, int(J.given));
            else
                hipLaunchKernelGGL((k_cg_init<T, V, 0>), c.grid, c.block, 0, s, c.a, d, mean, int(J.op->singular),
                                   J.b, J.bp, J.x, J.r, J.q, int(J.given));
            I.rr = fold_or_direct(d, d.part_b, 2, nb, 0, d.tot, s);
            if (pc.kind == 1 && d.percol)
                hipLaunchKernelGGL(k_fold, dim3(d.G), dim3(256), 0, s, d.part_b + size_t(2) * nb * d.G, nb, d.G,
                                   d.tot + 4 * d.G);
            FVX_HIP(hipGetLastError());
        });
        I.a = c.a;
        I.d = d;
        I.b = J.b;
        I.x = J.x;
        I.bp = J.bp;
        I.r = J.r;
        I.p0 = J.p0;
        I.p1 = J.p1;
        I.q = J.q;
        I.z[0] = J.z0;
        I.z[1] = J.z1;
        I.zf = pc.kind == 2   ? (pc.degree % 2 == 0 ? J.z0 : J.z1)  // written by step degree - 1
               : pc.kind == 3 ? amg_output<T>(pc.amg, *J.amgw)
                              : nullptr;
        I.bb = d.percol ? Src{d.tot + d.G, 1} : Src{d.part_b + size_t(nb) * d.G, nb};
        I.pq = d.percol ? Src{d.tot + 2 * d.G, 1} : Src{d.part_a, nb};
        I.rz = d.percol ? Src{d.tot + 4 * d.G, 1} : Src{d.part_b + size_t(2) * nb * d.G, nb};
        I.nblk = nb;
        keys[j] = GroupKey{c.t.block, c.t.vec, int(J.op->zfaces), J.op->W, c.a.lines};
    }
    // Order jobs by group, give each a block range aligned to 8, upload.
    std::vector<int> order(jobs.size());
    for (size_t j = 0; j < jobs.size(); ++j) order[j] = int(j);
    std::vector<GroupKey> gk;
    std::vector<std::vector<int>> members;
    for (size_t j = 0; j < jobs.size(); ++j) {
        size_t g = 0;
        while (g < gk.size() && !(gk[g] == keys[j])) ++g;
        if (g == gk.size()) {
            gk.push_back(keys[j]);
            members.emplace_back();
        }
        members[g].push_back(int(j));
    }
    struct Launch {
        GroupKey key;
        int offset, n, blocks;
        std::vector<int> jobs;
    };
    std::vector<Launch> launches;
    std::vector<BItem<T>> packed;
    for (size_t g = 0; g < gk.size(); ++g) {
        Launch L{gk[g], int(packed.size()), 0, 0, members[g]};
        int first = 0;
        for (int j : members[g]) {
            BItem<T> I = items[j];
            I.first = first;
            first += int(ceil_div(I.nblk, 8) * 8);
            packed.push_back(I);
        }
        L.n = int(members[g].size());
        L.blocks = first;
        launches.push_back(L);
    }
    FVX_HIP(hipMemcpyAsync(items_dev, packed.data(), sizeof(BItem<T>) * packed.size(), hipMemcpyHostToDevice, s));
    FVX_HIP(hipStreamSynchronize(s));
    // Per-column groups fold their partials for the next kernel: 0 p.q (after
    // A), 1 r.r (after B), 2 r.z (after B with Jacobi, after the last
    // Chebyshev step).
    auto fold_percol = [&](const Launch &L, int what) {
        for (int j : L.jobs) {
            const CgDev &d = jobs[j].d;
            if (!d.percol) continue;
            const int nb = items[j].nblk;
            if (what == 0)
                hipLaunchKernelGGL(k_fold, dim3(d.G), dim3(256), 0, s, d.part_a, nb, d.G, d.tot + 2 * d.G);
            else if (what == 1)
                hipLaunchKernelGGL(k_fold, dim3(d.G), dim3(256), 0, s, d.part_b, nb, d.G, d.tot);
            else
                hipLaunchKernelGGL(k_fold, dim3(d.G), dim3(256), 0, s, d.part_b + size_t(2) * nb * d.G, nb, d.G,
                                   d.tot + 4 * d.G);
        }
    };
    // The Chebyshev preconditioner on the current r of every item.
    auto cheb_pass = [&](const Launch &L) {
        const BItem<T> *dev = items_dev + L.offset;
        by_v<T>(L.key.vec, [&](auto Vt) {
            constexpr int V = decltype(Vt)::value;
            by_width(L.key.w, [&](auto Wt) {
                constexpr int WT = decltype(Wt)::value;
                for (int j = 1; j < pc.degree; ++j) {
                    const T c1 = T(pc.c1[j]), c2 = T(pc.c2[j]), ith = T(pc.inv_theta);
                    const bool last = j == pc.degree - 1;
                    auto go = [&](auto Zt, auto Mt, auto Lt) {
                        hipLaunchKernelGGL((kb_cheb<T, V, decltype(Zt)::value, WT, decltype(Mt)::value,
                                                    decltype(Lt)::value>),
                                           dim3(L.blocks), dim3(L.key.block), 0, s, dev, L.n, j, c1, c2, ith);
                    };
                    auto by_fl = [&](auto Zt) {
                        auto with_mode = [&](auto Mt) {
                            if (last)
                                go(Zt, Mt, std::true_type{});
                            else
                                go(Zt, Mt, std::false_type{});
                        };
                        if (j == 1)
                            with_mode(std::integral_constant<int, 0>{});
                        else if (j == 2)
                            with_mode(std::integral_constant<int, 1>{});
                        else
                            with_mode(std::integral_constant<int, 2>{});
                    };
                    if (L.key.z)
                        by_fl(std::true_type{});
                    else
                        by_fl(std::false_type{});
                }
            });
        });
        fold_percol(L, 2);
    };
    // The multigrid V-cycle on the current r of every item (one item per
    // launch: a hierarchy belongs to one operator); its last step runs with
    // the CG's tile and writes the r.z partials.
    auto amg_pass = [&](const Launch &L) {
        for (int j : L.jobs) {
            const CgJob<T> &J = jobs[j];
            const Ctx<T> c(J.op);
            const AmgFinal<T> fin{c.a, c.grid, c.block, c.t.vec};
            amg_vcycle<T>(pc.amg, J.r, *J.amgw, J.d, &fin, s);
        }
        fold_percol(L, 2);
    };
    auto pre_pass = [&](const Launch &L) {
        if (pc.kind == 2) cheb_pass(L);
        if (pc.kind == 3) amg_pass(L);
    };
    for (const Launch &L : launches) pre_pass(L);
    // Iterations launched between polls: min(poll, 8) first, then the number
    // the residual's decay since the previous poll predicts to reach every
    // job's tolerance (plus one), at most `poll`.  Kernels launched after
    // convergence return at once but still cost a launch each, so the batch
    // follows the prediction; the arithmetic does not depend on it.
    // One iteration of every item: per launch group the direction kernel, the
    // update kernel, the folds of per-column partials and the preconditioner.
    // Every iteration launches the same kernels with the same arguments.
    auto iteration = [&]() {
        for (const Launch &L : launches) {
            const BItem<T> *dev = items_dev + L.offset;
            by_pre(pc.kind, [&](auto Pt) {
                constexpr int PRE = decltype(Pt)::value;
                by_v<T>(L.key.vec, [&](auto Vt) {
                    constexpr int V = decltype(Vt)::value;
                    constexpr int PB = PRE == 1 ? 1 : 0;
                    const dim3 gb(L.blocks), bb(L.key.block);
                    // line tiles exist for the compiled width 4 (the Cartesian
                    // 5-point base) only
                    by_width(L.key.w, [&](auto Wt) {
                        constexpr int WT = decltype(Wt)::value;
                        const bool ln = WT == 4 && L.key.lines;
                        if (L.key.z) {
                            if (ln)
                                hipLaunchKernelGGL((kb_cg_a<T, V, true, WT, PRE, WT == 4>), gb, bb, 0, s, dev, L.n);
                            else
                                hipLaunchKernelGGL((kb_cg_a<T, V, true, WT, PRE, false>), gb, bb, 0, s, dev, L.n);
                        } else {
                            if (ln)
                                hipLaunchKernelGGL((kb_cg_a<T, V, false, WT, PRE, WT == 4>), gb, bb, 0, s, dev, L.n);
                            else
                                hipLaunchKernelGGL((kb_cg_a<T, V, false, WT, PRE, false>), gb, bb, 0, s, dev, L.n);
                        }
                    });
                    fold_percol(L, 0);
                    by_width(L.key.w, [&](auto Wt) {
                        constexpr int WT = decltype(Wt)::value;
                        const bool ln = WT == 4 && L.key.lines;
                        if (L.key.z) {
                            if (ln)
                                hipLaunchKernelGGL((kb_cg_b<T, V, true, WT, PB, WT == 4>), gb, bb, 0, s, dev, L.n);
                            else
                                hipLaunchKernelGGL((kb_cg_b<T, V, true, WT, PB, false>), gb, bb, 0, s, dev, L.n);
                        } else {
                            if (ln)
                                hipLaunchKernelGGL((kb_cg_b<T, V, false, WT, PB, WT == 4>), gb, bb, 0, s, dev, L.n);
                            else
                                hipLaunchKernelGGL((kb_cg_b<T, V, false, WT, PB, false>), gb, bb, 0, s, dev, L.n);
                        }
                    });
                    fold_percol(L, 1);
                    if (PRE == 1) fold_percol(L, 2);
                });
            });
            pre_pass(L);
        }
    };
    // Graph replay: the key of every captured argument (see graph_cache).
    KeyBuf key;
    int dev = 0;
    if (launch_mode == FVX_LAUNCH_GRAPH) {
        FVX_HIP(hipGetDevice(&dev));
        key.u(dev);
        key.u(sizeof(T));
        key.p(items_dev);
        key.u(pc.kind);
        key.u(pc.degree);
        key.u(pc.amg ? int64_t(pc.amg->serial) : 0);
        key.d(pc.inv_theta);
        for (double c : pc.c1) key.d(c);
        for (double c : pc.c2) key.d(c);
        for (const CgJob<T> &J : jobs) {
            key.u(int64_t(J.op->serial));
            for (int t = 0; t < 2; ++t) {
                key.tile(J.op->tile[t]);
                key.tile(J.op->cg_tile[t]);
            }
            // The state by value (the V-cycle's last step takes it); its
            // rtol2 is read from the descriptors only, so it is left out.
            const CgDev &d = J.d;
            for (const void *q : {(const void *)d.st, (const void *)d.rho, (const void *)d.active,
                                  (const void *)d.alpha, (const void *)d.bnorm2, (const void *)d.r0,
                                  (const void *)d.rho_last, (const void *)d.iters, (const void *)d.part_a,
                                  (const void *)d.part_b, (const void *)d.tot, (const void *)d.mean,
                                  (const void *)J.r, (const void *)J.z0, (const void *)J.z1})
                key.p(q);
            key.u(d.G);
            key.u(d.percol);
            key.u(d.count);
            key.p(pc.kind == 3 ? (const void *)amg_output<T>(pc.amg, *J.amgw) : nullptr);
        }
        for (const Launch &L : launches) {
            for (int x : {L.key.block, L.key.vec, L.key.z, L.key.w, L.key.lines, L.offset, L.n, L.blocks}) key.u(x);
            for (int j : L.jobs) key.u(j);
        }
    }
    // Replays `count` iterations from the cached graphs (binary decomposition
    // of count), capturing each size on first use.
    auto replay = [&](int count) {
        GraphCache &gc = graph_cache();
        std::lock_guard<std::mutex> lk(gc.mu);
        GraphSet &g = graph_set(gc, key.v, dev);
        for (int j = kGraphSizes - 1; j >= 0; --j) {
            const int m = 1 << j;
            while (count >= m) {
                if (!g.ex[j])
                    g.ex[j] = capture_graph(gc, s, [&] {
                        for (int i = 0; i < m; ++i) iteration();
                    });
                FVX_HIP(hipGraphLaunch(g.ex[j], s));
                count -= m;
            }
        }
    };
    int it = 0, next = std::min(poll, 8);
    std::vector<int> it_prev(jobs.size(), 0);
    std::vector<double> r2_prev(jobs.size(), 1.0);
    while (true) {
        const int batch = std::min(next, std::max(1, max_iter + 1 - it));
        // The first interval runs launch by launch in either mode (it also
        // settles every lazily chosen tile before anything is captured).
        if (launch_mode == FVX_LAUNCH_GRAPH && it > 0)
            replay(batch);
        else
            for (int i = 0; i < batch; ++i) iteration();
        it += batch;
        FVX_HIP(hipGetLastError());
        bool all_done = true;
        const int nj = int(jobs.size());
        std::vector<PollRec> rec(nj);
        hipLaunchKernelGGL(kb_done<T>, dim3(unsigned(ceil_div(nj, 256))), dim3(256), 0, s, items_dev, nj, flags_dev);
        FVX_HIP(hipGetLastError());
        FVX_HIP(hipMemcpyAsync(rec.data(), flags_dev, sizeof(PollRec) * size_t(nj), hipMemcpyDeviceToHost, s));
        FVX_HIP(hipStreamSynchronize(s));
        for (const auto &r : rec) all_done &= r.done != 0;
        if (all_done || it > max_iter) break;
        // items_dev is ordered by launch group; map back to jobs.
        next = 1;
        int slot = 0;
        for (const Launch &L : launches)
            for (int j : L.jobs) {
                const PollRec &r = rec[slot++];
                if (r.done) continue;
                const double target = jobs[j].rtol * jobs[j].rtol;
                const int span = it - it_prev[j];
                int need = poll;
                if (span > 0 && r.r2 > 0.0 && r2_prev[j] > 0.0 && r.r2 < r2_prev[j]) {
                    const double per = std::log(r.r2 / r2_prev[j]) / span;  // log decay per iteration (< 0)
                    const double rem = std::log(target / r.r2) / per;
                    if (std::isfinite(rem)) need = int(std::min<double>(poll, std::max(0.0, std::ceil(rem)) + 1.0));
                }
                next = std::max(next, need);
                it_prev[j] = it;
                r2_prev[j] = r.r2;
            }
    }
}

// x projection (singular L) and the FP64 true residual per group; returns
// ||bp - L x||^2 per group.
std::vector<double> finish_f64(const fvx_op *op, CgDev d, double *x, const double *bp, double *q, hipStream_t s) {
    Ctx<double> c(op);
    const int nb = c.g.n_blocks;
    std::vector<double> out;
    by_v<double>(c.t.vec, [&](auto Vt) {
        constexpr int V = decltype(Vt)::value;
        Src mean{nullptr, 0};
        if (op->singular) {
            hipLaunchKernelGGL((k_sum<double, V>), c.grid, c.block, 0, s, c.a, d, x, d.part_a);
            mean = fold_or_direct(d, d.part_a, 1, nb, 0, d.tot + 3 * d.G, s);
        }
        hipLaunchKernelGGL((k_fix_x<double, V>), c.grid, c.block, 0, s, c.a, d, mean, int(op->singular), x);
        launch_lap<double>(op, x, q, nullptr, s);
        hipLaunchKernelGGL((k_resid<double, V>), c.grid, c.block, 0, s, c.a, d, bp, q, (double *)nullptr, d.part_b);
        FVX_HIP(hipGetLastError());
        auto t = host_totals(d, d.part_b, 2, nb, s);
        out.assign(t.begin(), t.begin() + d.G);
    });
    return out;
}

void fill_stats(fvx_solve_stats *st, const HostScalars &h, const std::vector<double> &res2, int status) {
    if (!st) return;
    st->status = status;
    st->iters = 0;
    st->relres_rec = st->relres_true = st->r0_over_b = st->bnorm = 0.0;
    for (size_t g = 0; g < h.bnorm2.size(); ++g) {
        st->iters = std::max(st->iters, h.iters[g]);
        const double bb = h.bnorm2[g];
        if (bb > 0.0) {
            st->relres_rec = std::max(st->relres_rec, std::sqrt(h.rho_last[g] / bb));
            st->r0_over_b = std::max(st->r0_over_b, std::sqrt(h.r0[g] / bb));
            st->relres_true = std::max(st->relres_true, std::sqrt(res2[g] / bb));
        }
        st->bnorm = std::max(st->bnorm, std::sqrt(bb));
    }
    st->rhs_projected = h.st.rhs_projected;
}

void check_opts(const fvx_op *op, const fvx_solve_opts *o) {
    FVX_REQUIRE(op && o, FVX_E_ARG, "NULL op or options");
    FVX_REQUIRE(op->stencil == 7, FVX_E_UNSUPPORTED, "solves use the 7-point finite-volume operator");
    FVX_REQUIRE(o->rtol > 0 && o->rtol < 1, FVX_E_ARG, "rtol must be in (0, 1)");
    FVX_REQUIRE(o->max_iter >= 1, FVX_E_ARG, "max_iter must be >= 1");
    FVX_REQUIRE(o->precision == FVX_F64 || o->precision == FVX_MIXED, FVX_E_ARG,
                "precision must be FVX_F64 or FVX_MIXED");
    FVX_REQUIRE(o->guess == FVX_GUESS_ZERO || o->guess == FVX_GUESS_GIVEN, FVX_E_ARG, "bad guess mode");
    FVX_REQUIRE(o->poll_every >= 1, FVX_E_ARG, "poll_every must be >= 1");
    FVX_REQUIRE(o->launch == FVX_LAUNCH_PHASES || o->launch == FVX_LAUNCH_GRAPH, FVX_E_ARG, "unknown launch mode");
    FVX_REQUIRE(o->precond == FVX_PRECOND_NONE || o->precond == FVX_PRECOND_JACOBI ||
                    o->precond == FVX_PRECOND_CHEBYSHEV || o->precond == FVX_PRECOND_AMG,
                FVX_E_ARG, "unknown preconditioner");
    if (o->precond == FVX_PRECOND_AMG) amg_check_solve(o->amg, op, o->precision == FVX_MIXED);
    if (o->precond == FVX_PRECOND_CHEBYSHEV)
        FVX_REQUIRE(o->cheb_degree >= 1 && o->cheb_degree <= 16 && o->cheb_ratio > 1.0 && std::isfinite(o->cheb_ratio),
                    FVX_E_ARG, "Chebyshev preconditioner: degree 1..16, ratio > 1");
    if (o->precision == FVX_MIXED) {
        FVX_REQUIRE(op->has_f32, FVX_E_ARG, "mixed precision needs an operator built with FP32 copies");
        FVX_REQUIRE(o->inner_rtol > 0 && o->inner_rtol < 1 && o->max_outer >= 1, FVX_E_ARG,
                    "bad inner_rtol or max_outer");
    }
    if (op->percol)
        FVX_REQUIRE(op->k <= 128, FVX_E_UNSUPPORTED, "independent-plane solves support k <= 128");
}

// One problem of a (possibly single-problem) solve.
struct Problem {
    const fvx_op *op;
    const double *B;
    double *X;
    Workspace w;
    HostScalars h;
    std::vector<double> res2;
    int status = FVX_OK, total_inner = 0, outer = 0;
    bool outer_active = true;
};

void solve_f64_batch(std::vector<Problem> &P, const fvx_solve_opts *o, BItem<double> *items, PollRec *flags,
                     hipStream_t s) {
    std::vector<CgJob<double>> jobs;
    for (auto &p : P)
        jobs.push_back(CgJob<double>{p.op, p.w.outer, p.B, p.X, p.w.bp, p.w.r, p.w.p0, p.w.p1, p.w.q,
                                     o->guess == FVX_GUESS_GIVEN, o->rtol, o->max_iter, p.w.z[0], p.w.z[1]});
    for (size_t i = 0; i < P.size(); ++i) jobs[i].amgw = &P[i].w.amg64;
    run_cg_batch<double>(jobs, items, flags, o->poll_every, make_precond(o), o->launch, s);
    for (auto &p : P) {
        p.h = read_state(p.w.outer, s);
        p.res2 = finish_f64(p.op, p.w.outer, p.X, p.w.bp, p.w.q, s);
        p.status = p.h.st.status;
    }
}

// Mixed precision for every problem: FP64 outer defect correction with an
// FP32-SpMM inner CG (FP64 dot products and scalars).  Each problem takes the
// same steps and decisions as when solved alone; the inner CGs of all problems
// still iterating run as one batch.
void solve_mixed_batch(std::vector<Problem> &P, const fvx_solve_opts *o, BItem<float> *items, PollRec *flags,
                       hipStream_t s) {
    for (auto &p : P) {
        CgDev D = p.w.outer;
        const fvx_op *op = p.op;
        Ctx<double> c(op);
        const int nb = c.g.n_blocks, G = D.G;
        reset_state(D, o->max_iter, s);
        p.h.bnorm2.assign(G, 0.0);
        p.h.r0.assign(G, 0.0);
        p.h.rho_last.assign(G, 0.0);
        p.h.iters.assign(G, 0);
        by_v<double>(c.t.vec, [&](auto Vt) {
            constexpr int V = decltype(Vt)::value;
            Src mean{nullptr, 0};
            if (op->singular) {
                hipLaunchKernelGGL((k_sum<double, V>), c.grid, c.block, 0, s, c.a, D, p.B, D.part_a);
                mean = fold_or_direct(D, D.part_a, 1, nb, 0, D.tot + 3 * G, s);
            }
            const bool given = o->guess == FVX_GUESS_GIVEN;
            if (given) launch_lap<double>(op, p.X, p.w.q, nullptr, s);
            hipLaunchKernelGGL((k_cg_init<double, V, 0>), c.grid, c.block, 0, s, c.a, D, mean, int(op->singular),
                               p.B, p.w.bp, p.X, p.w.r, p.w.q, int(given));
            FVX_HIP(hipGetLastError());
        });
        const auto t0 = host_totals(D, D.part_b, 2, nb, s);
        p.h.st = read_state(D, s).st;
        for (int g = 0; g < G; ++g) {
            p.h.bnorm2[g] = t0[G + g];
            p.h.r0[g] = t0[g];
            if (!std::isfinite(t0[g]) || !std::isfinite(t0[G + g])) p.status = FVX_E_NONFINITE;
        }
        if (p.h.st.status < 0) p.status = p.h.st.status;
        // The final projection reads ||b||^2 per group on the device.
        FVX_HIP(hipMemcpyAsync(D.bnorm2, p.h.bnorm2.data(), 8 * G, hipMemcpyHostToDevice, s));
        FVX_HIP(hipStreamSynchronize(s));
        if (p.status < 0) p.outer_active = false;
    }
    while (true) {
        // FP64 outer residual r = bp - L x, its norm and plain mean per group.
        std::vector<CgJob<float>> jobs;
        std::vector<Problem *> in_jobs;
        for (auto &p : P) {
            if (!p.outer_active) continue;
            CgDev D = p.w.outer;
            const fvx_op *op = p.op;
            Ctx<double> c(op);
            const int nb = c.g.n_blocks, G = D.G;
            std::vector<double> gmean(G), gact(G);
            bool any = false;
            double need = 0.5;  // inner reduction the outer target still needs
            by_v<double>(c.t.vec, [&](auto Vt) {
                constexpr int V = decltype(Vt)::value;
                launch_lap<double>(op, p.X, p.w.q, nullptr, s);
                hipLaunchKernelGGL((k_resid<double, V>), c.grid, c.block, 0, s, c.a, D, p.w.bp, p.w.q, p.w.r,
                                   D.part_b);
                FVX_HIP(hipGetLastError());
                const auto t = host_totals(D, D.part_b, 2, nb, s);
                for (int g = 0; g < G; ++g) {
                    p.h.rho_last[g] = t[g];
                    const bool act = p.h.bnorm2[g] > 0.0 && t[g] > o->rtol * o->rtol * p.h.bnorm2[g];
                    gact[g] = act ? 1.0 : 0.0;
                    if (act) need = std::min(need, 0.5 * o->rtol * std::sqrt(p.h.bnorm2[g] / t[g]));
                    gmean[g] = op->singular ? t[G + g] / double(D.count) : 0.0;
                    any |= act;
                    if (!std::isfinite(t[g])) p.status = FVX_E_NONFINITE;
                }
                if (p.status < 0 || !any) {
                    p.outer_active = false;
                    return;
                }
                if (p.outer >= o->max_outer || p.total_inner >= o->max_iter) {
                    p.status = FVX_NOT_CONVERGED;
                    p.outer_active = false;
                    return;
                }
                FVX_HIP(hipMemcpyAsync(p.w.gmean, gmean.data(), 8 * G, hipMemcpyHostToDevice, s));
                FVX_HIP(hipMemcpyAsync(p.w.gact, gact.data(), 8 * G, hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL((k_to_inner<V>), c.grid, c.block, 0, s, c.a, D, p.w.r, p.w.gmean, p.w.gact, p.w.b32);
                FVX_HIP(hipGetLastError());
                FVX_HIP(hipStreamSynchronize(s));  // gmean/gact host buffers are reused next pass
            });
            if (!p.outer_active) continue;
            const int budget = std::max(1, o->max_iter - p.total_inner);
            // The inner tolerance is inner_rtol, loosened in a last correction
            // to half of what separates the outer residual from its target.
            const double inner_rtol = std::max(o->inner_rtol, need);
            jobs.push_back(CgJob<float>{op, p.w.inner, p.w.b32, p.w.x32, p.w.bp32, p.w.r32, p.w.p32a, p.w.p32b,
                                        p.w.q32, false, inner_rtol, budget, p.w.z32[0], p.w.z32[1], &p.w.amg32});
            in_jobs.push_back(&p);
        }
        if (jobs.empty()) break;
        run_cg_batch<float>(jobs, items, flags, o->poll_every, make_precond(o), o->launch, s);
        for (Problem *pp : in_jobs) {
            Problem &p = *pp;
            const auto hi = read_state(p.w.inner, s);
            int it = 0;
            for (auto v : hi.iters) it = std::max(it, v);
            p.total_inner += it;
            if (hi.st.status < 0) {
                p.status = hi.st.status;
                p.outer_active = false;
                continue;
            }
            Ctx<double> c(p.op);
            by_v<double>(c.t.vec, [&](auto Vt) {
                constexpr int V = decltype(Vt)::value;
                hipLaunchKernelGGL((k_add_inner<V>), c.grid, c.block, 0, s, c.a, p.X, p.w.x32);
            });
            FVX_HIP(hipGetLastError());
            ++p.outer;
        }
    }
    for (auto &p : P) {
        p.res2 = finish_f64(p.op, p.w.outer, p.X, p.w.bp, p.w.q, s);
        p.h.st.status = p.status;
    }
}

// Workspace of a batch: the item descriptors, then each problem's workspace.
struct BatchLayout {
    size_t items64, items32, flags, total;
    std::vector<size_t> offs;
};

BatchLayout batch_layout(int n, const fvx_op *const *ops, bool mixed, bool cheb, const fvx_amg *amg) {
    BatchLayout L;
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += (b + 255) / 256 * 256;
        return o;
    };
    L.items64 = take(sizeof(BItem<double>) * size_t(n));
    L.items32 = take(sizeof(BItem<float>) * size_t(n));
    L.flags = take(sizeof(PollRec) * size_t(n));
    for (int i = 0; i < n; ++i) L.offs.push_back(take(carve(nullptr, ops[i], mixed, cheb, amg).bytes));
    L.total = off;
    return L;
}

int solve_batch(int n, const fvx_op *const *ops, const double *const *B, double *const *X, const fvx_solve_opts *o,
                void *ws, size_t ws_bytes, fvx_solve_stats *stats, hipStream_t s) {
    FVX_REQUIRE(n >= 1 && ops && B && X && ws, FVX_E_ARG, "NULL argument or empty batch");
    FVX_REQUIRE(reinterpret_cast<uintptr_t>(ws) % 256 == 0, FVX_E_ARG, "ws must be 256-byte aligned");
    for (int i = 0; i < n; ++i) {
        check_opts(ops[i], o);
        FVX_REQUIRE(B[i] && X[i], FVX_E_ARG, "NULL B[i] or X[i]");
        FVX_REQUIRE(reinterpret_cast<uintptr_t>(B[i]) % 16 == 0 && reinterpret_cast<uintptr_t>(X[i]) % 16 == 0,
                    FVX_E_ARG, "B[i] and X[i] must be 16-byte aligned");
    }
    const bool mixed = o->precision == FVX_MIXED;
    const bool cheb = make_precond(o).kind == 2;
    const fvx_amg *amg = make_precond(o).kind == 3 ? o->amg : nullptr;
    FVX_REQUIRE(!amg || n == 1, FVX_E_ARG, "the multigrid preconditioner serves single solves");
    const BatchLayout L = batch_layout(n, ops, mixed, cheb, amg);
    FVX_REQUIRE(ws_bytes >= L.total, FVX_E_NOMEM, "workspace too small: need " + std::to_string(L.total));
    char *base = static_cast<char *>(ws);
    std::vector<Problem> P(n);
    for (int i = 0; i < n; ++i) {
        P[i].op = ops[i];
        P[i].B = B[i];
        P[i].X = X[i];
        P[i].w = carve(base + L.offs[i], ops[i], mixed, cheb, amg);
    }
    if (mixed)
        solve_mixed_batch(P, o, reinterpret_cast<BItem<float> *>(base + L.items32),
                          reinterpret_cast<PollRec *>(base + L.flags), s);
    else
        solve_f64_batch(P, o, reinterpret_cast<BItem<double> *>(base + L.items64),
                        reinterpret_cast<PollRec *>(base + L.flags), s);
    int worst = FVX_OK;
    for (int i = 0; i < n; ++i) {
        fill_stats(stats ? &stats[i] : nullptr, P[i].h, P[i].res2, P[i].status);
        if (stats) {
            stats[i].outer = mixed ? P[i].outer : 0;
            if (mixed) stats[i].iters = P[i].total_inner;
        }
        if (P[i].status < 0 && (worst >= 0 || P[i].status < worst)) worst = P[i].status;
        if (P[i].status > 0 && worst == FVX_OK) worst = P[i].status;
    }
    return worst;
}

// The scratch of fvx_poisson_solve_noalloc: a file-scope device array of a
// fixed size (each device holds its own copy for the life of the process).
// Host code never passes the array's name to a kernel or a copy: the name is
// a host-side stand-in, not a device address.  The device address is looked
// up once per device, with that device current, and kept.
__device__ __align__(256) char scratch[FVX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

void *noalloc_scratch() {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    FVX_HIP(hipGetDevice(&dev));
    FVX_REQUIRE(dev >= 0 && dev < kMaxDevices, FVX_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        FVX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        FVX_REQUIRE(p && reinterpret_cast<uintptr_t>(p) % 256 == 0, FVX_E_HIP, "scratch address lookup failed");
        addr[dev] = p;
    }
    return addr[dev];
}

}  // namespace

double guess_residual_ratio(const fvx_op *op, const double *B, const double *X, void *ws, hipStream_t s) {
    const Workspace w = carve(ws, op, false, false);
    const CgDev D = w.outer;
    const Ctx<double> c(op);
    const int nb = c.g.n_blocks;
    reset_state(D, 1, s);
    by_v<double>(c.t.vec, [&](auto Vt) {
        constexpr int V = decltype(Vt)::value;
        Src mean{nullptr, 0};
        if (op->singular) {
            hipLaunchKernelGGL((k_sum<double, V>), c.grid, c.block, 0, s, c.a, D, B, D.part_a);
            mean = fold_or_direct(D, D.part_a, 1, nb, 0, D.tot + 3 * D.G, s);
        }
        launch_lap<double>(op, X, w.q, nullptr, s);
        // given = 1: x is only read.
        hipLaunchKernelGGL((k_cg_init<double, V, 0>), c.grid, c.block, 0, s, c.a, D, mean, int(op->singular), B,
                           w.bp, const_cast<double *>(X), w.r, w.q, 1);
        FVX_HIP(hipGetLastError());
    });
    const auto t = host_totals(D, D.part_b, 2, nb, s);
    double worst = 0.0;
    for (int g = 0; g < D.G; ++g) {
        const double rr = t[g], bb = t[D.G + g];
        if (!std::isfinite(rr) || !std::isfinite(bb)) return INFINITY;
        if (bb > 0.0)
            worst = std::max(worst, std::sqrt(rr / bb));
        else if (rr > 0.0)
            return INFINITY;
    }
    return worst;
}

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
    o->precond = FVX_PRECOND_NONE;
    o->cheb_degree = 8;
    o->cheb_ratio = 300.0;
    o->amg = nullptr;
    o->launch = FVX_LAUNCH_GRAPH;
    return FVX_OK;
}

int fvx_solve_bytes(const fvx_op *op, const fvx_solve_opts *o, size_t *bytes) {
    return guard([&] {
        fvx::check_opts(op, o);
        FVX_REQUIRE(bytes, FVX_E_ARG, "bytes is NULL");
        const fvx_op *ops[1] = {op};
        const fvx::Precond pc = fvx::make_precond(o);
        *bytes = fvx::batch_layout(1, ops, o->precision == FVX_MIXED, pc.kind == 2, pc.kind == 3 ? o->amg : nullptr)
                     .total;
        return FVX_OK;
    });
}

int fvx_poisson_solve(const fvx_op *op, const double *B, double *X, const fvx_solve_opts *o, void *ws,
                      size_t ws_bytes, fvx_solve_stats *stats, void *stream) {
    return guard([&] {
        const auto t0 = std::chrono::steady_clock::now();
        const fvx_op *ops[1] = {op};
        const double *Bs[1] = {B};
        double *Xs[1] = {X};
        const int rc = fvx::solve_batch(1, ops, Bs, Xs, o, ws, ws_bytes, stats, fvx::as_stream(stream));
        if (stats) stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (rc < 0) throw fvx::Error(rc, fvx_status_str(rc));
        return rc;
    });
}

int fvx_poisson_solve_noalloc(const fvx_op *op, const double *B, double *X, const fvx_solve_opts *o,
                              fvx_solve_stats *stats, void *stream) {
    return guard([&] {
        const auto t0 = std::chrono::steady_clock::now();
        FVX_REQUIRE(op && o, FVX_E_ARG, "NULL argument");
        const fvx_op *ops[1] = {op};
        const fvx::Precond pc = fvx::make_precond(o);
        fvx::check_opts(op, o);
        const size_t need =
            fvx::batch_layout(1, ops, o->precision == FVX_MIXED, pc.kind == 2, pc.kind == 3 ? o->amg : nullptr).total;
        FVX_REQUIRE(need <= FVX_NOALLOC_SCRATCH_BYTES, FVX_E_NOMEM,
                    "fvx_poisson_solve_noalloc: this solve needs " + std::to_string(need) +
                        " bytes of scratch; the library's built-in scratch holds " +
                        std::to_string(size_t(FVX_NOALLOC_SCRATCH_BYTES)));
        void *ws = fvx::noalloc_scratch();
        const double *Bs[1] = {B};
        double *Xs[1] = {X};
        fvx_solve_opts phases = *o;  // graph capture allocates: launch phase by phase
        phases.launch = FVX_LAUNCH_PHASES;
        const int rc = fvx::solve_batch(1, ops, Bs, Xs, &phases, ws, FVX_NOALLOC_SCRATCH_BYTES, stats,
                                        fvx::as_stream(stream));
        if (stats) stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (rc < 0) throw fvx::Error(rc, fvx_status_str(rc));
        return rc;
    });
}

int fvx_solve_batch_bytes(int n, const fvx_op *const *ops, const fvx_solve_opts *o, size_t *bytes) {
    return guard([&] {
        FVX_REQUIRE(n >= 1 && ops && bytes, FVX_E_ARG, "bad argument");
        for (int i = 0; i < n; ++i) fvx::check_opts(ops[i], o);
        const fvx::Precond pc = fvx::make_precond(o);
        FVX_REQUIRE(pc.kind != 3 || n == 1, FVX_E_ARG, "the multigrid preconditioner serves single solves");
        *bytes = fvx::batch_layout(n, ops, o->precision == FVX_MIXED, pc.kind == 2, pc.kind == 3 ? o->amg : nullptr)
                     .total;
        return FVX_OK;
    });
}

int fvx_poisson_solve_batch(int n, const fvx_op *const *ops, const double *const *B, double *const *X,
                            const fvx_solve_opts *o, void *ws, size_t ws_bytes, fvx_solve_stats *stats, void *stream) {
    return guard([&] {
        const auto t0 = std::chrono::steady_clock::now();
        const int rc = fvx::solve_batch(n, ops, B, X, o, ws, ws_bytes, stats, fvx::as_stream(stream));
        const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (stats)
            for (int i = 0; i < n; ++i) stats[i].seconds = sec;
        return rc;
    });
}

}  // extern "C"

extern "C" {

int fvx_op_get_cg_tile(const fvx_op *op, int dtype, fvx_tile *tile) {
    return guard([&] {
        FVX_REQUIRE(op && tile, FVX_E_ARG, "NULL argument");
        FVX_REQUIRE(dtype == FVX_F64 || (dtype == FVX_F32 && op->has_f32), FVX_E_ARG, "bad dtype for this op");
        *tile = dtype == FVX_F64 ? fvx::cg_tile<double>(op) : fvx::cg_tile<float>(op);
        return FVX_OK;
    });
}

int fvx_op_set_cg_tile(fvx_op *op, int dtype, const fvx_tile *tile) {
    return guard([&] {
        FVX_REQUIRE(op, FVX_E_ARG, "op is NULL");
        FVX_REQUIRE(dtype == FVX_F64 || (dtype == FVX_F32 && op->has_f32), FVX_E_ARG, "bad dtype for this op");
        if (!tile || tile->block == 0) {
            op->cg_tile[dtype] = fvx_tile{};
            return FVX_OK;
        }
        // stage_lds of a CG tile selects line tiles (no LDS stage): validate
        // the rest like an SpMM tile
        fvx_tile chk = *tile;
        FVX_REQUIRE(chk.stage_lds == 0 || chk.stage_lds == 1, FVX_E_ARG, "CG tile stage_lds (line tiles) must be 0 or 1");
        chk.stage_lds = 0;
        fvx::check_tile(op, dtype, chk);
        FVX_REQUIRE(tile->block <= (op->percol ? fvx::kMaxPercolBlock : fvx::kMaxCgBlock), FVX_E_ARG,
                    "CG tile block too large (512, or 256 for independent planes)");
        op->cg_tile[dtype] = *tile;
        return FVX_OK;
    });
}

int fvx_tune_cg_bytes(const fvx_op *op, int dtype, size_t *bytes) {
    return guard([&]() -> int {
        FVX_REQUIRE(op && bytes, FVX_E_ARG, "NULL argument");
        fvx_solve_opts o{};
        fvx_solve_opts_default(&o);
        o.precision = dtype == FVX_F32 ? FVX_MIXED : FVX_F64;
        size_t ws = 0;
        const int rc = fvx_solve_bytes(op, &o, &ws);
        if (rc != FVX_OK) return rc;
        const size_t v = (sizeof(double) * size_t(op->n_b) * op->ld + 255) / 256 * 256;
        *bytes = (ws + 255) / 256 * 256 + 2 * v;
        return FVX_OK;
    });
}

int fvx_tune_cg(fvx_op *op, int dtype, void *ws, size_t ws_bytes, int iters, void *stream,
                fvx_tune_result *results, int max_results, int *n_results) {
    return guard([&]() -> int {
        FVX_REQUIRE(op && ws, FVX_E_ARG, "NULL op or workspace");
        FVX_REQUIRE(dtype == FVX_F64 || (dtype == FVX_F32 && op->has_f32), FVX_E_ARG, "bad dtype for this op");
        FVX_REQUIRE(reinterpret_cast<uintptr_t>(ws) % 256 == 0, FVX_E_ARG, "ws must be 256-byte aligned");
        iters = std::max(8, iters);
        size_t need = 0;
        const int q = fvx_tune_cg_bytes(op, dtype, &need);
        if (q != FVX_OK) return q;
        FVX_REQUIRE(ws_bytes >= need, FVX_E_NOMEM, "workspace too small: need " + std::to_string(need));
        fvx_solve_opts o{};
        fvx_solve_opts_default(&o);
        o.precision = dtype == FVX_F32 ? FVX_MIXED : FVX_F64;
        o.rtol = 1e-300;  // never met: every timed solve runs `iters` CG iterations
        o.inner_rtol = 1e-300;
        o.max_outer = 1;
        o.max_iter = iters;
        o.poll_every = iters;
        o.launch = FVX_LAUNCH_PHASES;  // the kernels' own time
        size_t sws = 0;
        fvx_solve_bytes(op, &o, &sws);
        sws = (sws + 255) / 256 * 256;
        const size_t v = (sizeof(double) * size_t(op->n_b) * op->ld + 255) / 256 * 256;
        double *B = reinterpret_cast<double *>(static_cast<char *>(ws) + sws);
        double *X = reinterpret_cast<double *>(static_cast<char *>(ws) + sws + v);
        hipStream_t s = fvx::as_stream(stream);
        const int64_t n = int64_t(op->n_b) * op->ld;
        hipLaunchKernelGGL(fvx::k_fill_pattern, dim3(1024), dim3(256), 0, s, B, n);
        FVX_HIP(hipGetLastError());
        // Candidates: the widest vector, one pass per row group, and the block
        // size, XCD remap and grid cap that the CG kernels are sensitive to.
        const fvx_tile base = fvx::default_tile(op, dtype);
        std::vector<fvx_tile> cands;
        for (int block : {128, 256, 512}) {
            if (op->percol && block > fvx::kMaxPercolBlock) continue;
            if (block < base.lanes_per_row) continue;
            for (int remap : {1, 0})
                for (int cap : {1024, 512, 2048})
                    for (int lines : {0, 1}) {
                        fvx_tile t = base;
                        t.block = block;
                        t.xcd_remap = remap;
                        t.max_blocks = cap;
                        t.stage_lds = lines;
                        t.nt_store = 0;
                        const bool ok = dtype == FVX_F64 ? fvx::cg_lines_ok<double>(op, t) : fvx::cg_lines_ok<float>(op, t);
                        if (lines && !ok) continue;
                        cands.push_back(t);
                    }
        }
        if (cands.empty()) cands.push_back(base);
        const fvx_tile keep = op->cg_tile[dtype];
        fvx_tile best = cands[0];
        double best_us = 1e300;
        int count = 0;
        try {
            for (const fvx_tile &t : cands) {
                op->cg_tile[dtype] = t;
                fvx_solve_stats st{};
                double us = 1e300;
                for (int rep = 0; rep < 3; ++rep) {
                    const int rc = fvx_poisson_solve(op, B, X, &o, ws, sws, &st, stream);
                    FVX_REQUIRE(rc >= 0, rc, "CG tile timing solve failed");
                    if (rep > 0) us = std::min(us, 1e6 * st.seconds / double(std::max(1, st.iters)));
                }
                if (results && count < max_results) results[count] = fvx_tune_result{t, us};
                ++count;
                // line tiles split launch groups in a batch and use twice the
                // registers: taken only on a clear win over the best so far
                if (us < (t.stage_lds ? 0.95 : 1.0) * best_us) {
                    best_us = us;
                    best = t;
                }
            }
        } catch (...) {
            op->cg_tile[dtype] = keep;
            throw;
        }
        op->cg_tile[dtype] = best;
        if (n_results) *n_results = count;
        return FVX_OK;
    });
}

}  // extern "C"
