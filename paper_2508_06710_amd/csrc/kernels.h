// Device-side building blocks shared by the HIP translation units: vector
// loads, the XCD-aware tile order, and the per-row SpMM bodies.
#pragma once

#include "common.h"

namespace fvx {

template <typename T, int V>
using vec_t = T __attribute__((ext_vector_type(V)));

template <typename T, int V>
__device__ __forceinline__ vec_t<T, V> ldv(const T *p) {
    return *reinterpret_cast<const vec_t<T, V> *>(p);
}

// Store of the first `valid` of V values; NT marks full-vector stores
// non-temporal (the output is not read again by this kernel).  NT is a
// compile-time choice: a run-time flag lets the compiler merge the two stores
// and drop the hint.
template <typename T, int V, bool NT = false>
__device__ __forceinline__ void stv_masked(T *p, const vec_t<T, V> &v, int valid) {
    if (valid >= V) {
        if constexpr (NT)
            __builtin_nontemporal_store(v, reinterpret_cast<vec_t<T, V> *>(p));
        else
            *reinterpret_cast<vec_t<T, V> *>(p) = v;
    } else {
#pragma unroll
        for (int t = 0; t < V; ++t)
            if (t < valid) p[t] = v[t];
    }
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remapping hardware block b to a logical tile index so that the blocks
// of one XCD take one contiguous range of rows keeps the neighbour rows a
// block gathers in the L2 that already holds them.  A bijection on [0, n).
__device__ __forceinline__ int64_t logical_block_of(int b, int n, int remap) {
    if (!remap || n < 8) return b;
    const int xcd = b & 7, local = b >> 3;
    const int q = n >> 3, r = n & 7;
    return xcd < r ? int64_t(xcd) * (q + 1) + local : int64_t(r) * (q + 1) + int64_t(xcd - r) * q + local;
}

__device__ __forceinline__ int64_t logical_block(int remap) { return logical_block_of(blockIdx.x, gridDim.x, remap); }

// Values of the neighbouring planes of this lane's V columns, l-1 and l+1
// (mod k), taken from the row-group lanes that hold them when all k columns
// of the row sit in one pass of the group (lanes_per_row * V >= k).
template <typename T, int V>
struct PlaneNeighbours {
    T left0;   // value of column c0 - 1 (mod k)
    T rightV;  // value of column c0 + V (or column 0 past the last column)
};

template <typename T, int V>
__device__ __forceinline__ PlaneNeighbours<T, V> plane_neighbours(const vec_t<T, V> &xo, int sub, int lpr, int k) {
    const int last = (k - 1) / V;  // lane of the row group holding column k-1
    const int src_r = sub == last ? 0 : sub + 1;
    const int src_l = sub == 0 ? last : sub - 1;
    const T prov_l = sub == last ? xo[(k - 1) % V] : xo[V - 1];
    PlaneNeighbours<T, V> n;
    n.rightV = __shfl(xo[0], src_r, lpr);
    n.left0 = __shfl(prov_l, src_l, lpr);
    return n;
}

// The same two values when the row group covers the k columns in several
// passes (lanes_per_row * V < k): from the neighbouring lanes of this pass,
// and from memory for the lanes at the edges of the pass.  Lanes past column
// k in the last pass are inactive; no active lane uses their values.
template <typename T, int V, class Ld>
__device__ __forceinline__ PlaneNeighbours<T, V> plane_neighbours_pass(const vec_t<T, V> &xo, const Ld &in,
                                                                       int64_t row, int c0, int sub, int lpr, int k) {
    const T l = __shfl(xo[V - 1], sub == 0 ? lpr - 1 : sub - 1, lpr);
    const T r = __shfl(xo[0], sub == lpr - 1 ? 0 : sub + 1, lpr);
    PlaneNeighbours<T, V> n;
    n.left0 = sub == 0 ? in.scalar(row, c0 == 0 ? k - 1 : c0 - 1) : l;
    n.rightV = (sub == lpr - 1 || c0 + V >= k) ? in.scalar(row, c0 + V >= k ? 0 : c0 + V) : r;
    return n;
}

template <typename T, int V, class Ld>
__device__ __forceinline__ PlaneNeighbours<T, V> neighbours_of(const vec_t<T, V> &xo, const Ld &in, int64_t row,
                                                               int c0, int sub, int lpr, int k, bool single) {
    return single ? plane_neighbours<T, V>(xo, sub, lpr, k) : plane_neighbours_pass<T, V>(xo, in, row, c0, sub, lpr, k);
}

// Column l-1 (mod k) and l+1 (mod k) of element t of this lane.
template <typename T, int V>
__device__ __forceinline__ T left_of(const vec_t<T, V> &xo, const PlaneNeighbours<T, V> &n, int t) {
    return t > 0 ? xo[t > 0 ? t - 1 : 0] : n.left0;
}
template <typename T, int V>
__device__ __forceinline__ T right_of(const vec_t<T, V> &xo, const PlaneNeighbours<T, V> &n, int t, int l,
                                      int k) {
    return (l == k - 1 || t + 1 >= V) ? n.rightV : xo[t + 1 < V ? t + 1 : 0];
}

// Row loaders: how a lap SpMM reads its input multivector.  PlainLoad reads
// X; DirLoad forms the CG search direction r + beta p on the fly (beta per
// column), so the SpMM and the direction update share one pass.
template <typename T, int V>
struct PlainLoad {
    const T *__restrict__ X;
    int ld;
    __device__ __forceinline__ vec_t<T, V> vec(int64_t row, int c0) const { return ldv<T, V>(X + row * ld + c0); }
    __device__ __forceinline__ T scalar(int64_t row, int l) const { return X[row * ld + l]; }
};

template <typename T, int V>
struct DirLoad {
    const T *__restrict__ R;
    const T *__restrict__ P;
    int ld;
    vec_t<T, V> beta;  // beta of this lane's V columns (equal entries when global)
    // one fused multiply-add per element, in the vector and the scalar form
    // alike: a neighbour's p' formed here equals the p' its owner stores
    __device__ __forceinline__ vec_t<T, V> vec(int64_t row, int c0) const {
        return __builtin_elementwise_fma(beta, ldv<T, V>(P + row * ld + c0), ldv<T, V>(R + row * ld + c0));
    }
    __device__ __forceinline__ T scalar(int64_t row, int l) const {
        return __builtin_elementwise_fma(beta[0], P[row * ld + l], R[row * ld + l]);
    }
};

// Direction of preconditioned CG with the Jacobi preconditioner formed on the
// fly: p' = D^-1 r + beta p, D^-1 per base row (shared by the planes).
template <typename T, int V>
struct DirLoadJ {
    const T *__restrict__ R;
    const T *__restrict__ P;
    const T *__restrict__ Dinv;
    int ld;
    vec_t<T, V> beta;
    __device__ __forceinline__ vec_t<T, V> vec(int64_t row, int c0) const {
        return __builtin_elementwise_fma(beta, ldv<T, V>(P + row * ld + c0), Dinv[row] * ldv<T, V>(R + row * ld + c0));
    }
    __device__ __forceinline__ T scalar(int64_t row, int l) const {
        return __builtin_elementwise_fma(beta[0], P[row * ld + l], Dinv[row] * R[row * ld + l]);
    }
};

// First Chebyshev iterate z_1 = D^-1 r / theta, formed on the fly.
template <typename T, int V>
struct ChebFirstLoad {
    const T *__restrict__ R;
    const T *__restrict__ Dinv;
    int ld;
    T inv_theta;
    __device__ __forceinline__ vec_t<T, V> vec(int64_t row, int c0) const {
        return (Dinv[row] * inv_theta) * ldv<T, V>(R + row * ld + c0);
    }
    __device__ __forceinline__ T scalar(int64_t row, int l) const { return (Dinv[row] * inv_theta) * R[row * ld + l]; }
};

// One base-block row: its WT off-diagonal column indices and values (padding
// entries point at the row itself with value 0), diagonal, and coupling weight.
template <typename T, int WT>
struct RowMeta {
    int32_t col[WT > 0 ? WT : 1];
    T val[WT > 0 ? WT : 1];
    T diag, w;
};

template <typename T, int WT, bool Z>
__device__ __forceinline__ RowMeta<T, WT> meta_global(const OpDev<T> &A, int64_t n_b, int64_t row) {
    RowMeta<T, WT> m;
#pragma unroll
    for (int e = 0; e < WT; ++e) {
        m.col[e] = A.ell_col[e * n_b + row];
        m.val[e] = A.ell_val[e * n_b + row];
    }
    m.diag = A.diag[row];
    m.w = Z ? A.w[row] : T(0);
    return m;
}

// The same entries on a Cartesian 5-point base: the neighbours' indices from
// (i, j) = (row mod nx, row div nx) (periodic axes wrap, an absent neighbour
// is the row itself) and the coefficients from the row's record
// [diag, w, S, W, E, N, 0, 0] (one 64-byte line in FP64, 32 bytes in FP32).
// The builder writes such an operator's ELL rows in the same S, W, E, N order
// with the same values, so both give the same RowMeta; this one issues 3 (FP64)
// or 2 (FP32) vector loads from one line in place of 10 scattered ones, and the
// gathers wait on no load.
template <typename T, bool Z>
__device__ __forceinline__ RowMeta<T, 4> meta_cart(const OpDev<T> &A, int64_t row) {
    const uint32_t r = uint32_t(row), nx = uint32_t(A.cart_nx), ny = uint32_t(A.cart_ny);
    const uint32_t j = r / nx, i = r - j * nx;
    RowMeta<T, 4> m;
    m.col[0] = int32_t(j > 0 ? r - nx : (A.cart_py ? r + nx * (ny - 1) : r));
    m.col[1] = int32_t(i > 0 ? r - 1 : (A.cart_px ? r + nx - 1 : r));
    m.col[2] = int32_t(i < nx - 1 ? r + 1 : (A.cart_px ? r - (nx - 1) : r));
    m.col[3] = int32_t(j < ny - 1 ? r + nx : (A.cart_py ? r - nx * (ny - 1) : r));
    const T *rec = A.cart + size_t(r) * 8;
    if constexpr (sizeof(T) == 8) {
        const vec_t<T, 2> a = *reinterpret_cast<const vec_t<T, 2> *>(rec);
        const vec_t<T, 2> b = *reinterpret_cast<const vec_t<T, 2> *>(rec + 2);
        const vec_t<T, 2> c = *reinterpret_cast<const vec_t<T, 2> *>(rec + 4);
        m.diag = a[0];
        m.w = Z ? a[1] : T(0);
        m.val[0] = b[0];
        m.val[1] = b[1];
        m.val[2] = c[0];
        m.val[3] = c[1];
    } else {
        const vec_t<T, 4> a = *reinterpret_cast<const vec_t<T, 4> *>(rec);
        const vec_t<T, 4> b = *reinterpret_cast<const vec_t<T, 4> *>(rec + 4);
        m.diag = a[0];
        m.w = Z ? a[1] : T(0);
        m.val[0] = a[2];
        m.val[1] = a[3];
        m.val[2] = b[0];
        m.val[3] = b[1];
    }
    return m;
}

// A row's entries from the Cartesian record when the operator has one (a
// uniform branch), else from the ELL arrays.
template <typename T, int WT, bool Z>
__device__ __forceinline__ RowMeta<T, WT> meta_of(const OpDev<T> &A, int64_t n_b, int64_t row) {
    if constexpr (WT == 4) {
        if (A.cart) return meta_cart<T, Z>(A, row);
    }
    return meta_global<T, WT, Z>(A, n_b, row);
}

// LDS stage of one tile's base-block rows: [rows][WT] columns, [rows][WT]
// values, [rows] diagonal, [rows] coupling weight.
__host__ __device__ constexpr size_t stage_col_bytes(int rows, int wt) {
    return (size_t(rows) * wt * sizeof(int32_t) + 15) / 16 * 16;
}
template <typename T, int WT>
__host__ __device__ constexpr size_t stage_bytes(int rows) {
    return stage_col_bytes(rows, WT) + size_t(rows) * (WT + 2) * sizeof(T);
}

// All threads of the block: copy the rows [row0, row0 + rows) of the base
// block (ELL stride n_b) into the stage with coalesced loads; rows at or past
// n_valid get the padding pattern (column 0, value 0).
template <typename T, int WT, bool Z>
__device__ __forceinline__ void stage_rows(const OpDev<T> &A, int64_t n_b, int64_t n_valid, int64_t row0, int rows,
                                           char *smem) {
    int32_t *s_col = reinterpret_cast<int32_t *>(smem);
    T *s_val = reinterpret_cast<T *>(smem + stage_col_bytes(rows, WT));
    T *s_dw = s_val + size_t(rows) * WT;
    for (int i = threadIdx.x; i < rows * WT; i += blockDim.x) {
        const int e = i / rows, r = i - e * rows;
        const int64_t row = row0 + r;
        const bool ok = row < n_valid;
        s_col[r * WT + e] = ok ? A.ell_col[e * n_b + row] : 0;
        s_val[r * WT + e] = ok ? A.ell_val[e * n_b + row] : T(0);
    }
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        const int64_t row = row0 + r;
        const bool ok = row < n_valid;
        s_dw[2 * r] = ok ? A.diag[row] : T(0);
        s_dw[2 * r + 1] = (ok && Z) ? A.w[row] : T(0);
    }
}

template <typename T, int WT>
__device__ __forceinline__ RowMeta<T, WT> meta_staged(const char *smem, int rows, int r) {
    const int32_t *s_col = reinterpret_cast<const int32_t *>(smem);
    const T *s_val = reinterpret_cast<const T *>(smem + stage_col_bytes(rows, WT));
    const T *s_dw = s_val + size_t(rows) * WT;
    RowMeta<T, WT> m;
#pragma unroll
    for (int e = 0; e < WT; ++e) {
        m.col[e] = s_col[r * WT + e];
        m.val[e] = s_val[r * WT + e];
    }
    m.diag = s_dw[2 * r];
    m.w = s_dw[2 * r + 1];
    return m;
}

// One row and one V-wide column chunk of the Laplacian SpMM from the row's
// base-block entries (compiled width WT > 0):
//   acc = diag_i x_i + sum_e a_ie x_{j(e)} + w_i (x_i[l+1] + x_i[l-1])
// Every gather is in flight before the first multiply-add.  The row's entries
// serve all V columns of the lane (and, across the row group, all k columns).
// xo returns this row's own V input values (used by fused dot products).
template <typename T, int V, bool Z, int WT, class Ld>
__device__ __forceinline__ vec_t<T, V> lap_row_meta(const RowMeta<T, WT> &m, const Ld &in, int k, int64_t row,
                                                    int c0, int sub, int lpr, bool single, vec_t<T, V> &xo) {
    using vt = vec_t<T, V>;
    xo = in.vec(row, c0);
    vt xj[WT];
#pragma unroll
    for (int e = 0; e < WT; ++e) xj[e] = in.vec(m.col[e], c0);
    vt acc = m.diag * xo;
#pragma unroll
    for (int e = 0; e < WT; ++e) acc = __builtin_elementwise_fma(vt(m.val[e]), xj[e], acc);
    if constexpr (Z) {
        const auto nb = neighbours_of<T, V>(xo, in, row, c0, sub, lpr, k, single);
#pragma unroll
        for (int t = 0; t < V; ++t) {
            const int l = c0 + t;
            acc[t] = __builtin_elementwise_fma(m.w, left_of<T, V>(xo, nb, t) + right_of<T, V>(xo, nb, t, l, k), acc[t]);
        }
    }
    return acc;
}

// Same product for a run-time ELL width (rows wider than the compiled widths).
template <typename T, int V, bool Z, class Ld>
__device__ __forceinline__ vec_t<T, V> lap_row_dyn(const OpDev<T> &A, const Ld &in, int64_t n_b, int k, int W,
                                                   int64_t row, int c0, int sub, int lpr, bool single,
                                                   vec_t<T, V> &xo) {
    using vt = vec_t<T, V>;
    xo = in.vec(row, c0);
    vt acc = A.diag[row] * xo;
    // Entries in groups of 4: the group's column indices, values and gathers
    // are all issued before its multiply-adds (same order of the sum).
    int e = 0;
    for (; e + 4 <= W; e += 4) {
        int64_t j[4];
        T v[4];
        vt xj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            j[u] = A.ell_col[(e + u) * n_b + row];
            v[u] = A.ell_val[(e + u) * n_b + row];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) xj[u] = in.vec(j[u], c0);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_elementwise_fma(vt(v[u]), xj[u], acc);
    }
    for (; e < W; ++e) {
        const int64_t j = A.ell_col[e * n_b + row];
        const T v = A.ell_val[e * n_b + row];
        acc = __builtin_elementwise_fma(vt(v), in.vec(j, c0), acc);
    }
    if constexpr (Z) {
        const T wr = A.w[row];
        const auto nb = neighbours_of<T, V>(xo, in, row, c0, sub, lpr, k, single);
#pragma unroll
        for (int t = 0; t < V; ++t) {
            const int l = c0 + t;
            acc[t] = __builtin_elementwise_fma(wr, left_of<T, V>(xo, nb, t) + right_of<T, V>(xo, nb, t, l, k), acc[t]);
        }
    }
    return acc;
}

// Dispatch on compiled width: global row entries or run-time width.
template <typename T, int V, bool Z, int WT, class Ld>
__device__ __forceinline__ vec_t<T, V> lap_row_ld(const OpDev<T> &A, const Ld &in, int64_t n_b, int k, int W,
                                                  int64_t row, int c0, int sub, int lpr, bool single,
                                                  vec_t<T, V> &xo) {
    if constexpr (WT > 0)
        return lap_row_meta<T, V, Z, WT>(meta_of<T, WT, Z>(A, n_b, row), in, k, row, c0, sub, lpr, single, xo);
    else
        return lap_row_dyn<T, V, Z>(A, in, n_b, k, W, row, c0, sub, lpr, single, xo);
}

template <typename T, int V, bool Z, int WT>
__device__ __forceinline__ vec_t<T, V> lap_row(const OpDev<T> &A, const T *__restrict__ X, int64_t n_b, int k,
                                               int ld, int W, int64_t row, int c0, int sub, int lpr, bool single,
                                               vec_t<T, V> &xo) {
    return lap_row_ld<T, V, Z, WT>(A, PlainLoad<T, V>{X, ld}, n_b, k, W, row, c0, sub, lpr, single, xo);
}

// ---------------------------------------------------------------------------
// Structured 13/27-point operators (one pass of a row group covers all k
// columns and V divides k)
// ---------------------------------------------------------------------------

// Column (c + D) mod k of each of this lane's V columns c = c0 .. c0+V-1:
// from the lane's own values when it holds that column, else from the lane
// of the row group that does.
template <typename T, int V, int D>
__device__ __forceinline__ vec_t<T, V> plane_shift(const vec_t<T, V> &xo, int c0, int lpr, int k) {
    vec_t<T, V> out;
#pragma unroll
    for (int t = 0; t < V; ++t) {
        const int u = t + D;
        if (u >= 0 && u < V) {
            out[t] = xo[u >= 0 && u < V ? u : 0];
        } else {
            const int g = ((c0 + u) % k + k) % k;
            out[t] = __shfl(xo[((u % V) + V) % V], g / V, lpr);
        }
    }
    return out;
}

// Row metadata load; UNI: the row is the same for the whole wavefront, so the
// load goes through the constant address space (a scalar load into SGPRs).
template <bool UNI, typename T>
__device__ __forceinline__ T ld_meta(const T *p, int64_t i) {
    if constexpr (UNI) {
        typedef const __attribute__((address_space(4))) T *cptr;
        return ((cptr)p)[i];
    } else {
        return p[i];
    }
}

// Everything one row of a structured operator reads: its metadata and the
// V columns of this lane in the row itself and its 8 in-plane neighbours.
template <typename T, int V, bool E1, bool S2>
struct StencilRow {
    T v0[8], v1[E1 ? 8 : 1];
    T dg, w1, w2;
    vec_t<T, V> xo, xj[8];
};

template <typename T, int V, bool E1, bool S2, bool UNI>
__device__ __forceinline__ void stencil_load(StencilRow<T, V, E1, S2> &r, const OpDev<T> &A,
                                             const T *__restrict__ X, int64_t n_b, int ld, int64_t row, int c0,
                                             bool active) {
    int32_t col[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        col[e] = ld_meta<UNI>(A.ell_col, e * n_b + row);
        r.v0[e] = ld_meta<UNI>(A.ell_val, e * n_b + row);
        if constexpr (E1) r.v1[e] = ld_meta<UNI>(A.ell_v1, e * n_b + row);
    }
    r.dg = ld_meta<UNI>(A.diag, row);
    r.w1 = ld_meta<UNI>(A.w, row);
    r.w2 = S2 ? ld_meta<UNI>(A.w2, row) : T(0);
    if (active) {
        r.xo = ldv<T, V>(X + row * ld + c0);
#pragma unroll
        for (int e = 0; e < 8; ++e) r.xj[e] = ldv<T, V>(X + int64_t(col[e]) * ld + c0);
    }
}

// One row of the structured operator:
//   diag x_i + sum_e v0_e x_j(e) + w1 (x_i[l+1] + x_i[l-1])
//   [+ w2 (x_i[l+2] + x_i[l-2])]                 (13-point, S2)
//   [+ sum_e v1_e (x_j(e)[l+1] + x_j(e)[l-1])]   (27-point, E1)
// Each neighbour row is loaded once; its shifted planes come from lane
// shuffles.  Explicit fused multiply-adds fix the rounding of every term, so
// the result does not depend on the tile.
template <typename T, int V, bool E1, bool S2>
__device__ __forceinline__ vec_t<T, V> stencil_apply(const StencilRow<T, V, E1, S2> &r, int c0, int lpr, int k) {
    using vt = vec_t<T, V>;
    auto fma_into = [](T a, const vt &b, vt &acc) { acc = __builtin_elementwise_fma(vt(a), b, acc); };
    vt acc = r.dg * r.xo;
#pragma unroll
    for (int e = 0; e < 8; ++e) fma_into(r.v0[e], r.xj[e], acc);
    fma_into(r.w1, plane_shift<T, V, 1>(r.xo, c0, lpr, k) + plane_shift<T, V, -1>(r.xo, c0, lpr, k), acc);
    if constexpr (S2)
        fma_into(r.w2, plane_shift<T, V, 2>(r.xo, c0, lpr, k) + plane_shift<T, V, -2>(r.xo, c0, lpr, k), acc);
    if constexpr (E1) {
#pragma unroll
        for (int e = 0; e < 8; ++e)
            fma_into(r.v1[e], plane_shift<T, V, 1>(r.xj[e], c0, lpr, k) + plane_shift<T, V, -1>(r.xj[e], c0, lpr, k),
                     acc);
    }
    return acc;
}

// Multi-pass rows: lane sub of a row group of lpr lanes holds columns
// p * lpr * V + sub * V + t of every pass p.  The columns of one row form a
// ring of k = P * lpr * V planes.
template <typename T, int V, bool E1, bool S2, int P>
struct StencilPasses {
    T v0[8], v1[E1 ? 8 : 1];
    T dg, w1, w2;
    vec_t<T, V> xo[P], xj[8][P];
};

template <typename T, int V, bool E1, bool S2, int P>
__device__ __forceinline__ void stencil_load_passes(StencilPasses<T, V, E1, S2, P> &r, const OpDev<T> &A,
                                                    const T *__restrict__ X, int64_t n_b, int ld, int64_t row, int c0,
                                                    int span) {
    int32_t col[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        col[e] = A.ell_col[e * n_b + row];
        r.v0[e] = A.ell_val[e * n_b + row];
        if constexpr (E1) r.v1[e] = A.ell_v1[e * n_b + row];
    }
    r.dg = A.diag[row];
    r.w1 = A.w[row];
    r.w2 = S2 ? A.w2[row] : T(0);
#pragma unroll
    for (int p = 0; p < P; ++p) r.xo[p] = ldv<T, V>(X + row * ld + p * span + c0);
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int p = 0; p < P; ++p) r.xj[e][p] = ldv<T, V>(X + int64_t(col[e]) * ld + p * span + c0);
}

// Columns (c + D) mod k of this lane's V columns of pass p, D in -2..2.  A
// value that lives dl lanes away comes from that lane by a shuffle; the
// source lanes whose reader sits across the group's edge hand over their
// value of the neighbouring pass instead (each source lane has one reader).
// Needs |dl| <= lpr, i.e. lpr * V >= 2.
template <typename T, int V, int P, int D>
__device__ __forceinline__ vec_t<T, V> ring_shift(const vec_t<T, V> (&x)[P], int p, int sub, int lpr) {
    vec_t<T, V> out;
#pragma unroll
    for (int t = 0; t < V; ++t) {
        const int u = t + D;
        if (u >= 0 && u < V) {
            out[t] = x[p][u >= 0 && u < V ? u : 0];
        } else {
            const int dl = u >= 0 ? u / V : -((-u + V - 1) / V);
            const int e = u - dl * V;
            const bool wrap = dl > 0 ? sub < dl : sub >= lpr + dl;
            const int pw = dl > 0 ? (p + 1) % P : (p + P - 1) % P;
            const T val = wrap ? x[pw][e] : x[p][e];
            out[t] = __shfl(val, (sub + dl) & (lpr - 1), lpr);
        }
    }
    return out;
}

// Pass p of a multi-pass row; the terms and their order are those of
// stencil_apply, so the result is bit-identical to the single-pass kernel.
template <typename T, int V, bool E1, bool S2, int P>
__device__ __forceinline__ vec_t<T, V> stencil_apply_pass(const StencilPasses<T, V, E1, S2, P> &r, int p, int sub,
                                                          int lpr) {
    using vt = vec_t<T, V>;
    auto fma_into = [](T a, const vt &b, vt &acc) { acc = __builtin_elementwise_fma(vt(a), b, acc); };
    vt acc = r.dg * r.xo[p];
#pragma unroll
    for (int e = 0; e < 8; ++e) fma_into(r.v0[e], r.xj[e][p], acc);
    fma_into(r.w1, ring_shift<T, V, P, 1>(r.xo, p, sub, lpr) + ring_shift<T, V, P, -1>(r.xo, p, sub, lpr), acc);
    if constexpr (S2)
        fma_into(r.w2, ring_shift<T, V, P, 2>(r.xo, p, sub, lpr) + ring_shift<T, V, P, -2>(r.xo, p, sub, lpr), acc);
    if constexpr (E1) {
#pragma unroll
        for (int e = 0; e < 8; ++e)
            fma_into(r.v1[e], ring_shift<T, V, P, 1>(r.xj[e], p, sub, lpr) + ring_shift<T, V, P, -1>(r.xj[e], p, sub, lpr),
                     acc);
    }
    return acc;
}

// Picks the kernel instance for (vec, planes coupled); vec * sizeof(T) <= 16.
template <typename T, typename F>
void by_vec(int vec, bool z, F &&f) {
    auto go = [&](auto vtag) {
        constexpr int V = decltype(vtag)::value;
        if constexpr (V * sizeof(T) <= 16) {
            if (z)
                f(std::integral_constant<int, V>{}, std::true_type{});
            else
                f(std::integral_constant<int, V>{}, std::false_type{});
        } else {
            throw Error(FVX_E_ARG, "vector width too large for this precision");
        }
    };
    switch (vec) {
        case 1: go(std::integral_constant<int, 1>{}); break;
        case 2: go(std::integral_constant<int, 2>{}); break;
        case 4: go(std::integral_constant<int, 4>{}); break;
        default: throw Error(FVX_E_ARG, "bad vector width");
    }
}

// Launch arguments of a row-tiled kernel (lanes_per_row lanes per row,
// tiles of rows_per_tile rows, tiles_per_block consecutive tiles per block).
template <typename T>
struct RowArgs {
    OpDev<T> A;
    int64_t n_b, n_rows;
    int k, ld, W, Wd, lpr, rows_per_tile, remap;
    int64_t tiles_per_block;
    int64_t F_b;
    // Line-blocked tiles of the CG kernels on a Cartesian base (0: row
    // tiles): a tile is rows_per_tile cells along x times `lines` grid lines,
    // n_xtiles tiles along x, n_ltiles in all, ltiles_per_block per block.
    int lines;
    uint32_t n_xtiles, n_ltiles;
    int64_t ltiles_per_block;
};

template <typename T>
inline RowArgs<T> row_args(const fvx_op *op, int64_t n_rows, RowGrid &g, const fvx_tile &t,
                           int max_blocks = 1 << 22) {
    if (t.max_blocks > 0) max_blocks = std::min(max_blocks, t.max_blocks);
    g = row_grid(n_rows, t, max_blocks);
    RowArgs<T> a;
    a.A = dev<T>(op);
    a.n_b = op->n_b;
    a.n_rows = n_rows;
    a.k = op->k;
    a.ld = op->ld;
    a.W = op->W;
    a.Wd = op->Wd;
    a.lpr = t.lanes_per_row;
    a.rows_per_tile = g.rows_per_tile;
    a.remap = t.xcd_remap;
    a.tiles_per_block = g.tiles_per_block;
    a.F_b = op->F_b;
    a.lines = 0;
    a.n_xtiles = a.n_ltiles = 0;
    a.ltiles_per_block = 0;
    return a;
}

}  // namespace fvx
