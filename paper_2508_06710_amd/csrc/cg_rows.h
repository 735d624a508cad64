// Row-tiled kernel bodies shared by the CG solver and the multigrid
// preconditioner: the virtual-block mapping, the row loop of a tile, and the
// Chebyshev smoothing step.
#pragma once

#include "cg_common.h"

namespace fvx {

// A kernel body runs one virtual block vb.blk of a grid of vb.nblk blocks.
// A single-problem launch maps hardware blocks onto virtual blocks (XCD-aware
// order); a batched launch maps them onto (problem, virtual block) items.  The
// arithmetic of a virtual block does not depend on which launch runs it.
struct VB {
    int64_t blk;
    int nblk;
};

__device__ __forceinline__ VB vb_single(int remap) { return VB{logical_block(remap), int(gridDim.x)}; }

#define ROW_PROLOGUE                                 \
    const int lpr = a.lpr;                           \
    const int sub = threadIdx.x & (lpr - 1);         \
    const int grp = threadIdx.x / lpr;               \
    const int64_t blk = vb.blk;                      \
    const int64_t t0 = blk * a.tiles_per_block;

#define FOR_ROWS                                                         \
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {              \
        const int64_t row = t * a.rows_per_tile + grp;                   \
        if (row >= a.n_rows) break;                                      \
        for (int c0 = sub * V; c0 < a.k; c0 += lpr * V)

#define END_ROWS }

// Line-blocked tiles of the CG kernels on a Cartesian 5-point base, when one
// pass of a row group covers the k columns: the row group of cell column i
// takes kCgLines grid lines j0 .. j0 + kCgLines - 1 and loads the
// kCgLines + 2 values of its column once (each line's own value is the
// north neighbour of the line below and the south neighbour of the line
// above), the west and east values of every line, and each line's
// coefficient record, all before the first multiply-add.  Each line's sum is
// that of lap_row_meta with the Cartesian row metadata (S, W, E, N in that
// order, an absent neighbour being the row itself with coefficient 0, the
// plane neighbours from lane shuffles), so a line-blocked kernel gives
// bitwise the row-tiled kernel's products.
constexpr int kCgLines = 4;

// The kCgLines products of tile t for this row group: acc[q] = (L x)[row_q]
// and xo[q] = x[row_q] for the rows row_q = (j0 + q) nx + i, x read through
// `in`; valid[q] says whether row_q is inside the grid (a ragged tile loads
// in-range values and its caller stores nothing for the others).
template <typename T, int V, bool Z, class Ld>
__device__ __forceinline__ void cart_lines(const RowArgs<T> &a, const Ld &in, uint32_t t, uint32_t grp, int sub,
                                           int lpr, vec_t<T, V> (&acc)[kCgLines], vec_t<T, V> (&xo)[kCgLines],
                                           int64_t (&row)[kCgLines], bool (&valid)[kCgLines]) {
    using vt = vec_t<T, V>;
    constexpr int R = kCgLines;
    const OpDev<T> &A = a.A;
    const uint32_t nx = uint32_t(A.cart_nx);
    const int ny = A.cart_ny;
    const uint32_t tj = t / a.n_xtiles, ti = t - tj * a.n_xtiles;
    const uint32_t i_raw = ti * uint32_t(a.rows_per_tile) + grp;
    const bool in_x = i_raw < nx;
    const uint32_t i = in_x ? i_raw : nx - 1;
    const int j0 = int(tj) * R;
    const int c0 = sub * V;
    // line index -> stored line: wrap when periodic in y, else clamp (a wall
    // neighbour is the line itself, with coefficient 0)
    auto line = [&](int jj) -> uint32_t {
        const int jw = jj + (jj < 0 ? ny : 0) - (jj >= ny ? ny : 0);
        const int jc = min(max(jj, 0), ny - 1);
        return uint32_t(A.cart_py ? jw : jc);
    };
    const uint32_t iW = i > 0 ? i - 1 : (A.cart_px ? nx - 1 : i);
    const uint32_t iE = i < nx - 1 ? i + 1 : (A.cart_px ? 0 : i);
    vt col[R + 2], xW[R], xE[R];
    RowMeta<T, 4> m[R];
#pragma unroll
    for (int q = 0; q < R + 2; ++q) col[q] = in.vec(int64_t(line(j0 - 1 + q)) * nx + i, c0);
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const uint32_t jr = (j0 + q < ny ? uint32_t(j0 + q) : uint32_t(ny - 1)) * nx;
        xW[q] = in.vec(int64_t(jr + iW), c0);
        xE[q] = in.vec(int64_t(jr + iE), c0);
        m[q] = meta_cart<T, Z>(A, int64_t(jr + i));
        row[q] = int64_t(jr + i);
        valid[q] = in_x && j0 + q < ny;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        xo[q] = col[q + 1];
        vt s = m[q].diag * xo[q];
        s = __builtin_elementwise_fma(vt(m[q].val[0]), col[q], s);
        s = __builtin_elementwise_fma(vt(m[q].val[1]), xW[q], s);
        s = __builtin_elementwise_fma(vt(m[q].val[2]), xE[q], s);
        s = __builtin_elementwise_fma(vt(m[q].val[3]), col[q + 2], s);
        if constexpr (Z) {
            const auto nb = plane_neighbours<T, V>(xo[q], sub, lpr, a.k);
#pragma unroll
            for (int u = 0; u < V; ++u) {
                const int l = c0 + u;
                s[u] = __builtin_elementwise_fma(m[q].w, left_of<T, V>(xo[q], nb, u) + right_of<T, V>(xo[q], nb, u, l, a.k),
                                                 s[u]);
            }
        }
        acc[q] = s;
    }
}

// The line tiles of virtual block blk.
#define FOR_LINE_TILES                                                                   \
    const int64_t lt0 = blk * a.ltiles_per_block;                                          \
    const int64_t lt1 = min(int64_t(a.n_ltiles), lt0 + a.ltiles_per_block);                \
    for (int64_t t = lt0; t < lt1; ++t)

// One step j >= 1 of the Chebyshev semi-iteration for D^-1 A z = D^-1 r
// (A = -L; Saad, Algorithm 12.1), in its three-term form: with d_{j-1} =
// z_j - z_{j-1},
//   z_{j+1} = z_j + c1 (z_j - z_{j-1}) + c2 D^-1 (r - A z_j),
// c1 = rho_j rho_{j-1}, c2 = 2 rho_j / delta from the host.  MODE 0 (j = 1):
// z_1 = D^-1 r / theta is formed on the fly from r and z_0 = 0; MODE 1
// (j = 2): z_1 is formed again from the row's own r; MODE 2 (j >= 3): z_{j-1}
// is read from zio, which then receives z_{j+1} (each row reads its own
// entry before writing it; the gather reads only zin).  LAST: the partials
// of r.z_{j+1} go to the r.z slot of part_b.
template <typename T, int V, bool Z, int WT, int MODE, bool LAST>
__device__ void b_cheb(const RowArgs<T> &a, const CgDev &d, VB vb, const T *__restrict__ r,
                       const T *__restrict__ zin, T *__restrict__ zio, T c1, T c2, T inv_theta) {
    if (d.st->done) return;
    __shared__ double lds[kMaxPercolBlock * kMaxV];
    ROW_PROLOGUE
    const int G = d.G;
    const bool single = lpr * V >= a.k;
    double c[1][V] = {};
    FOR_ROWS {
        const int64_t o = row * a.ld + c0;
        vec_t<T, V> zj, acc;
        if constexpr (MODE == 0)
            acc = lap_row_ld<T, V, Z, WT>(a.A, ChebFirstLoad<T, V>{r, a.A.dinv, a.ld, inv_theta}, a.n_b, a.k, a.W,
                                          row, c0, sub, lpr, single, zj);
        else
            acc = lap_row_ld<T, V, Z, WT>(a.A, PlainLoad<T, V>{zin, a.ld}, a.n_b, a.k, a.W, row, c0, sub, lpr,
                                          single, zj);
        const vec_t<T, V> rv = ldv<T, V>(r + o);
        const T di = a.A.dinv[row];
        vec_t<T, V> zprev;
        if constexpr (MODE == 0)
            zprev = vec_t<T, V>(0);
        else if constexpr (MODE == 1)
            zprev = (di * inv_theta) * rv;
        else
            zprev = ldv<T, V>(zio + o);
        const vec_t<T, V> zn = zj + c1 * (zj - zprev) + (c2 * di) * (rv + acc);  // r - A z = r + L z
        stv_masked<T, V>(zio + o, zn, a.k - c0);
        if constexpr (LAST) {
#pragma unroll
            for (int u = 0; u < V; ++u)
                if (c0 + u < a.k) c[0][u] += double(rv[u]) * double(zn[u]);
        }
    }
    END_ROWS
    if constexpr (LAST)
        write_partials<1, V>(c, sub, lpr, G, d.percol, d.part_b + 2 * int64_t(vb.nblk) * G, blk, vb.nblk, lds);
}

}  // namespace fvx
