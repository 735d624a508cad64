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
