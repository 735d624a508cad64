// SpMM kernels for the repeated-block operators: Laplacian, divergence,
// gradient, and the plane-major <-> row-major conversion.
//
// Work mapping (gfx950, wave64): a row group of `lanes_per_row` lanes owns
// one matrix row; each lane owns `vec` consecutive columns (one 16-byte load
// for FP64 x2 / FP32 x4), so a row group covers lanes_per_row * vec of the k
// columns per pass.  The row's matrix entries are read once per row group
// and applied to every column it holds -- the reuse that Section 2 (Eq. 1,
// Algorithm 1) turns SpMV into SpMM for.  Multivector rows are k-contiguous,
// so the lanes of a row group issue one coalesced load per neighbour row.
#include "kernels.h"

namespace fvx {
namespace {

// Y = (I_k (x) A_b + C) X, optionally scaled per column.  With S, each tile's
// base-block rows are first staged in LDS by the whole workgroup (coalesced
// loads) and every lane of a row reads them from there.
template <typename T, int V, bool Z, int WT, bool S, bool NT>
__global__ __launch_bounds__(1024) void k_lap(RowArgs<T> a, const T *__restrict__ X, T *__restrict__ Y,
                                              const double *__restrict__ cs) {
    extern __shared__ __align__(16) char smem[];
    const int lpr = a.lpr;
    const int sub = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const bool single = lpr * V >= a.k;
    const int64_t t0 = logical_block(a.remap) * a.tiles_per_block;
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row0 = t * a.rows_per_tile, row = row0 + grp;
        if constexpr (S) {
            if (row0 >= a.n_rows) break;  // uniform across the workgroup
            __syncthreads();              // the previous tile's readers are done
            stage_rows<T, WT, Z>(a.A, a.n_b, a.n_rows, row0, a.rows_per_tile, smem);
            __syncthreads();
            if (row >= a.n_rows) continue;
        } else {
            if (row >= a.n_rows) break;
        }
        for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
            vec_t<T, V> xo, acc;
            if constexpr (S)
                acc = lap_row_meta<T, V, Z, WT>(meta_staged<T, WT>(smem, a.rows_per_tile, grp), PlainLoad<T, V>{X, a.ld},
                                                a.k, row, c0, sub, lpr, single, xo);
            else
                acc = lap_row<T, V, Z, WT>(a.A, X, a.n_b, a.k, a.ld, a.W, row, c0, sub, lpr, single, xo);
            if (cs) {
#pragma unroll
                for (int q = 0; q < V; ++q)
                    if (c0 + q < a.k) acc[q] *= T(cs[c0 + q]);
            }
            stv_masked<T, V, NT>(Y + row * a.ld + c0, acc, a.k - c0);
        }
    }
}

// The same product on a Cartesian base with the 5-point face graph, when one
// pass of a row group covers the k columns exactly (lanes_per_row * V == k,
// lanes_per_row >= 8): the neighbours' indices come from (i, j) instead of
// the ELL columns, and the row's 8 coefficients [diag, w, S, W, E, N, 0, 0]
// arrive with one coalesced load per row group (lane q takes coefficient q)
// and shuffles -- so the gathers depend on no load.  The four entries are
// applied in the order S, W, E, N, which is the order of the ELL row of such
// an operator (an absent neighbour has coefficient 0 and points at the row
// itself), with the multiply-adds of lap_row_meta: the result is bitwise that
// of k_lap.
// Arguments of k_lap_cart: the grid and the operator's record, nothing else.
template <typename T>
struct CartArgs {
    const T *rec;            // [n_b][8]: diag, w, S, W, E, N, 0, 0
    uint32_t nx, ny, n_b, ld;
    uint32_t rows_per_tile, n_tiles;
    uint32_t n_xtiles;       // k_lap_cart_lines: tiles along x
    int px, py, lpr, remap;
};

// O32: the multivectors are below 4 GiB, so every address is a uniform base
// plus a 32-bit byte offset.  Tiles of rows_per_tile rows, a grid-stride loop
// over them (one tile per workgroup without a grid cap).
template <typename T, int V, bool Z, bool NT, bool O32, int LPR, bool CS>
__global__ __launch_bounds__(1024) void k_lap_cart(CartArgs<T> a, const T *__restrict__ X, T *__restrict__ Y,
                                                   const double *__restrict__ cs) {
    using vt = vec_t<T, V>;
    constexpr int lpr = LPR;  // the row-group width, a compile-time constant
    const int sub = threadIdx.x & (lpr - 1);
    const uint32_t grp = threadIdx.x / lpr;
    const uint32_t c0 = uint32_t(sub) * V;
    const uint32_t nx = a.nx, ny = a.ny;
    auto at = [&](const T *base, uint32_t rr) -> const T * {
        if constexpr (O32)
            return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                               (rr * a.ld + c0) * uint32_t(sizeof(T)));
        else
            return base + int64_t(rr) * a.ld + c0;
    };
    for (uint32_t t = uint32_t(logical_block(a.remap)); t < a.n_tiles; t += gridDim.x) {
        const uint32_t r = t * a.rows_per_tile + grp;
        if (r >= a.n_b) break;  // uniform over the row group
        const uint32_t j = r / nx, i = r - j * nx;
        const uint32_t cS = j > 0 ? r - nx : (a.py ? r + nx * (ny - 1) : r);
        const uint32_t cW = i > 0 ? r - 1 : (a.px ? r + nx - 1 : r);
        const uint32_t cE = i < nx - 1 ? r + 1 : (a.px ? r - (nx - 1) : r);
        const uint32_t cN = j < ny - 1 ? r + nx : (a.py ? r - nx * (ny - 1) : r);
        const vt xo = ldv<T, V>(at(X, r));
        const vt xS = ldv<T, V>(at(X, cS)), xW = ldv<T, V>(at(X, cW));
        const vt xE = ldv<T, V>(at(X, cE)), xN = ldv<T, V>(at(X, cN));
        const T mine = a.rec[r * 8u + uint32_t(sub & 7)];
        // all six loads are in flight before the first shuffle waits on one
        __builtin_amdgcn_sched_barrier(0);
        const T d = __shfl(mine, 0, lpr), w = __shfl(mine, 1, lpr);
        const T vS = __shfl(mine, 2, lpr), vW = __shfl(mine, 3, lpr), vE = __shfl(mine, 4, lpr), vN = __shfl(mine, 5, lpr);
        vt acc = d * xo;
        acc = __builtin_elementwise_fma(vt(vS), xS, acc);
        acc = __builtin_elementwise_fma(vt(vW), xW, acc);
        acc = __builtin_elementwise_fma(vt(vE), xE, acc);
        acc = __builtin_elementwise_fma(vt(vN), xN, acc);
        if constexpr (Z) {
            // the group covers the k columns exactly: column c0 - 1 is the
            // previous lane's last value (lane lpr - 1 holds column k - 1), and
            // column c0 + V the next lane's first (lane 0 holds column 0)
            const T left0 = __shfl(xo[V - 1], (sub + lpr - 1) & (lpr - 1), lpr);
            const T rightV = __shfl(xo[0], (sub + 1) & (lpr - 1), lpr);
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const T lq = q > 0 ? xo[q > 0 ? q - 1 : 0] : left0;
                const T rq = q + 1 < V ? xo[q + 1 < V ? q + 1 : 0] : rightV;
                acc[q] = __builtin_elementwise_fma(w, lq + rq, acc[q]);
            }
        }
        if constexpr (CS) {
#pragma unroll
            for (int q = 0; q < V; ++q) acc[q] *= T(cs[c0 + q]);
        }
        vt *out = const_cast<vt *>(reinterpret_cast<const vt *>(at(Y, r)));
        if constexpr (NT)
            __builtin_nontemporal_store(acc, out);
        else
            *out = acc;
    }
}

// The same product with R grid lines along y per row group (R = 2 or 4, at
// most ny): a tile is rows_per_tile cells along x times R lines, and the row
// group of cell column i loads the R + 2 values x(i, j0 - 1 .. j0 + R) once,
// so that each line's own value is also the north neighbour of the line below
// and the south neighbour of the line above (R + 2 loads in place of 3R), and
// a lane keeps about R times the bytes of k_lap_cart in flight.  Lines past
// ny (a ragged last tile) load in-range values and store nothing.  Each
// line's neighbour values and coefficients are those of k_lap_cart (a wall
// neighbour is the cell itself, a periodic one wraps), combined in the same
// order: the result is bitwise that of k_lap_cart.
template <typename T, int V, bool Z, bool NT, bool O32, int R, int LPR, bool CS>
__global__ __launch_bounds__(1024) void k_lap_cart_lines(CartArgs<T> a, const T *__restrict__ X, T *__restrict__ Y,
                                                         const double *__restrict__ cs) {
    using vt = vec_t<T, V>;
    constexpr int lpr = LPR;  // the row-group width, a compile-time constant
    const int sub = threadIdx.x & (lpr - 1);
    const uint32_t grp = threadIdx.x / lpr;
    const uint32_t c0 = uint32_t(sub) * V;
    const uint32_t nx = a.nx;
    const int ny = int(a.ny);
    auto at = [&](const T *base, uint32_t rr) -> const T * {
        if constexpr (O32)
            return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                               (rr * a.ld + c0) * uint32_t(sizeof(T)));
        else
            return base + int64_t(rr) * a.ld + c0;
    };
    // line index -> stored line: wrap when periodic in y, else clamp (the
    // wall neighbour of lines 0 and ny - 1 is the line itself); selects, no
    // branches, so the loads below stay in one basic block
    auto line = [&](int jj) -> uint32_t {
        const int jw = jj + (jj < 0 ? ny : 0) - (jj >= ny ? ny : 0);
        const int jc = min(max(jj, 0), ny - 1);
        return uint32_t(a.py ? jw : jc);
    };
    for (uint32_t t = uint32_t(logical_block(a.remap)); t < a.n_tiles; t += gridDim.x) {
        const uint32_t tj = t / a.n_xtiles, ti = t - tj * a.n_xtiles;
        const uint32_t i = ti * a.rows_per_tile + grp;
        if (i >= nx) continue;  // uniform over the row group
        const int j0 = int(tj) * R;
        const uint32_t iW = i > 0 ? i - 1 : (a.px ? nx - 1 : i);
        const uint32_t iE = i < nx - 1 ? i + 1 : (a.px ? 0 : i);
        vt col[R + 2], xW[R], xE[R];
        T mine[R];
#pragma unroll
        for (int q = 0; q < R + 2; ++q) col[q] = ldv<T, V>(at(X, line(j0 - 1 + q) * nx + i));
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const uint32_t jr = (j0 + q < ny ? uint32_t(j0 + q) : uint32_t(ny - 1)) * nx;
            xW[q] = ldv<T, V>(at(X, jr + iW));
            xE[q] = ldv<T, V>(at(X, jr + iE));
            mine[q] = a.rec[(jr + i) * 8u + uint32_t(sub & 7)];
        }
        // every load is in flight before the first shuffle waits on one; all
        // R lines are computed (no branch between the loads and their uses)
        // and only the lines inside the grid are stored
        __builtin_amdgcn_sched_barrier(0);
        vt acc[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const T d = __shfl(mine[q], 0, lpr), w = __shfl(mine[q], 1, lpr);
            const T vS = __shfl(mine[q], 2, lpr), vW = __shfl(mine[q], 3, lpr), vE = __shfl(mine[q], 4, lpr),
                    vN = __shfl(mine[q], 5, lpr);
            const vt xo = col[q + 1];
            acc[q] = d * xo;
            acc[q] = __builtin_elementwise_fma(vt(vS), col[q], acc[q]);
            acc[q] = __builtin_elementwise_fma(vt(vW), xW[q], acc[q]);
            acc[q] = __builtin_elementwise_fma(vt(vE), xE[q], acc[q]);
            acc[q] = __builtin_elementwise_fma(vt(vN), col[q + 2], acc[q]);
            if constexpr (Z) {
                const T left0 = __shfl(xo[V - 1], (sub + lpr - 1) & (lpr - 1), lpr);
                const T rightV = __shfl(xo[0], (sub + 1) & (lpr - 1), lpr);
#pragma unroll
                for (int p = 0; p < V; ++p) {
                    const T lp = p > 0 ? xo[p > 0 ? p - 1 : 0] : left0;
                    const T rp = p + 1 < V ? xo[p + 1 < V ? p + 1 : 0] : rightV;
                    acc[q][p] = __builtin_elementwise_fma(w, lp + rp, acc[q][p]);
                }
            }
            if constexpr (CS) {
#pragma unroll
                for (int p = 0; p < V; ++p) acc[q][p] *= T(cs[c0 + p]);
            }
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (j0 + q >= ny) break;  // uniform over the workgroup
            vt *out = const_cast<vt *>(reinterpret_cast<const vt *>(at(Y, uint32_t(j0 + q) * nx + i)));
            if constexpr (NT)
                __builtin_nontemporal_store(acc[q], out);
            else
                *out = acc[q];
        }
    }
}

// The same product when a row group covers the k columns in exactly P
// passes (k = P * lanes_per_row * V): the row's entries are read once, and
// every pass's own-row and neighbour-row loads are issued before the first
// multiply-add, so a lane keeps P times more bytes in flight.  The plane
// neighbours at pass edges come from the neighbouring pass's registers.  The
// operations per element are those of lap_row_meta, in the same order.
template <typename T, int V, bool Z, int WT, bool NT, int P>
__global__ __launch_bounds__(512) void k_lap_passes(RowArgs<T> a, const T *__restrict__ X, T *__restrict__ Y,
                                                     const double *__restrict__ cs) {
    const int lpr = a.lpr;
    const int sub = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const int64_t t0 = logical_block(a.remap) * a.tiles_per_block;
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        const RowMeta<T, WT> m = meta_of<T, WT, Z>(a.A, a.n_b, row);
        vec_t<T, V> xo[P], xj[P][WT];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int c0 = (p * lpr + sub) * V;
            xo[p] = ldv<T, V>(X + row * a.ld + c0);
#pragma unroll
            for (int e = 0; e < WT; ++e) xj[p][e] = ldv<T, V>(X + int64_t(m.col[e]) * a.ld + c0);
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int c0 = (p * lpr + sub) * V;
            vec_t<T, V> acc = m.diag * xo[p];
#pragma unroll
            for (int e = 0; e < WT; ++e) acc = __builtin_elementwise_fma(vec_t<T, V>(m.val[e]), xj[p][e], acc);
            if constexpr (Z) {
                // column c0 - 1: lane sub - 1 of this pass, or the last lane of the
                // previous pass (of the last pass for column k - 1); column c0 + V:
                // lane sub + 1, or lane 0 of the next pass (of pass 0 for column 0)
                const T l_same = __shfl(xo[p][V - 1], sub == 0 ? 0 : sub - 1, lpr);
                const T l_prev = __shfl(xo[p > 0 ? p - 1 : P - 1][V - 1], lpr - 1, lpr);
                const T r_same = __shfl(xo[p][0], sub == lpr - 1 ? 0 : sub + 1, lpr);
                const T r_next = __shfl(xo[p + 1 < P ? p + 1 : 0][0], 0, lpr);
                PlaneNeighbours<T, V> nb;
                nb.left0 = sub > 0 ? l_same : l_prev;
                nb.rightV = sub < lpr - 1 ? r_same : r_next;
#pragma unroll
                for (int q = 0; q < V; ++q)
                    acc[q] = __builtin_elementwise_fma(m.w, left_of<T, V>(xo[p], nb, q) + right_of<T, V>(xo[p], nb, q, c0 + q, a.k),
                                           acc[q]);
            }
            if (cs) {
#pragma unroll
                for (int q = 0; q < V; ++q) acc[q] *= T(cs[c0 + q]);
            }
            stv_masked<T, V, NT>(Y + row * a.ld + c0, acc, a.k - c0);
        }
    }
}

// Y = A X for the structured 13/27-point operators, one pass of a row group
// covering all k columns.  UNI: 64 lanes per row, so the metadata of a row is
// wavefront-uniform and comes in through scalar loads.
template <typename T, int V, bool E1, bool S2, bool NT, bool UNI>
__global__ __launch_bounds__(1024) void k_lap_stencil(RowArgs<T> a, const T *__restrict__ X, T *__restrict__ Y) {
    const int lpr = UNI ? 64 : a.lpr;
    const int sub = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const int c0 = sub * V;
    const bool active = c0 < a.k;
    const int64_t t0 = logical_block(a.remap) * a.tiles_per_block;
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        int64_t row = t * a.rows_per_tile + grp;
        if constexpr (UNI) row = __builtin_amdgcn_readfirstlane(int32_t(row));
        if (row >= a.n_rows) break;
        StencilRow<T, V, E1, S2> r;
        stencil_load<T, V, E1, S2, UNI>(r, a.A, X, a.n_b, a.ld, row, c0, active);
        if (active)
            stv_masked<T, V, NT>(Y + row * a.ld + c0, stencil_apply<T, V, E1, S2>(r, c0, lpr, a.k), a.k - c0);
    }
}

// The same product with P passes of a row group (k = P * lanes_per_row * V):
// every lane holds its V columns of all P passes of the row and of its 8
// neighbours, so the plane shifts rotate across the lanes of the group and,
// at the group's edge, into the next or previous pass.
template <typename T, int V, bool E1, bool S2, bool NT, int P, int LPR>
__global__ __launch_bounds__(512) void k_lap_stencil_passes(RowArgs<T> a, const T *__restrict__ X,
                                                            T *__restrict__ Y) {
    const int lpr = LPR ? LPR : a.lpr;  // LPR: the row-group width as a constant (0: from the arguments)
    const int sub = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const int span = lpr * V;
    const int c0 = sub * V;
    const int64_t t0 = logical_block(a.remap) * a.tiles_per_block;
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        StencilPasses<T, V, E1, S2, P> r;
        stencil_load_passes<T, V, E1, S2, P>(r, a.A, X, a.n_b, a.ld, row, c0, span);
#pragma unroll
        for (int p = 0; p < P; ++p)
            stv_masked<T, V, NT>(Y + row * a.ld + p * span + c0, stencil_apply_pass<T, V, E1, S2, P>(r, p, sub, lpr), V);
    }
}

// The structured 13/27-point products on line tiles, for a Cartesian base
// whose rows store their 8 in-plane entries in the fixed direction order
// (27-point SW, S, SE, W, E, NW, N, NE; 13-point SS, S, WW, W, E, EE, N, NN)
// and a tile whose 64 lanes cover the k = 64 V columns in one pass.  A
// wavefront takes one cell column i and R (2, 4 or 8) grid lines
// j0 .. j0 + R - 1; the
// row's coefficients are wavefront-uniform (scalar loads).  It loads each
// value of the column strip once: 27-point the columns i - 1, i, i + 1 of
// the lines j0 - 1 .. j0 + R (3 (R + 2) loads for R rows, against 9 R);
// 13-point the column i of the lines j0 - 2 .. j0 + R + 1 and the columns
// i +- 1, i +- 2 of each line (5 R + 4 against 9 R).  The plane shifts of a
// loaded value are formed once and serve every line that reads it.  A
// neighbour past a wall is read at the clamped cell, with coefficient 0 (the
// ELL row holds the row itself there), so each term and the order of the
// terms are those of stencil_apply: bitwise k_lap_stencil.  A row's
// coefficients come from its packed record (a few wide scalar loads in place
// of one per coefficient array): row 0's with the strip's loads, row q + 1's
// while row q is computed.
template <typename T, int V, bool E1, bool S2, bool NT, int R>
__global__ __launch_bounds__(512) void k_stencil_lines(RowArgs<T> a, const T *__restrict__ X, T *__restrict__ Y,
                                                        int nx, int ny, int px, int py, uint32_t n_xtiles,
                                                        uint32_t n_tiles) {
    using vt = vec_t<T, V>;
    constexpr int LPR = 64;
    const int lane = threadIdx.x & 63;
    const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // the wavefront's cell column
    const int c0 = lane * V;
    const int k = a.k;
    const OpDev<T> &A = a.A;
    auto wrapc = [](int v, int n, int per) {  // periodic wrap or wall clamp, always inside [0, n)
        return per ? ((v % n) + n) % n : min(max(v, 0), n - 1);
    };
    auto ld = [&](int j, int i) { return ldv<T, V>(X + (int64_t(j) * nx + i) * a.ld + c0); };
    auto fma_into = [](T cf, const vt &b, vt &acc) { acc = __builtin_elementwise_fma(vt(cf), b, acc); };
    auto shifts = [&](const vt &x, auto Dt) {  // x[l + D] + x[l - D]
        constexpr int D = decltype(Dt)::value;
        return plane_shift<T, V, D>(x, c0, LPR, k) + plane_shift<T, V, -D>(x, c0, LPR, k);
    };
    for (uint32_t t = uint32_t(logical_block(a.remap)); t < n_tiles; t += gridDim.x) {
        const uint32_t tj = t / n_xtiles, ti = t - tj * n_xtiles;
        const uint32_t i_raw = ti * uint32_t(a.rows_per_tile) + w;
        const bool in_x = i_raw < uint32_t(nx);  // uniform over the wavefront
        const int i = in_x ? int(i_raw) : nx - 1;
        const int j0 = int(tj) * R;
        constexpr int NC = E1 ? 18 : 11, NCP = srec_width(E1 ? 27 : 13);
        T cf[2][NC];
        auto load_coef = [&](int q, T(&c)[NC]) {
            const int64_t base = (int64_t(min(j0 + q, ny - 1)) * nx + i) * NCP;
#pragma unroll
            for (int e = 0; e < NC; ++e) c[e] = ld_meta<true>(A.srec, base + e);
        };
        load_coef(0, cf[0]);
        vt acc[R];
        if constexpr (E1) {
            // 27-point: columns iW, i, iE of the lines j0 - 1 .. j0 + R
            const int iW = wrapc(i - 1, nx, px), iE = wrapc(i + 1, nx, px);
            vt xw[R + 2], xc[R + 2], xe[R + 2];
#pragma unroll
            for (int q = 0; q < R + 2; ++q) {
                const int j = wrapc(j0 - 1 + q, ny, py);
                xw[q] = ld(j, iW);
                xc[q] = ld(j, i);
                xe[q] = ld(j, iE);
            }
            __builtin_amdgcn_sched_barrier(0);
            vt sw[R + 2], sc[R + 2], se[R + 2];
#pragma unroll
            for (int q = 0; q < R + 2; ++q) {
                sw[q] = shifts(xw[q], std::integral_constant<int, 1>{});
                sc[q] = shifts(xc[q], std::integral_constant<int, 1>{});
                se[q] = shifts(xe[q], std::integral_constant<int, 1>{});
            }
#pragma unroll
            for (int q = 0; q < R; ++q) {
                if (q + 1 < R) load_coef(q + 1, cf[(q + 1) & 1]);
                const T(&c)[NC] = cf[q & 1];
                const vt *xs[8] = {&xw[q], &xc[q], &xe[q], &xw[q + 1], &xe[q + 1], &xw[q + 2], &xc[q + 2], &xe[q + 2]};
                const vt *ss[8] = {&sw[q], &sc[q], &se[q], &sw[q + 1], &se[q + 1], &sw[q + 2], &sc[q + 2], &se[q + 2]};
                vt s_ = c[8] * xc[q + 1];
#pragma unroll
                for (int e = 0; e < 8; ++e) fma_into(c[e], *xs[e], s_);
                fma_into(c[9], sc[q + 1], s_);
#pragma unroll
                for (int e = 0; e < 8; ++e) fma_into(c[10 + e], *ss[e], s_);
                acc[q] = s_;
            }
        } else {
            // 13-point: column i of the lines j0 - 2 .. j0 + R + 1; columns i +- 1,
            // i +- 2 of each line
            const int iWW = wrapc(i - 2, nx, px), iW = wrapc(i - 1, nx, px);
            const int iE = wrapc(i + 1, nx, px), iEE = wrapc(i + 2, nx, px);
            vt xc[R + 4], xww[R], xw[R], xe[R], xee[R];
#pragma unroll
            for (int q = 0; q < R + 4; ++q) xc[q] = ld(wrapc(j0 - 2 + q, ny, py), i);
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int j = min(j0 + q, ny - 1);
                xww[q] = ld(j, iWW);
                xw[q] = ld(j, iW);
                xe[q] = ld(j, iE);
                xee[q] = ld(j, iEE);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < R; ++q) {
                if (q + 1 < R) load_coef(q + 1, cf[(q + 1) & 1]);
                const T(&c)[NC] = cf[q & 1];
                const vt &xo = xc[q + 2];
                const vt *xs[8] = {&xc[q], &xc[q + 1], &xww[q], &xw[q], &xe[q], &xee[q], &xc[q + 3], &xc[q + 4]};
                vt s_ = c[8] * xo;
#pragma unroll
                for (int e = 0; e < 8; ++e) fma_into(c[e], *xs[e], s_);
                fma_into(c[9], shifts(xo, std::integral_constant<int, 1>{}), s_);
                fma_into(c[10], shifts(xo, std::integral_constant<int, 2>{}), s_);
                acc[q] = s_;
            }
        }
        if (!in_x) continue;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (j0 + q >= ny) break;
            stv_masked<T, V, NT>(Y + (int64_t(j0 + q) * nx + i) * a.ld + c0, acc[q], V);
        }
    }
}

// D = M U: integrated divergence of in-plane face fluxes plus the fluxes
// through the faces between planes.
template <typename T, int V, bool Z, int WT>
__global__ __launch_bounds__(1024) void k_div(RowArgs<T> a, const T *__restrict__ U, const T *__restrict__ Wz,
                                              T *__restrict__ D) {
    const int lpr = a.lpr;
    const int sub = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const bool single = lpr * V >= a.k;
    const int64_t t0 = logical_block(a.remap) * a.tiles_per_block;
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
            vec_t<T, V> acc = 0;
            if constexpr (WT > 0) {
                int32_t f[WT];
                T cf[WT];
#pragma unroll
                for (int e = 0; e < WT; ++e) {
                    f[e] = a.A.cf_face[e * a.n_b + row];
                    cf[e] = a.A.cf_coef[e * a.n_b + row];
                }
                vec_t<T, V> u[WT];
#pragma unroll
                for (int e = 0; e < WT; ++e) u[e] = ldv<T, V>(U + int64_t(f[e]) * a.ld + c0);
#pragma unroll
                for (int e = 0; e < WT; ++e) acc += cf[e] * u[e];
            } else {
                for (int e = 0; e < a.Wd; ++e) {
                    const int64_t f = a.A.cf_face[e * a.n_b + row];
                    const T c = a.A.cf_coef[e * a.n_b + row];
                    acc += c * ldv<T, V>(U + f * a.ld + c0);
                }
            }
            if constexpr (Z) {
                const T ar = a.A.area[row];
                const vec_t<T, V> wo = ldv<T, V>(Wz + row * a.ld + c0);
                const auto nb = neighbours_of<T, V>(wo, PlainLoad<T, V>{Wz, a.ld}, row, c0, sub, lpr, a.k, single);
#pragma unroll
                for (int q = 0; q < V; ++q) acc[q] += ar * (wo[q] - left_of<T, V>(wo, nb, q));
            }
            stv_masked<T, V>(D + row * a.ld + c0, acc, a.k - c0);
        }
    }
}

// Out = C(u_s) Phi = M U_s Pi Phi: the convective operator of Section 3.1 --
// the divergence of the face fluxes u_f * (phi_c1 + phi_c2) / 2 (midpoint
// interpolation of the cell values to the face).  Each cell gathers, for each
// of its faces, the face velocity and the value of the cell across the face;
// the faces between planes take the neighbouring planes from the row itself.
// At most 512 threads per block: under a 1024-thread bound the compiler caps
// the kernel at 128 registers, and the wider face rows (6 and 8 faces per cell)
// spilled to scratch.
constexpr int kConvectBlock = 512;

template <typename T, int V, bool Z, int WT>
__global__ __launch_bounds__(kConvectBlock) void k_convect(RowArgs<T> a, const T *__restrict__ U, const T *__restrict__ Wz,
                                                  const T *__restrict__ Phi, T *__restrict__ Out) {
    const int lpr = a.lpr;
    const int sub = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const bool single = lpr * V >= a.k;
    const int64_t t0 = logical_block(a.remap) * a.tiles_per_block;
    const T half = T(0.5);
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
            const vec_t<T, V> po = ldv<T, V>(Phi + row * a.ld + c0);
            vec_t<T, V> acc = 0;
            auto face = [&](int64_t f, T cf) {
                const int64_t other = cf > T(0) ? a.A.f_c2[f] : a.A.f_c1[f];
                const vec_t<T, V> uf = ldv<T, V>(U + f * a.ld + c0);
                const vec_t<T, V> pn = ldv<T, V>(Phi + other * a.ld + c0);
                acc += (cf * half) * (uf * (po + pn));
            };
            if constexpr (WT > 0) {
#pragma unroll
                for (int e = 0; e < WT; ++e) face(a.A.cf_face[e * a.n_b + row], a.A.cf_coef[e * a.n_b + row]);
            } else {
                for (int e = 0; e < a.Wd; ++e) face(a.A.cf_face[e * a.n_b + row], a.A.cf_coef[e * a.n_b + row]);
            }
            if constexpr (Z) {
                const T ar = a.A.area[row];
                const vec_t<T, V> wo = ldv<T, V>(Wz + row * a.ld + c0);
                const auto nw = neighbours_of<T, V>(wo, PlainLoad<T, V>{Wz, a.ld}, row, c0, sub, lpr, a.k, single);
                const auto np = neighbours_of<T, V>(po, PlainLoad<T, V>{Phi, a.ld}, row, c0, sub, lpr, a.k, single);
#pragma unroll
                for (int q = 0; q < V; ++q) {
                    const int l = c0 + q;
                    const T up = wo[q] * (po[q] + right_of<T, V>(po, np, q, l, a.k));
                    const T dn = left_of<T, V>(wo, nw, q) * (left_of<T, V>(po, np, q) + po[q]);
                    acc[q] += (ar * half) * (up - dn);
                }
            }
            stv_masked<T, V>(Out + row * a.ld + c0, acc, a.k - c0);
        }
    }
}

// Gf = G_b P on in-plane faces (rows [0, F_b)), Gz on the faces between
// planes (rows [F_b, F_b + n_b)).
template <typename T, int V, bool Z>
__global__ __launch_bounds__(1024) void k_grad(RowArgs<T> a, const T *__restrict__ P, T *__restrict__ Gf,
                                               T *__restrict__ Gz, T alpha, int acc) {
    const int lpr = a.lpr;
    const int sub = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const bool single = lpr * V >= a.k;
    const int64_t t0 = logical_block(a.remap) * a.tiles_per_block;
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        if (row < a.F_b) {
            const int64_t c1 = a.A.f_c1[row], c2 = a.A.f_c2[row];
            const T inv = a.A.f_invd[row];
            for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
                vec_t<T, V> g = (ldv<T, V>(P + c2 * a.ld + c0) - ldv<T, V>(P + c1 * a.ld + c0)) * inv;
                if (acc) g = ldv<T, V>(Gf + row * a.ld + c0) + alpha * g;
                stv_masked<T, V>(Gf + row * a.ld + c0, g, a.k - c0);
            }
        } else if constexpr (Z) {
            const int64_t i = row - a.F_b;
            const T inv = a.A.inv_dz;
            for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
                const vec_t<T, V> po = ldv<T, V>(P + i * a.ld + c0);
                vec_t<T, V> g;
                const auto nb = neighbours_of<T, V>(po, PlainLoad<T, V>{P, a.ld}, i, c0, sub, lpr, a.k, single);
#pragma unroll
                for (int q = 0; q < V; ++q) g[q] = (right_of<T, V>(po, nb, q, c0 + q, a.k) - po[q]) * inv;
                if (acc) g = ldv<T, V>(Gz + i * a.ld + c0) + alpha * g;
                stv_masked<T, V>(Gz + i * a.ld + c0, g, a.k - c0);
            }
        }
    }
}

template <typename T>
__global__ void k_pack(int64_t n_rows, int k, int ld, const T *__restrict__ src, T *__restrict__ dst,
                       int to_rows) {
    const int64_t n = n_rows * k;
    for (int64_t idx = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; idx < n;
         idx += int64_t(gridDim.x) * blockDim.x) {
        const int64_t r = idx / k;
        const int l = int(idx - r * k);
        if (to_rows)
            dst[r * ld + l] = src[int64_t(l) * n_rows + r];
        else
            dst[int64_t(l) * n_rows + r] = src[r * ld + l];
    }
}


void check_ptr(const void *p, const char *what) {
    FVX_REQUIRE(p, FVX_E_ARG, std::string(what) + " is NULL");
    FVX_REQUIRE(reinterpret_cast<uintptr_t>(p) % 16 == 0, FVX_E_ARG, std::string(what) + " is not 16-byte aligned");
}

void check_dtype(const fvx_op *op, int dtype) {
    FVX_REQUIRE(op, FVX_E_ARG, "op is NULL");
    FVX_REQUIRE(dtype == FVX_F64 || dtype == FVX_F32, FVX_E_ARG, "dtype must be FVX_F64 or FVX_F32");
    FVX_REQUIRE(dtype == FVX_F64 || op->has_f32, FVX_E_ARG, "operator was built without FP32 copies");
}

}  // namespace

// Grid lines along y per row group of the Cartesian kernel: 1 without a
// workgroup cap or when one line per tile fits under it, else the fewest of
// 2 or 4 that does (4 if neither), at most ny.
int cart_lines(int64_t n_b, int nx, int ny, int rows_per_tile, int max_blocks) {
    if (max_blocks <= 0 || ceil_div(n_b, rows_per_tile) <= max_blocks) return 1;
    const int64_t xt = ceil_div(nx, rows_per_tile);
    int r = xt * ceil_div(ny, 2) <= max_blocks ? 2 : 4;
    while (r > ny) r >>= 1;
    return r;
}

template <typename T>
void launch_lap_stencil(const fvx_op *op, const T *X, T *Y, const double *cs, hipStream_t s) {
    FVX_REQUIRE(cs == nullptr, FVX_E_ARG, "colscale applies to independent planes only");
    RowGrid g;
    const fvx_tile &t = op->tile[dtype_of<T>()];
    const int span = t.lanes_per_row * t.vec;
    const int passes = span >= op->k ? 1 : op->k / span;
    FVX_REQUIRE(op->k % t.vec == 0 && (passes == 1 || (op->k == passes * span && (passes == 2 || passes == 4) &&
                                                       span >= 2 && t.block <= 512)),
                FVX_E_ARG, "13/27-point operators need a tile with 1, 2 or 4 passes over k, vec dividing k");
    auto a = row_args<T>(op, op->n_b, g, t);
    // line tiles: a direction-ordered operator, one pass of 64 lanes over k,
    // workgroups of at most 512 threads, and a workgroup cap that the
    // one-line tiles exceed
    int lines = 1;
    if (op->stencil_dir && t.lanes_per_row == 64 && op->k == 64 * t.vec && !t.stage_lds && t.max_blocks > 0 &&
        t.block <= 512 && ceil_div(op->n_b, g.rows_per_tile) > t.max_blocks) {
        // the fewest of 2, 4 or 8 lines per wavefront that fit under the cap
        // (8 if none does), at most ny
        const int64_t xt = ceil_div(op->grid_nx, g.rows_per_tile);
        lines = 2;
        while (lines < 8 && xt * ceil_div(op->grid_ny, lines) > t.max_blocks) lines *= 2;
        while (lines > op->grid_ny) lines >>= 1;
    }
    by_vec<T>(t.vec, true, [&](auto V, auto) {
        constexpr int v = decltype(V)::value;
        auto go = [&](auto E1t, auto S2t) {
            constexpr bool e1 = decltype(E1t)::value, s2 = decltype(S2t)::value;
            auto launch = [&](auto NTt) {
                constexpr bool nt = decltype(NTt)::value;
                if (lines > 1) {
                    const uint32_t n_xtiles = uint32_t(ceil_div(op->grid_nx, g.rows_per_tile));
                    const uint32_t n_tiles = n_xtiles * uint32_t(ceil_div(op->grid_ny, lines));
                    const int nblk = int(std::min<int64_t>(n_tiles, t.max_blocks));
                    if (lines == 8)
                        hipLaunchKernelGGL((k_stencil_lines<T, v, e1, s2, nt, 8>), dim3(nblk), dim3(t.block), 0, s, a,
                                           X, Y, op->grid_nx, op->grid_ny, op->grid_px, op->grid_py, n_xtiles, n_tiles);
                    else if (lines == 4)
                        hipLaunchKernelGGL((k_stencil_lines<T, v, e1, s2, nt, 4>), dim3(nblk), dim3(t.block), 0, s, a,
                                           X, Y, op->grid_nx, op->grid_ny, op->grid_px, op->grid_py, n_xtiles, n_tiles);
                    else
                        hipLaunchKernelGGL((k_stencil_lines<T, v, e1, s2, nt, 2>), dim3(nblk), dim3(t.block), 0, s, a,
                                           X, Y, op->grid_nx, op->grid_ny, op->grid_px, op->grid_py, n_xtiles, n_tiles);
                    return;
                }
                // the row-group width as a constant for the common widths, so that the
                // ring shifts' source lanes fold
                auto passes_kernel = [&](auto Pt) {
                    constexpr int P = decltype(Pt)::value;
                    switch (t.lanes_per_row) {
                        case 4:
                            hipLaunchKernelGGL((k_lap_stencil_passes<T, v, e1, s2, nt, P, 4>), dim3(g.n_blocks),
                                               dim3(t.block), 0, s, a, X, Y);
                            break;
                        case 8:
                            hipLaunchKernelGGL((k_lap_stencil_passes<T, v, e1, s2, nt, P, 8>), dim3(g.n_blocks),
                                               dim3(t.block), 0, s, a, X, Y);
                            break;
                        case 16:
                            hipLaunchKernelGGL((k_lap_stencil_passes<T, v, e1, s2, nt, P, 16>), dim3(g.n_blocks),
                                               dim3(t.block), 0, s, a, X, Y);
                            break;
                        default:
                            hipLaunchKernelGGL((k_lap_stencil_passes<T, v, e1, s2, nt, P, 0>), dim3(g.n_blocks),
                                               dim3(t.block), 0, s, a, X, Y);
                            break;
                    }
                };
                if (passes == 4)
                    passes_kernel(std::integral_constant<int, 4>{});
                else if (passes == 2)
                    passes_kernel(std::integral_constant<int, 2>{});
                else if (t.lanes_per_row == 64)
                    hipLaunchKernelGGL((k_lap_stencil<T, v, e1, s2, nt, true>), dim3(g.n_blocks), dim3(t.block), 0, s,
                                       a, X, Y);
                else
                    hipLaunchKernelGGL((k_lap_stencil<T, v, e1, s2, nt, false>), dim3(g.n_blocks), dim3(t.block), 0, s,
                                       a, X, Y);
            };
            t.nt_store ? launch(std::true_type{}) : launch(std::false_type{});
        };
        if (op->stencil == 27)
            go(std::true_type{}, std::false_type{});
        else
            go(std::false_type{}, std::true_type{});
    });
    FVX_HIP(hipGetLastError());
}

template <typename T>
void launch_lap(const fvx_op *op, const T *X, T *Y, const double *cs, hipStream_t s) {
    if (op->stencil != 7) {
        launch_lap_stencil<T>(op, X, Y, cs, s);
        return;
    }
    RowGrid g;
    const fvx_tile &t = op->tile[dtype_of<T>()];
    auto a = row_args<T>(op, op->n_b, g, t);
    by_vec<T>(t.vec, op->zfaces, [&](auto V, auto Z) {
        by_width(op->W, [&](auto Wt) {
            constexpr int v = decltype(V)::value, wt = decltype(Wt)::value;
            constexpr bool z = decltype(Z)::value;
            constexpr bool can_stage = wt > 0;
            const size_t shm = stage_bytes<T, wt>(g.rows_per_tile);
            const bool st = can_stage && t.stage_lds;
            const int span = t.lanes_per_row * v;
            const int passes = op->k % span == 0 ? op->k / span : 0;
            if (a.A.cart && !st && span == op->k && t.lanes_per_row >= 8) {
                const bool o32 = uint64_t(op->n_b) * uint64_t(op->ld) * sizeof(T) < (uint64_t(1) << 32);
                CartArgs<T> ca;
                ca.rec = a.A.cart;
                ca.nx = uint32_t(a.A.cart_nx);
                ca.ny = uint32_t(a.A.cart_ny);
                ca.n_b = uint32_t(op->n_b);
                ca.ld = uint32_t(op->ld);
                ca.rows_per_tile = uint32_t(g.rows_per_tile);
                ca.n_tiles = uint32_t(ceil_div(op->n_b, g.rows_per_tile));
                ca.n_xtiles = 0;
                ca.px = a.A.cart_px;
                ca.py = a.A.cart_py;
                ca.lpr = t.lanes_per_row;
                ca.remap = t.xcd_remap;
                const int lines = cart_lines(op->n_b, a.A.cart_nx, a.A.cart_ny, g.rows_per_tile, t.max_blocks);
                int n_blocks = g.n_blocks;
                if (lines > 1) {
                    ca.n_xtiles = uint32_t(ceil_div(a.A.cart_nx, g.rows_per_tile));
                    ca.n_tiles = ca.n_xtiles * uint32_t(ceil_div(a.A.cart_ny, lines));
                    n_blocks = int(std::min<int64_t>(ca.n_tiles, t.max_blocks));
                }
                // the row-group width (8, 16, 32 or 64 lanes here) as a constant, so
                // that the shuffles' source lanes fold, and the column scale as a flag
                auto launch = [&](auto NTt, auto Ot, auto Lt, auto Ct) {
                    constexpr bool nt = decltype(NTt)::value, o = decltype(Ot)::value, c = decltype(Ct)::value;
                    constexpr int L = decltype(Lt)::value;
                    if (lines == 4)
                        hipLaunchKernelGGL((k_lap_cart_lines<T, v, z, nt, o, 4, L, c>), dim3(n_blocks), dim3(t.block),
                                           0, s, ca, X, Y, cs);
                    else if (lines == 2)
                        hipLaunchKernelGGL((k_lap_cart_lines<T, v, z, nt, o, 2, L, c>), dim3(n_blocks), dim3(t.block),
                                           0, s, ca, X, Y, cs);
                    else
                        hipLaunchKernelGGL((k_lap_cart<T, v, z, nt, o, L, c>), dim3(n_blocks), dim3(t.block), 0, s, ca,
                                           X, Y, cs);
                };
                auto with_scale = [&](auto NTt, auto Ot, auto Lt) {
                    if (cs)
                        launch(NTt, Ot, Lt, std::true_type{});
                    else
                        launch(NTt, Ot, Lt, std::false_type{});
                };
                auto go = [&](auto NTt, auto Ot) {
                    switch (t.lanes_per_row) {
                        case 8: with_scale(NTt, Ot, std::integral_constant<int, 8>{}); break;
                        case 16: with_scale(NTt, Ot, std::integral_constant<int, 16>{}); break;
                        case 32: with_scale(NTt, Ot, std::integral_constant<int, 32>{}); break;
                        default: with_scale(NTt, Ot, std::integral_constant<int, 64>{}); break;
                    }
                };
                if (t.nt_store && o32)
                    go(std::true_type{}, std::true_type{});
                else if (t.nt_store)
                    go(std::true_type{}, std::false_type{});
                else if (o32)
                    go(std::false_type{}, std::true_type{});
                else
                    go(std::false_type{}, std::false_type{});
                return;
            }
            if constexpr (wt > 0) {
                if (!st && (passes == 2 || passes == 4) && t.block <= 512) {  // its launch bound
                    auto go = [&](auto Pt) {
                        constexpr int P = decltype(Pt)::value;
                        if (t.nt_store)
                            hipLaunchKernelGGL((k_lap_passes<T, v, z, wt, true, P>), dim3(g.n_blocks), dim3(t.block), 0,
                                               s, a, X, Y, cs);
                        else
                            hipLaunchKernelGGL((k_lap_passes<T, v, z, wt, false, P>), dim3(g.n_blocks), dim3(t.block),
                                               0, s, a, X, Y, cs);
                    };
                    if (passes == 2)
                        go(std::integral_constant<int, 2>{});
                    else
                        go(std::integral_constant<int, 4>{});
                    return;
                }
            }
            if (st && t.nt_store)
                hipLaunchKernelGGL((k_lap<T, v, z, wt, can_stage, true>), dim3(g.n_blocks), dim3(t.block), shm, s, a,
                                   X, Y, cs);
            else if (st)
                hipLaunchKernelGGL((k_lap<T, v, z, wt, can_stage, false>), dim3(g.n_blocks), dim3(t.block), shm, s, a,
                                   X, Y, cs);
            else if (t.nt_store)
                hipLaunchKernelGGL((k_lap<T, v, z, wt, false, true>), dim3(g.n_blocks), dim3(t.block), 0, s, a, X, Y,
                                   cs);
            else
                hipLaunchKernelGGL((k_lap<T, v, z, wt, false, false>), dim3(g.n_blocks), dim3(t.block), 0, s, a, X, Y,
                                   cs);
        });
    });
    FVX_HIP(hipGetLastError());
}

template <typename T>
void launch_div(const fvx_op *op, const T *U, const T *Wz, T *D, hipStream_t s) {
    RowGrid g;
    const fvx_tile &t = op->tile[dtype_of<T>()];
    auto a = row_args<T>(op, op->n_b, g, t);
    by_vec<T>(t.vec, op->zfaces, [&](auto V, auto Z) {
        by_width(op->Wd, [&](auto Wt) {
            hipLaunchKernelGGL((k_div<T, decltype(V)::value, decltype(Z)::value, decltype(Wt)::value>),
                               dim3(g.n_blocks), dim3(t.block), 0, s, a, U, Wz, D);
        });
    });
    FVX_HIP(hipGetLastError());
}

template <typename T>
void launch_convect(const fvx_op *op, const T *U, const T *Wz, const T *Phi, T *Out, hipStream_t s) {
    RowGrid g;
    fvx_tile t = op->tile[dtype_of<T>()];
    t.block = std::min(t.block, kConvectBlock);  // rows are independent: any block size gives the same result
    auto a = row_args<T>(op, op->n_b, g, t);
    by_vec<T>(t.vec, op->zfaces, [&](auto V, auto Z) {
        by_width(op->Wd, [&](auto Wt) {
            hipLaunchKernelGGL((k_convect<T, decltype(V)::value, decltype(Z)::value, decltype(Wt)::value>),
                               dim3(g.n_blocks), dim3(t.block), 0, s, a, U, Wz, Phi, Out);
        });
    });
    FVX_HIP(hipGetLastError());
}

template <typename T>
void launch_grad(const fvx_op *op, const T *P, T *Gf, T *Gz, hipStream_t s, double alpha, bool acc) {
    RowGrid g;
    const int64_t rows = op->F_b + (op->zfaces ? op->n_b : 0);
    const fvx_tile &t = op->tile[dtype_of<T>()];
    auto a = row_args<T>(op, rows, g, t);
    by_vec<T>(t.vec, op->zfaces, [&](auto V, auto Z) {
        hipLaunchKernelGGL((k_grad<T, decltype(V)::value, decltype(Z)::value>), dim3(g.n_blocks), dim3(t.block), 0,
                           s, a, P, Gf, Gz, T(alpha), int(acc));
    });
    FVX_HIP(hipGetLastError());
}

template <typename T>
void launch_pack(const fvx_op *op, int64_t n_rows, const T *src, T *dst, bool to_rows, hipStream_t s) {
    const int64_t n = n_rows * op->k;
    const int blocks = int(std::min<int64_t>(std::max<int64_t>(1, ceil_div(n, 256)), 65536));
    hipLaunchKernelGGL((k_pack<T>), dim3(blocks), dim3(256), 0, s, n_rows, op->k, op->ld, src, dst, int(to_rows));
    FVX_HIP(hipGetLastError());
}

template void launch_lap<double>(const fvx_op *, const double *, double *, const double *, hipStream_t);
template void launch_lap<float>(const fvx_op *, const float *, float *, const double *, hipStream_t);
template void launch_div<double>(const fvx_op *, const double *, const double *, double *, hipStream_t);
template void launch_div<float>(const fvx_op *, const float *, const float *, float *, hipStream_t);
template void launch_convect<double>(const fvx_op *, const double *, const double *, const double *, double *,
                                     hipStream_t);
template void launch_convect<float>(const fvx_op *, const float *, const float *, const float *, float *, hipStream_t);
template void launch_grad<double>(const fvx_op *, const double *, double *, double *, hipStream_t, double, bool);
template void launch_grad<float>(const fvx_op *, const float *, float *, float *, hipStream_t, double, bool);
template void launch_pack<double>(const fvx_op *, int64_t, const double *, double *, bool, hipStream_t);
template void launch_pack<float>(const fvx_op *, int64_t, const float *, float *, bool, hipStream_t);

}  // namespace fvx

using fvx::guard;

extern "C" {

int fvx_lap(const fvx_op *op, int dtype, const void *X, void *Y, const double *colscale, void *stream) {
    return guard([&] {
        fvx::check_dtype(op, dtype);
        fvx::check_ptr(X, "X");
        fvx::check_ptr(Y, "Y");
        FVX_REQUIRE(X != Y, FVX_E_ARG, "X and Y must not overlap");
        if (dtype == FVX_F64)
            fvx::launch_lap<double>(op, static_cast<const double *>(X), static_cast<double *>(Y), colscale,
                                    fvx::as_stream(stream));
        else
            fvx::launch_lap<float>(op, static_cast<const float *>(X), static_cast<float *>(Y), colscale,
                                   fvx::as_stream(stream));
        return FVX_OK;
    });
}

int fvx_lap_many(const fvx_op *op, int dtype, int n, const void *const *X, void *const *Y, void *stream) {
    return guard([&] {
        fvx::check_dtype(op, dtype);
        FVX_REQUIRE(n >= 0 && (n == 0 || (X && Y)), FVX_E_ARG, "bad pointer arrays");
        for (int i = 0; i < n; ++i) {
            fvx::check_ptr(X[i], "X[i]");
            fvx::check_ptr(Y[i], "Y[i]");
            FVX_REQUIRE(X[i] != Y[i], FVX_E_ARG, "X[i] and Y[i] must not overlap");
        }
        hipStream_t s = fvx::as_stream(stream);
        for (int i = 0; i < n; ++i) {
            if (dtype == FVX_F64)
                fvx::launch_lap<double>(op, static_cast<const double *>(X[i]), static_cast<double *>(Y[i]), nullptr, s);
            else
                fvx::launch_lap<float>(op, static_cast<const float *>(X[i]), static_cast<float *>(Y[i]), nullptr, s);
        }
        return FVX_OK;
    });
}

int fvx_div(const fvx_op *op, int dtype, const void *Uf, const void *Wz, void *D, void *stream) {
    return guard([&] {
        fvx::check_dtype(op, dtype);
        if (op->F_b > 0) fvx::check_ptr(Uf, "Uf");
        if (op->zfaces) fvx::check_ptr(Wz, "Wz");
        fvx::check_ptr(D, "D");
        if (dtype == FVX_F64)
            fvx::launch_div<double>(op, static_cast<const double *>(Uf), static_cast<const double *>(Wz),
                                    static_cast<double *>(D), fvx::as_stream(stream));
        else
            fvx::launch_div<float>(op, static_cast<const float *>(Uf), static_cast<const float *>(Wz),
                                   static_cast<float *>(D), fvx::as_stream(stream));
        return FVX_OK;
    });
}

static int grad_impl(const fvx_op *op, int dtype, const void *P, void *Gf, void *Gz, void *stream, double alpha,
                     bool acc) {
    return guard([&] {
        fvx::check_dtype(op, dtype);
        fvx::check_ptr(P, "P");
        if (op->F_b > 0) fvx::check_ptr(Gf, "Gf");
        if (op->zfaces) fvx::check_ptr(Gz, "Gz");
        if (op->F_b == 0 && !op->zfaces) return FVX_OK;
        if (dtype == FVX_F64)
            fvx::launch_grad<double>(op, static_cast<const double *>(P), static_cast<double *>(Gf),
                                     static_cast<double *>(Gz), fvx::as_stream(stream), alpha, acc);
        else
            fvx::launch_grad<float>(op, static_cast<const float *>(P), static_cast<float *>(Gf),
                                    static_cast<float *>(Gz), fvx::as_stream(stream), alpha, acc);
        return FVX_OK;
    });
}

int fvx_convect(const fvx_op *op, int dtype, const void *Uf, const void *Wz, const void *Phi, void *Out,
                void *stream) {
    return guard([&] {
        fvx::check_dtype(op, dtype);
        fvx::check_ptr(Uf, "Uf");
        fvx::check_ptr(Phi, "Phi");
        fvx::check_ptr(Out, "Out");
        FVX_REQUIRE(!op->zfaces || Wz, FVX_E_ARG, "Wz is required when the planes are coupled");
        FVX_REQUIRE(Out != Phi && Out != Uf && (!Wz || Out != Wz), FVX_E_ARG, "Out must not overlap the inputs");
        if (dtype == FVX_F64)
            fvx::launch_convect<double>(op, static_cast<const double *>(Uf), static_cast<const double *>(Wz),
                                        static_cast<const double *>(Phi), static_cast<double *>(Out),
                                        fvx::as_stream(stream));
        else
            fvx::launch_convect<float>(op, static_cast<const float *>(Uf), static_cast<const float *>(Wz),
                                       static_cast<const float *>(Phi), static_cast<float *>(Out),
                                       fvx::as_stream(stream));
        return FVX_OK;
    });
}

int fvx_grad(const fvx_op *op, int dtype, const void *P, void *Gf, void *Gz, void *stream) {
    return grad_impl(op, dtype, P, Gf, Gz, stream, 1.0, false);
}

int fvx_grad_axpy(const fvx_op *op, int dtype, double alpha, const void *P, void *Gf, void *Gz, void *stream) {
    return grad_impl(op, dtype, P, Gf, Gz, stream, alpha, true);
}

int fvx_pack(const fvx_op *op, int dtype, int64_t n_rows, const void *src, void *dst, void *stream) {
    return guard([&] {
        fvx::check_dtype(op, dtype);
        FVX_REQUIRE(src && dst && n_rows >= 0, FVX_E_ARG, "NULL buffer or negative rows");
        if (n_rows == 0) return FVX_OK;
        if (dtype == FVX_F64)
            fvx::launch_pack<double>(op, n_rows, static_cast<const double *>(src), static_cast<double *>(dst), true,
                                     fvx::as_stream(stream));
        else
            fvx::launch_pack<float>(op, n_rows, static_cast<const float *>(src), static_cast<float *>(dst), true,
                                    fvx::as_stream(stream));
        return FVX_OK;
    });
}

int fvx_unpack(const fvx_op *op, int dtype, int64_t n_rows, const void *src, void *dst, void *stream) {
    return guard([&] {
        fvx::check_dtype(op, dtype);
        FVX_REQUIRE(src && dst && n_rows >= 0, FVX_E_ARG, "NULL buffer or negative rows");
        if (n_rows == 0) return FVX_OK;
        if (dtype == FVX_F64)
            fvx::launch_pack<double>(op, n_rows, static_cast<const double *>(src), static_cast<double *>(dst), false,
                                     fvx::as_stream(stream));
        else
            fvx::launch_pack<float>(op, n_rows, static_cast<const float *>(src), static_cast<float *>(dst), false,
                                    fvx::as_stream(stream));
        return FVX_OK;
    });
}

}  // extern "C"
