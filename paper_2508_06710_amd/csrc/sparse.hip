// A general sparse matrix applied to a multivector: Y = diag(c) (A X), A any
// n_rows x n_cols CSR matrix (rectangular allowed), X and Y row-major
// multivectors of k columns (Section 2, Algorithm 1: every stored entry of A
// is read once per row group and applied to all k columns).  This is the
// operator form of the coarse-to-fine state mapping of the inline mesh
// refinement (Section 3.3) and of any other block-repeated product.
#include "kernels.h"

struct fvx_sparse {
    int64_t n_rows = 0, n_cols = 0, nnz = 0;
    bool has_f32 = false;
    int device = 0;
    const int32_t *ptr = nullptr, *col = nullptr;
    const double *val64 = nullptr;
    const float *val32 = nullptr;
    fvx_tile tile[2] = {};  // block 0: not set (a default is derived from k and the strides)
};

namespace fvx {
namespace {

template <typename T>
struct SpArgs {
    const int32_t *ptr, *col;
    const T *val;
    const double *colscale;
    int64_t n_rows;
    int k, ldx, ldy, lpr, cpr, rows_per_tile, remap;  // cpr: lanes per row that own columns
    int64_t tiles_per_block;
};

// Lanes of a row group that own columns: enough to cover k with V columns
// each (a power of two, at most lanes_per_row).  The remaining factor
// lanes_per_row / cpr splits the row's nonzeros.
inline int column_lanes(int k, int vec, int lpr) { return std::min(lpr, next_pow2(int(ceil_div(k, vec)))); }

// Row group of lpr lanes per row: cpr lanes own V consecutive columns each
// per pass, and S = lpr / cpr such sub-groups split the row's nonzeros
// (sub-group s takes entries s, s + S, ...) and add their sums by shuffles.
// Each sub-group applies its entries in order with fused multiply-adds, so
// tiles with the same split factor S give bitwise the same product.
template <typename T, int V, bool NT>
__global__ __launch_bounds__(1024) void k_spmm_csr(SpArgs<T> a, const T *__restrict__ X, T *__restrict__ Y) {
    using vt = vec_t<T, V>;
    const int sub = threadIdx.x & (a.lpr - 1);
    const int grp = threadIdx.x / a.lpr;
    const int cl = sub & (a.cpr - 1), sg = sub / a.cpr, S = a.lpr / a.cpr;
    const int64_t t0 = logical_block(a.remap) * a.tiles_per_block;
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        const int32_t j0 = a.ptr[row], j1 = a.ptr[row + 1];
        for (int c0 = cl * V; c0 < a.k; c0 += a.cpr * V) {
            vt acc = vt(0);
            for (int32_t j = j0 + sg; j < j1; j += S)
                acc = __builtin_elementwise_fma(vt(a.val[j]), ldv<T, V>(X + int64_t(a.col[j]) * a.ldx + c0), acc);
            // partners differ only in the split bits, so they share cl and the pass count
            for (int o = a.cpr; o < a.lpr; o <<= 1) {
#pragma unroll
                for (int u = 0; u < V; ++u) acc[u] += __shfl_xor(acc[u], o, a.lpr);
            }
            if (sg != 0) continue;
            if (a.colscale) {
#pragma unroll
                for (int u = 0; u < V; ++u)
                    if (c0 + u < a.k) acc[u] = T(a.colscale[c0 + u]) * acc[u];
            }
            stv_masked<T, V, NT>(Y + row * a.ldy + c0, acc, a.k - c0);
        }
    }
}

fvx_tile default_sparse_tile(int dtype, int k, int ldx, int ldy) {
    fvx_tile t{};
    const int vmax = dtype == FVX_F32 ? 4 : 2;
    t.vec = 1;
    for (int c = vmax; c >= 1; c >>= 1)
        if (ldx % c == 0 && ldy % c == 0) {
            t.vec = c;
            break;
        }
    t.lanes_per_row = std::min(64, next_pow2(int(ceil_div(k, t.vec))));
    t.block = 256;
    t.xcd_remap = 1;
    return t;
}

void check_sparse_tile(int dtype, const fvx_tile &t) {
    const int vmax = dtype == FVX_F32 ? 4 : 2;
    FVX_REQUIRE(t.vec == 1 || t.vec == 2 || (t.vec == 4 && vmax == 4), FVX_E_ARG,
                "tile.vec must be 1 or 2 (FP64), 1, 2 or 4 (FP32)");
    FVX_REQUIRE(t.lanes_per_row >= 1 && t.lanes_per_row <= 64 && (t.lanes_per_row & (t.lanes_per_row - 1)) == 0,
                FVX_E_ARG, "tile.lanes_per_row must be a power of two in 1..64");
    FVX_REQUIRE(t.block >= 64 && t.block <= 1024 && t.block % 64 == 0 && t.block >= t.lanes_per_row, FVX_E_ARG,
                "tile.block must be a multiple of 64 in 64..1024");
    FVX_REQUIRE(t.max_blocks >= 0 && t.stage_lds == 0 && (t.nt_store == 0 || t.nt_store == 1), FVX_E_ARG,
                "tile.max_blocks >= 0, stage_lds 0, nt_store 0 or 1");
}

template <typename T>
void launch_spmm(const fvx_sparse *A, int dtype, int k, const T *X, int ldx, T *Y, int ldy, const double *cs,
                 hipStream_t s) {
    fvx_tile t = A->tile[dtype].block > 0 ? A->tile[dtype] : default_sparse_tile(dtype, k, ldx, ldy);
    FVX_REQUIRE(ldx % t.vec == 0 && ldy % t.vec == 0, FVX_E_ARG, "tile.vec must divide ldx and ldy");
    FVX_REQUIRE(ldx >= ceil_div(k, t.vec) * t.vec && ldy >= k, FVX_E_ARG,
                "ldx must hold k columns rounded up to the vector width; ldy >= k");
    SpArgs<T> a{};
    a.ptr = A->ptr;
    a.col = A->col;
    a.val = dtype == FVX_F64 ? reinterpret_cast<const T *>(A->val64) : reinterpret_cast<const T *>(A->val32);
    a.colscale = cs;
    a.n_rows = A->n_rows;
    a.k = k;
    a.ldx = ldx;
    a.ldy = ldy;
    a.lpr = t.lanes_per_row;
    a.cpr = column_lanes(k, t.vec, t.lanes_per_row);
    a.rows_per_tile = t.block / t.lanes_per_row;
    a.remap = t.xcd_remap;
    const int64_t tiles = std::max<int64_t>(1, ceil_div(A->n_rows, a.rows_per_tile));
    const int64_t nb = std::min<int64_t>(tiles, t.max_blocks > 0 ? t.max_blocks : (int64_t(1) << 22));
    a.tiles_per_block = ceil_div(tiles, nb);
    const int n_blocks = int(ceil_div(tiles, a.tiles_per_block));
    auto go = [&](auto Vt) {
        constexpr int V = decltype(Vt)::value;
        if constexpr (V * sizeof(T) <= 16) {
            if (t.nt_store)
                hipLaunchKernelGGL((k_spmm_csr<T, V, true>), dim3(n_blocks), dim3(t.block), 0, s, a, X, Y);
            else
                hipLaunchKernelGGL((k_spmm_csr<T, V, false>), dim3(n_blocks), dim3(t.block), 0, s, a, X, Y);
        }
    };
    switch (t.vec) {
        case 1: go(std::integral_constant<int, 1>{}); break;
        case 2: go(std::integral_constant<int, 2>{}); break;
        default: go(std::integral_constant<int, 4>{}); break;
    }
    FVX_HIP(hipGetLastError());
}

struct SparseLayout {
    size_t ptr, col, val64, val32, total;
};

SparseLayout sparse_layout(int64_t n_rows, int64_t nnz, bool f32) {
    SparseLayout L{};
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += (b + 255) / 256 * 256;
        return o;
    };
    L.ptr = take(4 * size_t(n_rows + 1));
    L.col = take(4 * size_t(std::max<int64_t>(nnz, 1)));
    L.val64 = take(8 * size_t(std::max<int64_t>(nnz, 1)));
    L.val32 = f32 ? take(4 * size_t(std::max<int64_t>(nnz, 1))) : 0;
    L.total = off;
    return L;
}

void check_csr(int64_t n_rows, int64_t n_cols, const int32_t *ptr, const int32_t *col, const double *val) {
    FVX_REQUIRE(n_rows >= 1 && n_cols >= 1 && n_rows < (int64_t(1) << 31) && n_cols < (int64_t(1) << 31), FVX_E_ARG,
                "n_rows and n_cols must be in 1..2^31-1");
    FVX_REQUIRE(ptr && col && val, FVX_E_ARG, "NULL CSR array");
    FVX_REQUIRE(ptr[0] == 0, FVX_E_ARG, "ptr[0] must be 0");
    for (int64_t i = 0; i < n_rows; ++i) FVX_REQUIRE(ptr[i + 1] >= ptr[i], FVX_E_ARG, "ptr must be nondecreasing");
    for (int64_t j = 0; j < ptr[n_rows]; ++j) {
        FVX_REQUIRE(col[j] >= 0 && col[j] < n_cols, FVX_E_ARG, "column index out of range");
        FVX_REQUIRE(std::isfinite(val[j]), FVX_E_ARG, "non-finite matrix value");
    }
}

}  // namespace
}  // namespace fvx

using fvx::guard;

extern "C" {

int fvx_sparse_bytes(int64_t n_rows, int64_t nnz, int with_f32, size_t *bytes) {
    return guard([&] {
        FVX_REQUIRE(n_rows >= 1 && nnz >= 0 && bytes, FVX_E_ARG, "bad argument");
        *bytes = fvx::sparse_layout(n_rows, nnz, with_f32 != 0).total;
        return FVX_OK;
    });
}

int fvx_sparse_create(int64_t n_rows, int64_t n_cols, const int32_t *ptr, const int32_t *col, const double *val,
                      int with_f32, void *dev_mem, size_t bytes, void *stream, fvx_sparse **out) {
    return guard([&] {
        FVX_REQUIRE(out && dev_mem, FVX_E_ARG, "NULL argument");
        FVX_REQUIRE(reinterpret_cast<uintptr_t>(dev_mem) % 256 == 0, FVX_E_ARG, "device buffer must be 256-byte aligned");
        fvx::check_csr(n_rows, n_cols, ptr, col, val);
        const int64_t nnz = ptr[n_rows];
        const auto L = fvx::sparse_layout(n_rows, nnz, with_f32 != 0);
        FVX_REQUIRE(bytes >= L.total, FVX_E_NOMEM, "matrix buffer too small: need " + std::to_string(L.total));
        hipStream_t s = fvx::as_stream(stream);
        char *base = static_cast<char *>(dev_mem);
        FVX_HIP(hipMemcpyAsync(base + L.ptr, ptr, 4 * size_t(n_rows + 1), hipMemcpyHostToDevice, s));
        std::vector<float> v32;
        if (nnz > 0) {
            FVX_HIP(hipMemcpyAsync(base + L.col, col, 4 * size_t(nnz), hipMemcpyHostToDevice, s));
            FVX_HIP(hipMemcpyAsync(base + L.val64, val, 8 * size_t(nnz), hipMemcpyHostToDevice, s));
            if (with_f32) {
                v32.assign(val, val + nnz);
                FVX_HIP(hipMemcpyAsync(base + L.val32, v32.data(), 4 * size_t(nnz), hipMemcpyHostToDevice, s));
            }
        }
        FVX_HIP(hipStreamSynchronize(s));
        auto A = std::make_unique<fvx_sparse>();
        A->n_rows = n_rows;
        A->n_cols = n_cols;
        A->nnz = nnz;
        A->has_f32 = with_f32 != 0;
        A->ptr = reinterpret_cast<const int32_t *>(base + L.ptr);
        A->col = reinterpret_cast<const int32_t *>(base + L.col);
        A->val64 = reinterpret_cast<const double *>(base + L.val64);
        A->val32 = with_f32 ? reinterpret_cast<const float *>(base + L.val32) : nullptr;
        FVX_HIP(hipGetDevice(&A->device));
        *out = A.release();
        return FVX_OK;
    });
}

int fvx_sparse_destroy(fvx_sparse *A) {
    delete A;
    return FVX_OK;
}

int fvx_sparse_shape(const fvx_sparse *A, int64_t *n_rows, int64_t *n_cols, int64_t *nnz) {
    return guard([&] {
        FVX_REQUIRE(A, FVX_E_ARG, "NULL matrix");
        if (n_rows) *n_rows = A->n_rows;
        if (n_cols) *n_cols = A->n_cols;
        if (nnz) *nnz = A->nnz;
        return FVX_OK;
    });
}

int fvx_sparse_set_tile(fvx_sparse *A, int dtype, const fvx_tile *tile) {
    return guard([&] {
        FVX_REQUIRE(A && (dtype == FVX_F64 || (dtype == FVX_F32 && A->has_f32)), FVX_E_ARG, "bad matrix or dtype");
        if (!tile || tile->block == 0) {
            A->tile[dtype] = fvx_tile{};
            return FVX_OK;
        }
        fvx::check_sparse_tile(dtype, *tile);
        A->tile[dtype] = *tile;
        return FVX_OK;
    });
}

int fvx_sparse_spmm(const fvx_sparse *A, int dtype, int k, const void *X, int ldx, void *Y, int ldy,
                    const double *colscale, void *stream) {
    return guard([&] {
        FVX_REQUIRE(A && X && Y, FVX_E_ARG, "NULL argument");
        FVX_REQUIRE(dtype == FVX_F64 || (dtype == FVX_F32 && A->has_f32), FVX_E_ARG, "bad dtype for this matrix");
        FVX_REQUIRE(k >= 1 && ldx >= 1 && ldy >= 1, FVX_E_ARG, "k, ldx and ldy must be >= 1");
        FVX_REQUIRE(X != Y, FVX_E_ARG, "X and Y must not overlap");
        FVX_REQUIRE(reinterpret_cast<uintptr_t>(X) % 16 == 0 && reinterpret_cast<uintptr_t>(Y) % 16 == 0, FVX_E_ARG,
                    "X and Y must be 16-byte aligned");
        if (dtype == FVX_F64)
            fvx::launch_spmm<double>(A, dtype, k, static_cast<const double *>(X), ldx, static_cast<double *>(Y), ldy,
                                     colscale, fvx::as_stream(stream));
        else
            fvx::launch_spmm<float>(A, dtype, k, static_cast<const float *>(X), ldx, static_cast<float *>(Y), ldy,
                                    colscale, fvx::as_stream(stream));
        return FVX_OK;
    });
}

int fvx_sparse_tune(fvx_sparse *A, int dtype, int k, const void *X, int ldx, void *Y, int ldy, int reps,
                    void *stream, fvx_tune_result *results, int max_results, int *n_results) {
    return guard([&] {
        FVX_REQUIRE(A && X && Y && X != Y, FVX_E_ARG, "NULL or aliasing argument");
        FVX_REQUIRE(dtype == FVX_F64 || (dtype == FVX_F32 && A->has_f32), FVX_E_ARG, "bad dtype for this matrix");
        FVX_REQUIRE(k >= 1 && ldx >= k && ldy >= k, FVX_E_ARG, "k >= 1, ldx >= k, ldy >= k");
        hipStream_t s = fvx::as_stream(stream);
        reps = std::max(1, reps);
        // Row mappings first (vector width, lanes per row, workgroup), then the
        // launch options around the best one.
        std::vector<fvx_tile> shapes;
        const int vmax = dtype == FVX_F32 ? 4 : 2;
        for (int vec = vmax; vec >= 1; vec >>= 1) {
            if (ldx % vec || ldy % vec || ldx < fvx::ceil_div(k, vec) * vec) continue;
            const int base = std::min(64, fvx::next_pow2(int(fvx::ceil_div(k, vec))));
            // fewer lanes than columns (several passes), or more (split rows)
            for (int lpr = std::max(1, base / 4); lpr <= std::min(64, base * 8); lpr <<= 1)
                for (int block : {64, 128, 256, 512})
                    if (block >= lpr) shapes.push_back(fvx_tile{vec, lpr, block, 1, 0, 0, 0});
        }
        FVX_REQUIRE(!shapes.empty(), FVX_E_ARG, "no tile fits these strides");
        hipEvent_t e0, e1;
        FVX_HIP(hipEventCreate(&e0));
        FVX_HIP(hipEventCreate(&e1));
        const fvx_tile keep = A->tile[dtype];
        fvx_tile best = shapes[0];
        double best_us = 1e30;
        int n = 0;
        auto time_one = [&](const fvx_tile &t) {
            A->tile[dtype] = t;
            auto run = [&] {
                if (dtype == FVX_F64)
                    fvx::launch_spmm<double>(A, dtype, k, static_cast<const double *>(X), ldx, static_cast<double *>(Y),
                                             ldy, nullptr, s);
                else
                    fvx::launch_spmm<float>(A, dtype, k, static_cast<const float *>(X), ldx, static_cast<float *>(Y),
                                            ldy, nullptr, s);
            };
            run();
            FVX_HIP(hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r) run();
            FVX_HIP(hipEventRecord(e1, s));
            FVX_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            FVX_HIP(hipEventElapsedTime(&ms, e0, e1));
            const double us = 1e3 * double(ms) / reps;
            if (results && n < max_results) results[n] = fvx_tune_result{t, us};
            ++n;
            if (us < best_us) {
                best_us = us;
                best = t;
            }
        };
        try {
            for (const auto &t : shapes) time_one(t);
            const fvx_tile b = best;
            for (int cap : {0, 2048})
                for (int remap : {1, 0})
                    for (int nt : {0, 1}) {
                        if (cap == 0 && remap == 1 && nt == 0) continue;  // timed above
                        time_one(fvx_tile{b.vec, b.lanes_per_row, b.block, remap, cap, 0, nt});
                    }
        } catch (...) {
            A->tile[dtype] = keep;
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            throw;
        }
        A->tile[dtype] = best;
        if (n_results) *n_results = n;
        FVX_HIP(hipEventDestroy(e0));
        FVX_HIP(hipEventDestroy(e1));
        return FVX_OK;
    });
}

}  // extern "C"
