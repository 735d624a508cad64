// Internal declarations shared by the host builder, the HIP kernels and the
// C-ABI entry points of libfvx.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <functional>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "fvx.h"

// ---------------------------------------------------------------------------
// Host-side objects behind the opaque handles
// ---------------------------------------------------------------------------

namespace fvx {
// A process-wide number that no later object takes again (an address can be
// reused after a free; a serial cannot).  Cached launch graphs are keyed by it.
inline uint64_t next_serial() {
    static std::atomic<uint64_t> n{1};
    return n.fetch_add(1);
}
}  // namespace fvx

struct fvx_mesh {
    int n_cells = 0, n_faces = 0, n_walls = 0;
    int grid_nx = 0, grid_ny = 0;  // Cartesian builder: cell (i, j) is j*nx + i; 0 otherwise
    std::vector<double> xf, yf;    // Cartesian builder: face coordinates along x and y
    bool periodic_x = false, periodic_y = false;
    std::vector<double> area, cx, cy;
    std::vector<int32_t> c1, c2;
    std::vector<double> len, dist;
    std::vector<double> fnx, fny;  // unit face normal from c1 to c2 (empty when the builder has no geometry)
    std::vector<int32_t> wcell;
    std::vector<double> wlen, wdist;
};

namespace fvx {

// Device arrays of one precision.  All sizes are fixed by the base mesh; none
// grows with the number of planes k.
template <typename T>
struct OpDev {
    // Laplacian base block A_b: diagonal plus off-diagonal neighbours in
    // column-major ELL ([W][n_b]: entry e of row i at e*n_b + i; padding
    // entries point at the row itself with value 0).
    const T *diag = nullptr;
    const int32_t *ell_col = nullptr;
    const T *ell_val = nullptr;
    const T *w = nullptr;        // [n_b] plane-coupling weight area_i / dz
    // Divergence M_b: cell -> face incidence, column-major ELL [Wd][n_b],
    // coefficient +-len_f*dz (+ when the cell is the face's c1).
    const int32_t *cf_face = nullptr;
    const T *cf_coef = nullptr;
    const T *area = nullptr;     // [n_b] cell area (flux through faces between planes)
    // Gradient: per face its cells and 1/dist.
    const int32_t *f_c1 = nullptr, *f_c2 = nullptr;
    const T *f_invd = nullptr;
    T inv_dz = 0;
    // Structured 13/27-point operators: per ELL entry the coefficient of the
    // neighbour's planes l +- 1 (27-point), and the row's own planes l +- 2
    // coefficient (13-point); NULL otherwise.
    const T *ell_v1 = nullptr;
    const T *w2 = nullptr;
    // The same operators with their entries in the fixed direction order: per
    // row one record of srec_width(stencil) coefficients (8 in-plane entries,
    // diagonal, w, then 8 neighbouring-plane entries or w2); NULL otherwise.
    const T *srec = nullptr;
    // Jacobi scaling of the SPD form -L: 1 / (-diag) per base row (1 where
    // the diagonal vanishes), shared by the k planes.
    const T *dinv = nullptr;
    // Velocity interpolation of the time step (NULL when the mesh has no face
    // normals): cell -> face, u_f = n_f . (u_c1 + u_c2) / 2; face -> cell,
    // the adjoint weighted by face and cell volumes,
    //   (Gamma_sc g)_c = sum_f (len_f dist_f / (2 area_c)) n_f g_f.
    const T *fnx = nullptr, *fny = nullptr;   // [F_b]
    const T *gsx = nullptr, *gsy = nullptr;   // [F_b] len_f dist_f n_f / 2
    const T *inv_area = nullptr;              // [n_b]
    // Cartesian base (cell (i, j) at j*nx + i) whose face graph is the
    // 5-point stencil: per row [diag, w, c_S, c_W, c_E, c_N, 0, 0] with the
    // neighbours' indices computed from (i, j) (an absent neighbour has
    // coefficient 0); NULL when the base is not such a grid.
    const T *cart = nullptr;
    int cart_nx = 0, cart_ny = 0, cart_px = 0, cart_py = 0;
};

}  // namespace fvx

struct fvx_op {
    int64_t n_b = 0, F_b = 0, nnz_b = 0;
    int32_t k = 0, ld = 0, coupling = 0;
    bool zfaces = false;    // faces between planes exist (periodic coupling, k >= 2)
    bool singular = true;   // L has the constant null space
    bool percol = false;    // columns are independent systems
    double dz = 0;
    int W = 0, Wd = 0;      // ELL widths (Laplacian off-diagonals, cell->face)
    bool has_f32 = false;
    int grid_nx = 0, grid_ny = 0;  // structured base (Cartesian builder), else 0
    int stencil = 7;                // 7: finite-volume face graph; 13, 27: structured operators
    int grid_px = 0, grid_py = 0;   // structured base: periodic x / y
    bool stencil_dir = false;       // 13/27: ELL entries in the fixed direction order (see op.cpp)
    int device = 0;
    fvx::OpDev<double> d64;
    fvx::OpDev<float> d32;
    fvx_tile tile[2];
    fvx_tile cg_tile[2] = {};  // CG launch tile per precision (block 0: not set)
    uint64_t serial = fvx::next_serial();
};

namespace fvx {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &s) : std::runtime_error(s), code(c) {}
};

void set_last_error(const std::string &s);

// Runs f and converts exceptions into status codes; records the message.
int guard(const std::function<int()> &f);

#define FVX_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::fvx::Error(FVX_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define FVX_REQUIRE(cond, code, msg)                     \
    do {                                                 \
        if (!(cond)) throw ::fvx::Error((code), (msg));  \
    } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int kMaxStageRows = 64;  // rows per tile whose base-block rows fit the LDS stage
inline int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Row stride of multivectors for k planes: k itself when k <= 2 or a multiple
// of 4, else k rounded up to a multiple of 4 (so 16-byte vector loads stay
// aligned for both precisions).
// Coefficients per row of a structured operator's packed record (13-point:
// 11, padded to 12 for 16-byte records).
constexpr int srec_width(int stencil) { return stencil == 27 ? 18 : 12; }

inline int32_t ld_for_k(int32_t k) { return (k <= 2 || k % 4 == 0) ? k : (k + 3) / 4 * 4; }

// ELL widths the kernels are compiled for (all gathers of a row issue before
// the first multiply-add); rows are padded to the next of them.  Wider rows
// use a loop over a run-time width.
inline int ell_width(int w) {
    if (w == 0) return 0;  // no neighbours: nothing to gather, nothing to pad
    for (int c : {3, 4, 6, 8})
        if (w <= c) return c;
    return w;
}

// Calls f(std::integral_constant<int, W>) for a compiled width, or with 0
// (run-time width) otherwise.
template <typename F>
void by_width(int w, F &&f) {
    switch (w) {
        case 3: f(std::integral_constant<int, 3>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        case 6: f(std::integral_constant<int, 6>{}); break;
        case 8: f(std::integral_constant<int, 8>{}); break;
        default: f(std::integral_constant<int, 0>{}); break;
    }
}

fvx_tile default_tile(const fvx_op *op, int dtype);
void check_tile(const fvx_op *op, int dtype, const fvx_tile &t);

// ---------------------------------------------------------------------------
// Launchers (spmm.hip)
// ---------------------------------------------------------------------------
template <typename T>
void launch_lap(const fvx_op *op, const T *X, T *Y, const double *colscale, hipStream_t s);
template <typename T>
void launch_div(const fvx_op *op, const T *U, const T *Wz, T *D, hipStream_t s);
template <typename T>
void launch_convect(const fvx_op *op, const T *U, const T *Wz, const T *Phi, T *Out, hipStream_t s);
template <typename T>
void launch_grad(const fvx_op *op, const T *P, T *Gf, T *Gz, hipStream_t s, double alpha = 1.0,
                 bool acc = false);
template <typename T>
void launch_pack(const fvx_op *op, int64_t n_rows, const T *src, T *dst, bool to_rows, hipStream_t s);

template <typename T>
const OpDev<T> &dev(const fvx_op *op);
template <>
inline const OpDev<double> &dev<double>(const fvx_op *op) { return op->d64; }
template <>
inline const OpDev<float> &dev<float>(const fvx_op *op) { return op->d32; }

template <typename T>
inline int dtype_of();
template <>
inline int dtype_of<double>() { return FVX_F64; }
template <>
inline int dtype_of<float>() { return FVX_F32; }

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Number of thread blocks of a row-tiled launch: each block walks a contiguous
// range of row tiles.  Blocks are capped so per-block reduction partials stay
// small; plain SpMMs use a large cap.
struct RowGrid {
    int64_t n_rows;
    int rows_per_tile;   // rows one block covers per step = block / lanes_per_row
    int64_t tiles_per_block;
    int n_blocks;
};
RowGrid row_grid(int64_t n_rows, const fvx_tile &t, int max_blocks);

// Assembled 3D Laplacian (plane-major rows l*n_b + c) expanded from the base
// block and the plane coupling: the "no block reuse" form of the operator.
void expand_csr(const fvx_mesh &m, const fvx_op_desc &d, std::vector<int32_t> &ptr, std::vector<int32_t> &col,
                std::vector<double> &val);

// max over the CG groups of ||bp - L x|| / ||bp|| (bp: b after the solver's
// projection) for a given x, in FP64; +inf when a value is not finite or a
// group has bp = 0 but a nonzero residual.  ws: a solve workspace of op.
// Synchronises s.
double guess_residual_ratio(const fvx_op *op, const double *B, const double *X, void *ws, hipStream_t s);

}  // namespace fvx
