// Aggregation multigrid preconditioner: the hierarchy object and the V-cycle
// used by the CG driver.
#pragma once

#include <memory>
#include <vector>

#include "cg_rows.h"

namespace fvx {
constexpr int kMaxAmgLevels = 16;
constexpr int kMaxAmgDegree = 8;
constexpr int kMaxAmgCoarse = 2048;
}  // namespace fvx

struct fvx_amg {
    struct Level {
        const fvx_op *op = nullptr;          // level 0: the caller's operator
        std::unique_ptr<fvx_op> own;         // coarse levels: built by the hierarchy
        int kind = 0;                        // how the next level is made: 0 none (coarsest), 1 base, 2 planes
        std::vector<int32_t> agg;            // kind 1: base cell -> aggregate (host)
        const int32_t *agg_dev = nullptr;    // kind 1: the same on the device
        const int32_t *mem_ptr = nullptr;    // kind 1: members of each aggregate (CSR over the next level's rows)
        const int32_t *mem_idx = nullptr;
    };
    std::vector<Level> lv;
    fvx_amg_opts o{};
    bool coupled = false;                    // planes coupled (one system); else k independent systems
    int n_d = 0;                             // unknowns of the coarsest dense solve per system
    int modes = 0;                           // > 0: coarsest solved per plane (mode): coupled planes floor(k/2) + 1
                                             //   mode systems of n_d = n_b; independent planes 1, shared
    const double *pinv64 = nullptr;          // [n_d][n_d] coarsest pseudo-inverse (AoS order: cell, plane),
    const float *pinv32 = nullptr;           //   or [modes][n_d][n_d], one per plane mode
    const double *phi = nullptr;             // coupled modes: [k][k] real Fourier basis, row j = basis function j
    const double *phi_t = nullptr;           //   and its transpose
    double inv_theta = 1.0;
    double c1[fvx::kMaxAmgDegree] = {}, c2[fvx::kMaxAmgDegree] = {};  // smoother step j uses c1[j], c2[j]
    uint64_t serial = fvx::next_serial();
};

namespace fvx {

// Per-level vectors of one V-cycle in precision T: r (restricted right-hand
// side; unused on level 0), s[2] (pre-smoothing), q[2] (post-smoothing);
// the coarsest level uses r and q[0].
template <typename T>
struct AmgWork {
    struct Lv {
        T *r = nullptr, *s[2] = {nullptr, nullptr}, *q[2] = {nullptr, nullptr};
    };
    Lv lv[kMaxAmgLevels];
    double *mr = nullptr, *mz = nullptr;  // plane modes: [k][n_b] right-hand sides and solutions
    CgState *st = nullptr;                // a never-set "done" flag for calls outside a solve
};

// Bytes of the V-cycle vectors of precision dtype (plus the flag).
size_t amg_work_bytes(const fvx_amg *h, int dtype);
// Pointers into base (nullptr: sizes only).
template <typename T>
AmgWork<T> amg_carve(const fvx_amg *h, char *base);
// The level-0 buffer that receives z.
template <typename T>
T *amg_output(const fvx_amg *h, const AmgWork<T> &w);

// The launch of the last post-smoothing step on level 0 inside a solve: the
// CG's own tile and grid, so that its r.z partials land where the CG reads
// them.
template <typename T>
struct AmgFinal {
    RowArgs<T> a;
    dim3 grid, block;
    int vec;
};

// One V-cycle z = M^-1 r on the stream.  Every kernel returns at once when
// d.st->done is set.  fin: the CG's launch of the last step (writes the r.z
// partials of d), or nullptr.
template <typename T>
void amg_vcycle(const fvx_amg *h, const T *r, const AmgWork<T> &w, const CgDev &d, const AmgFinal<T> *fin,
                hipStream_t s);

// Requirements of a solve preconditioned by h on op.
void amg_check_solve(const fvx_amg *h, const fvx_op *op, bool mixed);

}  // namespace fvx
