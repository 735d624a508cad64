// Aggregation multigrid preconditioner for the repeated-block Poisson
// operator (Section 4: CG preconditioned by an algebraic multigrid whose
// levels and transfers are all SpMMs over the stacked fields, Appendix A).
//
// Every level keeps the form I_k (x) A_b + C: the Galerkin product P^T A P
// with piecewise-constant aggregates P of such an operator is again one, with
// summed couplings.  Aggregating base cells sums in-plane couplings t, wall
// terms g and plane couplings w over the aggregates; merging planes 2l and
// 2l + 1 doubles t and g, keeps w and halves k.  So each coarse level is
// built as an ordinary fvx_op (from a face graph whose face coefficients are
// the coarse couplings, plane spacing 1) and runs the same SpMM kernels as
// the fine operator.  The host builds the hierarchy once; the device runs a
// V-cycle of
//   pre-smoothing   Chebyshev steps from z = 0 (the CG's fused step kernel),
//   restriction     r_c = P^T (r - A z), the residual's SpMM fused in,
//   coarse cycle    recursively; the coarsest level by its dense
//                   pseudo-inverse, or per plane mode (coupled planes: the
//                   real Fourier transform along the planes, the dense
//                   pseudo-inverse of each mode's base-plane system, the
//                   transform back),
//   prolongation    z += P e_c, fused with the first post-smoothing SpMM,
//   post-smoothing  Chebyshev steps from the corrected iterate.
#include <algorithm>
#include <cmath>
#include <exception>
#include <map>
#include <numeric>
#include <thread>

#include "amg.h"

namespace fvx {
namespace {

constexpr double kTie = 1e-9;  // couplings within this relative distance count as equal

// ---------------------------------------------------------------------------
// Host hierarchy
// ---------------------------------------------------------------------------

// One level on the host: in-plane couplings t (CSR, columns ascending, no
// diagonal), wall terms g, plane couplings w, cell areas, planes k.
struct HostLevel {
    int64_t n = 0;
    int k = 1;
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> val, g, w, area;
    int kind = 0;
    std::vector<int32_t> agg;  // kind 1
    int64_t nc = 0;            // kind 1: aggregates
};

void csr_from_maps(HostLevel &L, const std::vector<std::map<int32_t, double>> &rows) {
    L.ptr.assign(L.n + 1, 0);
    L.col.clear();
    L.val.clear();
    for (int64_t i = 0; i < L.n; ++i) {
        for (const auto &kv : rows[i]) {
            L.col.push_back(kv.first);
            L.val.push_back(kv.second);
        }
        L.ptr[i + 1] = int64_t(L.col.size());
    }
}

// The fine level from the mesh the operator was built from.
HostLevel fine_level(const fvx_mesh &m, const fvx_op *op, bool dirichlet) {
    HostLevel L;
    L.n = m.n_cells;
    L.k = op->k;
    std::vector<std::map<int32_t, double>> rows(L.n);
    for (int f = 0; f < m.n_faces; ++f) {
        const int a = m.c1[f], b = m.c2[f];
        if (a == b) continue;
        const double c = m.len[f] * op->dz / m.dist[f];
        rows[a][b] += c;
        rows[b][a] += c;
    }
    csr_from_maps(L, rows);
    L.g.assign(L.n, 0.0);
    if (dirichlet)
        for (int i = 0; i < m.n_walls; ++i) L.g[m.wcell[i]] += m.wlen[i] * op->dz / m.wdist[i];
    L.w.assign(L.n, 0.0);
    if (op->zfaces)
        for (int64_t i = 0; i < L.n; ++i) L.w[i] = m.area[i] / op->dz;
    L.area = m.area;
    return L;
}

// One pass of pairwise aggregation: cells in index order; a free cell joins
// its free neighbour of largest coupling among those at least beta times its
// largest coupling (ties to the smallest index), else stays alone.  Then each
// cell left alone (with a neighbour) joins, in index order, the aggregate of
// its neighbour of largest coupling -- otherwise a cell whose strong
// neighbours are always taken first stays alone on every level and the
// coarsening stalls (unstructured meshes) -- and the aggregates are numbered
// again in their order.
std::vector<int32_t> pairwise(int64_t n, const std::vector<int64_t> &ptr, const std::vector<int32_t> &col,
                              const std::vector<double> &val, double beta, int64_t &nc) {
    std::vector<int32_t> agg(n, -1);
    nc = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (agg[i] >= 0) continue;
        double mx = 0.0;
        for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p) mx = std::max(mx, val[p]);
        const double thr = beta * mx * (1.0 - kTie);
        double best = -1.0;
        for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p)
            if (agg[col[p]] < 0 && col[p] != i && val[p] >= thr) best = std::max(best, val[p]);
        int32_t pick = -1;
        if (best > 0.0)
            for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p)
                if (agg[col[p]] < 0 && col[p] != i && val[p] >= thr && val[p] >= best * (1.0 - kTie) &&
                    (pick < 0 || col[p] < pick))
                    pick = col[p];
        agg[i] = int32_t(nc);
        if (pick >= 0) agg[pick] = int32_t(nc);
        ++nc;
    }
    std::vector<int64_t> size(nc, 0);
    for (int64_t i = 0; i < n; ++i) ++size[agg[i]];
    for (int64_t i = 0; i < n; ++i) {
        if (size[agg[i]] != 1) continue;
        double mx = -1.0;
        for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p)
            if (col[p] != i) mx = std::max(mx, val[p]);
        if (mx < 0.0) continue;
        int32_t j = -1;
        for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p)
            if (col[p] != i && val[p] >= mx * (1.0 - kTie) && (j < 0 || col[p] < j)) j = col[p];
        --size[agg[i]];
        agg[i] = agg[j];
        ++size[agg[j]];
    }
    std::vector<int32_t> renum(nc, -1);
    int64_t m = 0;
    for (int64_t c = 0; c < nc; ++c)
        if (size[c] > 0) renum[c] = int32_t(m++);
    for (int64_t i = 0; i < n; ++i) agg[i] = renum[agg[i]];
    nc = m;
    return agg;
}

// Couplings between aggregates (sums over cell pairs in different ones).
void coarse_couplings(const HostLevel &F, const std::vector<int32_t> &agg, int64_t nc, HostLevel &C) {
    std::vector<std::map<int32_t, double>> rows(nc);
    for (int64_t i = 0; i < F.n; ++i)
        for (int64_t p = F.ptr[i]; p < F.ptr[i + 1]; ++p) {
            const int32_t a = agg[i], b = agg[F.col[p]];
            if (a != b) rows[a][b] += F.val[p];
        }
    C.n = nc;
    csr_from_maps(C, rows);
}

// Two pairwise passes: the second pairs the aggregates of the first.
HostLevel aggregate(HostLevel &F, double beta) {
    int64_t n1 = 0, n2 = 0;
    const auto a1 = pairwise(F.n, F.ptr, F.col, F.val, beta, n1);
    HostLevel M;
    coarse_couplings(F, a1, n1, M);
    const auto a2 = pairwise(M.n, M.ptr, M.col, M.val, beta, n2);
    F.agg.resize(F.n);
    for (int64_t i = 0; i < F.n; ++i) F.agg[i] = a2[a1[i]];
    F.nc = n2;
    HostLevel C;
    coarse_couplings(F, F.agg, n2, C);
    C.k = F.k;
    C.g.assign(n2, 0.0);
    C.w.assign(n2, 0.0);
    C.area.assign(n2, 0.0);
    for (int64_t i = 0; i < F.n; ++i) {
        C.g[F.agg[i]] += F.g[i];
        C.w[F.agg[i]] += F.w[i];
        C.area[F.agg[i]] += F.area[i];
    }
    return C;
}

HostLevel merge_planes(const HostLevel &F) {
    HostLevel C = F;
    C.k = F.k / 2;
    C.kind = 0;
    C.agg.clear();
    for (auto &v : C.val) v *= 2.0;
    for (auto &v : C.g) v *= 2.0;
    return C;
}

// Lower median over cells of w_i / max_j t_ij (0 for a cell without
// in-plane neighbours).
double plane_dominance(const HostLevel &L) {
    std::vector<double> ratio(L.n, 0.0);
    for (int64_t i = 0; i < L.n; ++i) {
        double mx = 0.0;
        for (int64_t p = L.ptr[i]; p < L.ptr[i + 1]; ++p) mx = std::max(mx, L.val[p]);
        ratio[i] = mx > 0.0 ? L.w[i] / mx : 0.0;
    }
    const size_t m = (ratio.size() - 1) / 2;
    std::nth_element(ratio.begin(), ratio.begin() + m, ratio.end());
    return ratio[m];
}

// Pseudo-inverse terms one cycle multiplies when a level is solved per plane
// (mode): coupled planes, floor(k/2) + 1 modes of n x n, each read once for
// its cosine and sine right-hand sides; independent planes, the one n x n
// pseudo-inverse once per pair of planes.  A level is solved that way only
// within kModeTerms (64 MiB of FP64 terms per cycle).
constexpr int64_t kModeTerms = int64_t(1) << 23;
int64_t mode_units(const HostLevel &L, bool coupled) { return coupled ? L.k / 2 + 1 : (L.k + 1) / 2; }
bool by_modes(const HostLevel &L, bool coupled, const fvx_amg_opts &o) {
    return o.mode_cells > 0 && L.n <= o.mode_cells && mode_units(L, coupled) * L.n * L.n <= kModeTerms;
}

std::vector<HostLevel> build_levels(HostLevel L0, bool coupled, const fvx_amg_opts &o) {
    std::vector<HostLevel> L;
    L.push_back(std::move(L0));
    while (true) {
        HostLevel &lev = L.back();
        if (lev.n * lev.k <= o.coarse_max || int(L.size()) >= o.max_levels) break;
        if (by_modes(lev, coupled, o)) break;
        if (coupled && lev.k >= 2 && lev.k % 2 == 0 && plane_dominance(lev) > o.z_rule) {
            lev.kind = 2;
            HostLevel nxt = merge_planes(lev);
            L.push_back(std::move(nxt));
        } else {
            HostLevel nxt = aggregate(lev, o.beta);
            if (nxt.n == lev.n) {
                lev.agg.clear();
                lev.nc = 0;
                break;
            }
            lev.kind = 1;
            L.push_back(std::move(nxt));
        }
    }
    L.back().kind = 0;
    return L;
}

// Dense operator of the coarsest level per independent system, in AoS order
// (cell i, plane l) -> i * kk + l, kk = k for coupled planes, else 1.
std::vector<double> dense_level(const HostLevel &L, bool coupled) {
    const int kk = coupled ? L.k : 1;
    const int64_t n = L.n * kk;
    std::vector<double> A(size_t(n * n), 0.0);
    for (int64_t i = 0; i < L.n; ++i)
        for (int l = 0; l < kk; ++l) {
            const int64_t q = i * kk + l;
            double dg = L.g[i];
            for (int64_t p = L.ptr[i]; p < L.ptr[i + 1]; ++p) {
                dg += L.val[p];
                A[q * n + int64_t(L.col[p]) * kk + l] -= L.val[p];
            }
            if (coupled && kk >= 2) {
                dg += 2.0 * L.w[i];
                A[q * n + i * kk + (l + 1) % kk] -= L.w[i];
                A[q * n + i * kk + (l + kk - 1) % kk] -= L.w[i];
            }
            A[q * n + q] += dg;
        }
    return A;
}

// Inverse of an SPD matrix (n <= kMaxAmgCoarse) by Cholesky factorisation
// A = L L^T, M = L^-1 row by row, A^-1 = M^T M (every inner loop runs along
// a row).
std::vector<double> spd_inverse(std::vector<double> A, int64_t n) {
    for (int64_t j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int64_t p = 0; p < j; ++p) d -= A[j * n + p] * A[j * n + p];
        FVX_REQUIRE(d > 0.0 && std::isfinite(d), FVX_E_ARG, "coarsest multigrid level is not positive definite");
        d = std::sqrt(d);
        A[j * n + j] = d;
        for (int64_t i = j + 1; i < n; ++i) {
            double s = A[i * n + j];
            for (int64_t p = 0; p < j; ++p) s -= A[i * n + p] * A[j * n + p];
            A[i * n + j] = s / d;
        }
    }
    std::vector<double> M(size_t(n * n), 0.0);
    for (int64_t i = 0; i < n; ++i) {
        double *mi = &M[i * n];
        mi[i] = 1.0;
        for (int64_t p = 0; p < i; ++p) {
            const double l = A[i * n + p];
            const double *mp = &M[p * n];
            for (int64_t c = 0; c <= p; ++c) mi[c] -= l * mp[c];
        }
        const double inv_d = 1.0 / A[i * n + i];
        for (int64_t c = 0; c <= i; ++c) mi[c] *= inv_d;
    }
    std::vector<double> inv(size_t(n * n), 0.0);
    for (int64_t k = 0; k < n; ++k) {
        const double *mk = &M[k * n];
        for (int64_t i = 0; i <= k; ++i) {
            const double a = mk[i];
            double *row = &inv[i * n];
            for (int64_t c = 0; c <= k; ++c) row[c] += a * mk[c];
        }
    }
    return inv;
}

// Pseudo-inverse of the coarsest operator: the inverse with Dirichlet walls;
// for the singular operator (null space: constants) (A + a 1 1^T)^-1 minus
// 1 1^T / (a n^2), which is A^+ exactly.
std::vector<double> coarsest_pinv(const HostLevel &L, bool coupled, bool singular) {
    std::vector<double> A = dense_level(L, coupled);
    const int64_t n = L.n * (coupled ? L.k : 1);
    double alpha = 0.0;
    if (singular) {
        double tr = 0.0;
        for (int64_t i = 0; i < n; ++i) tr += A[i * n + i];
        if (!(tr > 0.0)) return std::vector<double>(size_t(n * n), 0.0);  // one cell: A = 0, A^+ = 0
        alpha = tr / double(n) / double(n);
        for (auto &v : A) v += alpha;
    }
    std::vector<double> inv = spd_inverse(std::move(A), n);
    if (singular) {
        const double c = 1.0 / (alpha * double(n) * double(n));
        for (auto &v : inv) v -= c;
    }
    return inv;
}

// Real Fourier basis along k periodic planes, orthonormal, row j over the
// planes l: j = 0 the constant 1/sqrt(k); for mode m = (j + 1) / 2 with
// 2m < k, sqrt(2/k) cos(2 pi m l / k) for odd j and sqrt(2/k) sin(...) for
// even j; for even k, j = k - 1 the alternating (-1)^l / sqrt(k).  Every row
// of mode m is an eigenvector of the periodic second difference
// (2 x_l - x_{l-1} - x_{l+1}) with eigenvalue 2 - 2 cos(2 pi m / k), also
// for k = 2, whose two plane neighbours coincide (eigenvalues 0 and 4).
std::vector<double> fourier_basis(int k) {
    constexpr double kPi = 3.14159265358979323846;
    std::vector<double> phi(size_t(k) * k);
    const double a0 = 1.0 / std::sqrt(double(k)), a1 = std::sqrt(2.0 / double(k));
    for (int j = 0; j < k; ++j) {
        const int m = (j + 1) / 2;
        for (int l = 0; l < k; ++l) {
            const double ang = 2.0 * kPi * double((int64_t(m) * l) % k) / double(k);  // reduced: exact phase
            double v;
            if (j == 0)
                v = a0;
            else if (2 * m == k)
                v = l % 2 ? -a0 : a0;
            else
                v = a1 * (j % 2 ? std::cos(ang) : std::sin(ang));
            phi[size_t(j) * k + l] = v;
        }
    }
    return phi;
}

// Pseudo-inverses of the plane modes of the coarsest level (coupled planes,
// periodic): mode m's system is A_b + (2 - 2 cos(2 pi m / k)) diag(w) on the
// base cells, singular only for m = 0 of a singular operator.  The modes are
// formed on the host threads, each into its own [n][n] slice.
std::vector<double> mode_pinvs(const HostLevel &L, bool singular, int modes) {
    constexpr double kPi = 3.14159265358979323846;
    const size_t nn = size_t(L.n) * size_t(L.n);
    std::vector<double> out(size_t(modes) * nn);
    std::vector<std::exception_ptr> err(static_cast<size_t>(modes));
    auto one = [&](int m) {
        try {
            HostLevel M = L;
            M.k = 1;
            const double lam = 2.0 - 2.0 * std::cos(2.0 * kPi * double(m) / double(L.k));
            for (int64_t i = 0; i < L.n; ++i) M.g[i] = L.g[i] + lam * L.w[i];
            const std::vector<double> p = coarsest_pinv(M, false, singular && m == 0);
            std::copy(p.begin(), p.end(), out.begin() + ptrdiff_t(size_t(m) * nn));
        } catch (...) {
            err[size_t(m)] = std::current_exception();
        }
    };
    const int nt = std::max(1, std::min(modes, int(std::thread::hardware_concurrency())));
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t)
        pool.emplace_back([&, t] {
            for (int m = t; m < modes; m += nt) one(m);
        });
    for (auto &th : pool) th.join();
    for (auto &e : err)
        if (e) std::rethrow_exception(e);
    return out;
}

// Face graph whose finite-volume operator with plane spacing 1 is the level:
// one face per coupled pair (len = coupling, dist = 1), a wall face per cell
// with a wall term, areas = plane couplings (coupled) or cell areas.
fvx_mesh level_mesh(const HostLevel &L, bool coupled) {
    fvx_mesh m;
    m.n_cells = int(L.n);
    m.area = coupled && L.k >= 2 ? L.w : L.area;
    m.cx.assign(L.n, 0.0);
    m.cy.assign(L.n, 0.0);
    for (int64_t i = 0; i < L.n; ++i)
        for (int64_t p = L.ptr[i]; p < L.ptr[i + 1]; ++p)
            if (L.col[p] > i) {
                m.c1.push_back(int32_t(i));
                m.c2.push_back(L.col[p]);
                m.len.push_back(L.val[p]);
                m.dist.push_back(1.0);
            }
    m.n_faces = int(m.c1.size());
    for (int64_t i = 0; i < L.n; ++i)
        if (L.g[i] > 0.0) {
            m.wcell.push_back(int32_t(i));
            m.wlen.push_back(L.g[i]);
            m.wdist.push_back(1.0);
        }
    m.n_walls = int(m.wcell.size());
    return m;
}

fvx_op_desc level_desc(const fvx_op *fine, const HostLevel &L, bool dirichlet) {
    fvx_op_desc d{};
    d.k = L.k;
    d.coupling = fine->coupling;
    d.dz = 1.0;
    d.wall_bc = dirichlet ? FVX_WALL_DIRICHLET : FVX_WALL_NEUMANN;
    d.with_f32 = fine->has_f32 ? 1 : 0;
    d.stencil = 7;
    return d;
}

struct Plan {
    std::vector<HostLevel> L;
    std::vector<fvx_mesh> meshes;  // levels >= 1
    std::vector<fvx_op_desc> descs;
    std::vector<size_t> op_bytes;
    std::vector<double> pinv;
    std::vector<double> phi;  // plane modes of coupled planes: the Fourier basis of the coarsest level's planes
    size_t pinv_terms = 0, phi_terms = 0;  // their sizes (also when they are not formed)
    bool coupled = false;
    int n_d = 0;
    int modes = 0;  // coarsest per plane (mode): coupled floor(k/2) + 1 systems; independent planes 1, shared
};

void check_amg_opts(const fvx_amg_opts *o) {
    FVX_REQUIRE(o, FVX_E_ARG, "NULL multigrid options");
    FVX_REQUIRE(o->degree >= 2 && o->degree <= kMaxAmgDegree, FVX_E_ARG, "multigrid smoother degree must be 2..8");
    FVX_REQUIRE(o->ratio > 1.0 && std::isfinite(o->ratio), FVX_E_ARG, "multigrid smoother ratio must be > 1");
    FVX_REQUIRE(o->beta > 0.0 && o->beta <= 1.0, FVX_E_ARG, "aggregation beta must be in (0, 1]");
    FVX_REQUIRE(o->z_rule >= 0.0 && std::isfinite(o->z_rule), FVX_E_ARG, "z_rule must be >= 0");
    FVX_REQUIRE(o->coarse_max >= 1 && o->coarse_max <= kMaxAmgCoarse, FVX_E_ARG, "coarse_max must be 1..2048");
    FVX_REQUIRE(o->max_levels >= 1 && o->max_levels <= kMaxAmgLevels, FVX_E_ARG, "max_levels must be 1..16");
    FVX_REQUIRE(o->mode_cells >= 0 && o->mode_cells <= kMaxAmgCoarse, FVX_E_ARG, "mode_cells must be 0..2048");
}

// form: compute the coarsest pseudo-inverses (false: their sizes only, for
// fvx_amg_bytes).
Plan make_plan(const fvx_mesh *m, const fvx_op *op, const fvx_amg_opts *o, bool form) {
    FVX_REQUIRE(m && op, FVX_E_ARG, "NULL mesh or operator");
    check_amg_opts(o);
    FVX_REQUIRE(op->stencil == 7, FVX_E_UNSUPPORTED, "the multigrid needs the 7-point finite-volume operator");
    FVX_REQUIRE(int64_t(m->n_cells) == op->n_b && int64_t(m->n_faces) == op->F_b, FVX_E_ARG,
                "operator was not built from this mesh");
    const bool dirichlet = !op->singular;
    Plan P;
    P.coupled = op->zfaces;
    P.L = build_levels(fine_level(*m, op, dirichlet), P.coupled, *o);
    const HostLevel &last = P.L.back();
    // A level within coarse_max keeps the dense solve (one launch; the solve
    // per plane takes three).
    if (last.n * last.k > o->coarse_max && by_modes(last, P.coupled, *o)) {
        P.n_d = int(last.n);
        P.modes = P.coupled ? last.k / 2 + 1 : 1;
        P.pinv_terms = size_t(P.modes) * size_t(last.n) * size_t(last.n);
        P.phi_terms = P.coupled ? size_t(last.k) * size_t(last.k) : 0;
        if (form && P.coupled) {
            P.pinv = mode_pinvs(last, op->singular, P.modes);
            P.phi = fourier_basis(last.k);
        } else if (form) {
            P.pinv = coarsest_pinv(last, false, op->singular);
        }
    } else {
        const int64_t nd = last.n * (P.coupled ? last.k : 1);
        FVX_REQUIRE(nd <= kMaxAmgCoarse, FVX_E_UNSUPPORTED,
                    "coarsening stopped above 2048 unknowns (raise max_levels or coarse_max)");
        P.n_d = int(nd);
        P.pinv_terms = size_t(nd) * size_t(nd);
        if (form) P.pinv = coarsest_pinv(last, P.coupled, op->singular);
    }
    for (size_t l = 1; l < P.L.size(); ++l) {
        P.meshes.push_back(level_mesh(P.L[l], P.coupled));
        P.descs.push_back(level_desc(op, P.L[l], dirichlet));
        size_t b = 0;
        const int rc = fvx_op_bytes(&P.meshes.back(), &P.descs.back(), &b);
        FVX_REQUIRE(rc == FVX_OK, rc, "coarse level operator");
        P.op_bytes.push_back(b);
    }
    return P;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Device bytes of a plan, in the order create lays them out.
size_t plan_bytes(const Plan &P, bool f32) {
    size_t off = 0;
    for (size_t b : P.op_bytes) off += align256(b);
    for (const auto &L : P.L)
        if (L.kind == 1) off += align256(4 * size_t(L.n)) * 2 + align256(4 * size_t(L.nc + 1));
    off += align256(8 * P.pinv_terms);
    if (f32) off += align256(4 * P.pinv_terms);
    off += 2 * align256(8 * P.phi_terms);
    return off;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Restriction of the residual to the aggregates: rc[c] = sum over the
// members i of aggregate c of (r - A z)_i = r_i + (L z)_i; a.n_rows is the
// number of aggregates, the row computation is the fine level's.
template <typename T, int V, bool Z, int WT, int MW>
__global__ __launch_bounds__(kMaxCgBlock) void k_amg_restrict(RowArgs<T> a, const CgState *__restrict__ st,
                                                              const int32_t *__restrict__ mptr,
                                                              const int32_t *__restrict__ midx,
                                                              const T *__restrict__ r, const T *__restrict__ z,
                                                              T *__restrict__ rc) {
    if (st->done) return;
    const VB vb = vb_single(a.remap);
    ROW_PROLOGUE
    const bool single = lpr * V >= a.k;
    const PlainLoad<T, V> in{z, a.ld};
    FOR_ROWS {
        vec_t<T, V> sum(0);
        int32_t p = mptr[row];
        const int32_t pe = mptr[row + 1];
        // MW = 4: four (then two) members per step, one round of loads for the
        // usual aggregate of up to four cells, for the small grids of the
        // coarse levels (one block per CU or fewer: latency, not occupancy,
        // sets their time); MW = 2 elsewhere (fewer registers).  Summed in
        // member order either way.
        for (; MW == 4 && p + 4 <= pe; p += 4) {
            const int64_t i0 = midx[p], i1 = midx[p + 1], i2 = midx[p + 2], i3 = midx[p + 3];
            vec_t<T, V> z0, z1, z2, z3;
            const vec_t<T, V> a0 = lap_row_ld<T, V, Z, WT>(a.A, in, a.n_b, a.k, a.W, i0, c0, sub, lpr, single, z0);
            const vec_t<T, V> a1 = lap_row_ld<T, V, Z, WT>(a.A, in, a.n_b, a.k, a.W, i1, c0, sub, lpr, single, z1);
            const vec_t<T, V> a2 = lap_row_ld<T, V, Z, WT>(a.A, in, a.n_b, a.k, a.W, i2, c0, sub, lpr, single, z2);
            const vec_t<T, V> a3 = lap_row_ld<T, V, Z, WT>(a.A, in, a.n_b, a.k, a.W, i3, c0, sub, lpr, single, z3);
            sum += ldv<T, V>(r + i0 * a.ld + c0) + a0;
            sum += ldv<T, V>(r + i1 * a.ld + c0) + a1;
            sum += ldv<T, V>(r + i2 * a.ld + c0) + a2;
            sum += ldv<T, V>(r + i3 * a.ld + c0) + a3;
        }
        for (; p + 2 <= pe; p += 2) {
            const int64_t i0 = midx[p], i1 = midx[p + 1];
            vec_t<T, V> z0, z1;
            const vec_t<T, V> a0 = lap_row_ld<T, V, Z, WT>(a.A, in, a.n_b, a.k, a.W, i0, c0, sub, lpr, single, z0);
            const vec_t<T, V> a1 = lap_row_ld<T, V, Z, WT>(a.A, in, a.n_b, a.k, a.W, i1, c0, sub, lpr, single, z1);
            sum += ldv<T, V>(r + i0 * a.ld + c0) + a0;
            sum += ldv<T, V>(r + i1 * a.ld + c0) + a1;
        }
        if (p < pe) {
            const int64_t i = midx[p];
            vec_t<T, V> zi;
            const vec_t<T, V> acc = lap_row_ld<T, V, Z, WT>(a.A, in, a.n_b, a.k, a.W, i, c0, sub, lpr, single, zi);
            sum += ldv<T, V>(r + i * a.ld + c0) + acc;
        }
        stv_masked<T, V>(rc + row * a.ld + c0, sum, a.k - c0);
    }
    END_ROWS
}

// Restriction of the residual to merged planes: rc[i][l] = (r - A z)[i][2l]
// + (r - A z)[i][2l+1] (V = 2: each lane holds one plane pair).
template <typename T, bool Z, int WT>
__global__ __launch_bounds__(kMaxCgBlock) void k_amg_restrict_z(RowArgs<T> a, const CgState *__restrict__ st,
                                                                const T *__restrict__ r, const T *__restrict__ z,
                                                                T *__restrict__ rc, int ldc) {
    constexpr int V = 2;
    if (st->done) return;
    const VB vb = vb_single(a.remap);
    ROW_PROLOGUE
    const bool single = lpr * V >= a.k;
    FOR_ROWS {
        vec_t<T, V> zi;
        const vec_t<T, V> acc =
            lap_row_ld<T, V, Z, WT>(a.A, PlainLoad<T, V>{z, a.ld}, a.n_b, a.k, a.W, row, c0, sub, lpr, single, zi);
        const vec_t<T, V> res = ldv<T, V>(r + row * a.ld + c0) + acc;
        rc[row * ldc + c0 / 2] = res[0] + res[1];
    }
    END_ROWS
}

// z + P e on the fly: the coarse correction of the row's aggregate (KIND 1)
// or of its merged plane pair (KIND 2).
template <typename T, int V, int KIND>
struct ProlongLoad {
    const T *__restrict__ Zs;
    const T *__restrict__ E;
    const int32_t *__restrict__ agg;
    int ld, lde;
    __device__ __forceinline__ vec_t<T, V> vec(int64_t row, int c0) const {
        vec_t<T, V> v = ldv<T, V>(Zs + row * ld + c0);
        if constexpr (KIND == 1) {
            v += ldv<T, V>(E + int64_t(agg[row]) * lde + c0);
        } else {
#pragma unroll
            for (int u = 0; u < V; ++u) v[u] += E[row * lde + (c0 + u) / 2];
        }
        return v;
    }
    __device__ __forceinline__ T scalar(int64_t row, int l) const {
        return Zs[row * ld + l] + (KIND == 1 ? E[int64_t(agg[row]) * lde + l] : E[row * lde + l / 2]);
    }
};

// Prolongation fused with the first post-smoothing step: zc = zs + P e;
// q0 = zc, q1 = zc + D^-1 (r - A zc) / theta (the first Chebyshev step from
// the guess zc).
template <typename T, int V, bool Z, int WT, int KIND>
__global__ __launch_bounds__(kMaxCgBlock) void k_amg_prolong(RowArgs<T> a, const CgState *__restrict__ st,
                                                             const int32_t *__restrict__ agg,
                                                             const T *__restrict__ zs, const T *__restrict__ e,
                                                             int lde, const T *__restrict__ r, T *__restrict__ q0,
                                                             T *__restrict__ q1, T inv_theta) {
    if (st->done) return;
    const VB vb = vb_single(a.remap);
    ROW_PROLOGUE
    const bool single = lpr * V >= a.k;
    FOR_ROWS {
        const int64_t o = row * a.ld + c0;
        vec_t<T, V> zc;
        const vec_t<T, V> acc = lap_row_ld<T, V, Z, WT>(a.A, ProlongLoad<T, V, KIND>{zs, e, agg, a.ld, lde}, a.n_b,
                                                        a.k, a.W, row, c0, sub, lpr, single, zc);
        const T di = a.A.dinv[row];
        const vec_t<T, V> z1 = zc + (di * inv_theta) * (ldv<T, V>(r + o) + acc);
        stv_masked<T, V>(q0 + o, zc, a.k - c0);
        stv_masked<T, V>(q1 + o, z1, a.k - c0);
    }
    END_ROWS
}

template <typename T, int V, bool Z, int WT, int MODE, bool LAST>
__global__ __launch_bounds__(kMaxCgBlock) void k_amg_cheb(RowArgs<T> a, CgDev d, const T *__restrict__ r,
                                                          const T *__restrict__ zin, T *__restrict__ zio, T c1, T c2,
                                                          T inv_theta) {
    b_cheb<T, V, Z, WT, MODE, LAST>(a, d, vb_single(a.remap), r, zin, zio, c1, c2, inv_theta);
}

// Coarsest level: z = A^+ r with the dense pseudo-inverse.  Coupled planes
// (one system of n_b * k unknowns, system index i * k + l): one block per
// output, each thread taking every 256th term of the row, all its loads in
// flight at once (the row has at most kMaxAmgCoarse terms), then a block
// reduction.  Independent planes (every plane uses the same [n_b][n_b]
// matrix): one wavefront per output (cell i, plane l).
constexpr int kDenseBlock = 256;
constexpr int kCoarseGridBlocks = 256;  // MI355X compute units

template <typename T>
__global__ __launch_bounds__(kDenseBlock) void k_amg_dense(const CgState *__restrict__ st, const T *__restrict__ pinv,
                                                           int n_b, int k, int ld, int coupled,
                                                           const T *__restrict__ r, T *__restrict__ z) {
    if (st->done) return;
    if (coupled) {
        __shared__ double part[kDenseBlock / 64];
        const int nd = n_b * k;
        const int out = int(blockIdx.x);
        const T *row = pinv + int64_t(out) * nd;
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < kMaxAmgCoarse / kDenseBlock; ++u) {
            const int p = int(threadIdx.x) + u * kDenseBlock;
            if (p < nd) {
                const int j = p / k;
                s += double(row[p]) * double(r[int64_t(j) * ld + (p - j * k)]);
            }
        }
        s = wave_sum(s);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < kDenseBlock / 64; ++w) t += part[w];
            const int i = out / k;
            z[int64_t(i) * ld + (out - i * k)] = T(t);
        }
        return;
    }
    const int lane = threadIdx.x & 63;
    const int64_t out = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    if (out >= int64_t(n_b) * k) return;  // uniform over the wavefront
    const int64_t i = out / k;
    const int l = int(out % k);
    const T *row = pinv + i * n_b;
    double s = 0.0;
    for (int64_t j = lane; j < n_b; j += 64) s += double(row[j]) * double(r[j * ld + l]);
    s = wave_sum(s);
    if (lane == 0) z[i * ld + l] = T(s);
}

// Coarsest level per plane mode.  The level's vectors are [n_b][ld] (cell,
// plane); the mode vectors are [k][n_b] (basis function, cell), one
// contiguous right-hand side per basis function.  Independent planes take
// the identity for the basis (phi, phi_t NULL: the transforms transpose).
// Forward transform mr[j][i] = sum_l phi[j][l] r[i][l]: one thread per
// (cell, basis function), the lanes of a cell reading the transposed table
// along its rows and the cell's planes by broadcast.
template <typename T>
__global__ __launch_bounds__(kDenseBlock) void k_amg_modes_fwd(const CgState *__restrict__ st,
                                                               const double *__restrict__ phi_t, int n_b, int k,
                                                               int ld, const T *__restrict__ r,
                                                               double *__restrict__ mr) {
    if (st->done) return;
    const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= int64_t(n_b) * k) return;
    const int64_t i = o / k;
    const int j = int(o - i * k);
    const T *ri = r + i * ld;
    double s = 0.0;
    if (phi_t) {
#pragma unroll 8
        for (int l = 0; l < k; ++l) s += phi_t[int64_t(l) * k + j] * double(ri[l]);
    } else {
        s = double(ri[j]);
    }
    mr[int64_t(j) * n_b + i] = s;
}

// The same transforms for at most kModeLdsK coupled planes with the basis
// (32 KiB at 64 planes) and the block's cells staged in LDS: one round of
// global loads per block, then the sums from LDS in the same order as above
// (the same results bit for bit).  A block takes kDenseBlock / k cells.
constexpr int kModeLdsK = 64;

template <typename T>
__global__ __launch_bounds__(kDenseBlock) void k_amg_modes_fwd_lds(const CgState *__restrict__ st,
                                                                   const double *__restrict__ phi_t, int n_b, int k,
                                                                   int ld, const T *__restrict__ r,
                                                                   double *__restrict__ mr) {
    if (st->done) return;
    __shared__ double sphi[kModeLdsK * kModeLdsK];
    __shared__ double sx[kDenseBlock];
    const int t = int(threadIdx.x), cpb = kDenseBlock / k;
    const int64_t c0 = int64_t(blockIdx.x) * cpb;
#pragma unroll 16
    for (int u = t; u < k * k; u += kDenseBlock) sphi[u] = phi_t[u];
    const int cc = t / k, q = t - cc * k;  // the block's cell, and the plane it loads / basis function it sums
    const bool live = cc < cpb && c0 + cc < n_b;
    if (live) sx[t] = double(r[(c0 + cc) * ld + q]);
    __syncthreads();
    if (!live) return;
    const double *xc = sx + cc * k;
    double s = 0.0;
    for (int l = 0; l < k; ++l) s += sphi[l * k + q] * xc[l];
    mr[int64_t(q) * n_b + c0 + cc] = s;
}

template <typename T>
__global__ __launch_bounds__(kDenseBlock) void k_amg_modes_inv_lds(const CgState *__restrict__ st,
                                                                   const double *__restrict__ phi, int n_b, int k,
                                                                   int ld, const double *__restrict__ mz,
                                                                   T *__restrict__ z) {
    if (st->done) return;
    __shared__ double sphi[kModeLdsK * kModeLdsK];
    __shared__ double sx[kDenseBlock];
    const int t = int(threadIdx.x), cpb = kDenseBlock / k;
    const int64_t c0 = int64_t(blockIdx.x) * cpb;
#pragma unroll 16
    for (int u = t; u < k * k; u += kDenseBlock) sphi[u] = phi[u];
    for (int u = t; u < cpb * k; u += kDenseBlock) {  // mz[j][c0 + cc] into sx[cc][j], consecutive cells per thread run
        const int j = u / cpb, cc = u - j * cpb;
        if (c0 + cc < n_b) sx[cc * k + j] = mz[int64_t(j) * n_b + c0 + cc];
    }
    __syncthreads();
    const int cc = t / k, q = t - cc * k;  // the block's cell and the plane it writes
    if (cc >= cpb || c0 + cc >= n_b) return;
    const double *mc = sx + cc * k;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += sphi[j * k + q] * mc[j];
    z[(c0 + cc) * ld + q] = T(s);
}

// Mode solves: rows i of a pseudo-inverse times two right-hand sides.
// PAIR (n_b even, so every row and right-hand side starts 16-byte aligned in
// FP64): each lane takes two neighbouring terms per load.
// Coupled planes, unit u = mode m: mode m's pseudo-inverse, basis functions
// 2m - 1 (cosine) and 2m (sine; mode 0 has basis function 0 alone, mode k/2
// of even k basis function k - 1 alone).  Independent planes (shared), unit
// u: the one pseudo-inverse, planes 2u and 2u + 1 (< k).  One wavefront per
// unit and pair of rows (2p, 2p + 1), 8 terms of each row per lane in
// flight, the right-hand sides read once for both rows and each row once for
// both right-hand sides.
template <typename T, bool PAIR>
__global__ __launch_bounds__(kDenseBlock) void k_amg_modes_solve(const CgState *__restrict__ st,
                                                                 const T *__restrict__ pinv, int n_b, int k,
                                                                 int units, int shared,
                                                                 const double *__restrict__ mr,
                                                                 double *__restrict__ mz) {
    if (st->done) return;
    const int lane = threadIdx.x & 63;
    const int64_t pair = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t pairs = (n_b + 1) / 2;
    if (pair >= int64_t(units) * pairs) return;  // uniform over the wavefront
    const int u = int(pair / pairs);
    const int64_t i = 2 * (pair - int64_t(u) * pairs);
    const bool two = i + 1 < n_b;
    const int m = shared ? 0 : u;
    const int jc = shared ? 2 * u : (m == 0 ? 0 : 2 * m - 1);
    const bool has_s = shared ? 2 * u + 1 < k : (m > 0 && 2 * m < k);
    const int js = has_s ? jc + 1 : jc;
    const T *p0 = pinv + (int64_t(m) * n_b + i) * n_b;
    const T *p1 = two ? p0 + n_b : p0;
    const double *rc = mr + int64_t(jc) * n_b, *rs = mr + int64_t(js) * n_b;
    double c0 = 0.0, s0 = 0.0, c1 = 0.0, s1 = 0.0;
    if constexpr (PAIR) {
        using t2 = vec_t<T, 2>;
        using d2 = vec_t<double, 2>;
        const int h = n_b / 2;
        for (int t0 = lane; t0 < h; t0 += 64 * 4) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int t = t0 + 64 * v;
                if (t < h) {
                    const t2 a = reinterpret_cast<const t2 *>(p0)[t], b = reinterpret_cast<const t2 *>(p1)[t];
                    const d2 x = reinterpret_cast<const d2 *>(rc)[t], y = reinterpret_cast<const d2 *>(rs)[t];
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        c0 += double(a[e]) * x[e];
                        s0 += double(a[e]) * y[e];
                        c1 += double(b[e]) * x[e];
                        s1 += double(b[e]) * y[e];
                    }
                }
            }
        }
    } else {
        for (int t0 = lane; t0 < n_b; t0 += 64 * 8) {
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const int t = t0 + 64 * v;
                if (t < n_b) {
                    const double a = double(p0[t]), b = double(p1[t]), x = rc[t], y = rs[t];
                    c0 += a * x;
                    s0 += a * y;
                    c1 += b * x;
                    s1 += b * y;
                }
            }
        }
    }
    c0 = wave_sum(c0);
    s0 = wave_sum(s0);
    c1 = wave_sum(c1);
    s1 = wave_sum(s1);
    if (lane == 0) {
        mz[int64_t(jc) * n_b + i] = c0;
        if (has_s) mz[int64_t(js) * n_b + i] = s0;
        if (two) {
            mz[int64_t(jc) * n_b + i + 1] = c1;
            if (has_s) mz[int64_t(js) * n_b + i + 1] = s1;
        }
    }
}

// Back transform z[i][l] = sum_j phi[j][l] mz[j][i]: one thread per (cell,
// plane), the lanes reading the table along its rows.
template <typename T>
__global__ __launch_bounds__(kDenseBlock) void k_amg_modes_inv(const CgState *__restrict__ st,
                                                               const double *__restrict__ phi, int n_b, int k, int ld,
                                                               const double *__restrict__ mz, T *__restrict__ z) {
    if (st->done) return;
    const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= int64_t(n_b) * k) return;
    const int64_t i = o / k;
    const int l = int(o - i * k);
    double s = 0.0;
    if (phi) {
#pragma unroll 8
        for (int j = 0; j < k; ++j) s += phi[int64_t(j) * k + l] * mz[int64_t(j) * n_b + i];
    } else {
        s = mz[int64_t(l) * n_b + i];
    }
    z[i * ld + l] = T(s);
}

// r.z partials into the r.z slot of part_b (a one-level hierarchy inside a
// solve: the dense solve has no smoothing step to write them).
template <typename T, int V>
__global__ __launch_bounds__(kMaxCgBlock) void k_amg_rz(RowArgs<T> a, CgDev d, const T *__restrict__ r,
                                                        const T *__restrict__ z) {
    if (d.st->done) return;
    __shared__ double lds[kMaxPercolBlock * kMaxV];
    const VB vb = vb_single(a.remap);
    ROW_PROLOGUE
    double c[1][V] = {};
    FOR_ROWS {
        const vec_t<T, V> rv = ldv<T, V>(r + row * a.ld + c0), zv = ldv<T, V>(z + row * a.ld + c0);
#pragma unroll
        for (int u = 0; u < V; ++u)
            if (c0 + u < a.k) c[0][u] += double(rv[u]) * double(zv[u]);
    }
    END_ROWS
    write_partials<1, V>(c, sub, lpr, d.G, d.percol, d.part_b + 2 * int64_t(vb.nblk) * d.G, blk, vb.nblk, lds);
}

__global__ void k_amg_clear_state(CgState *st) {
    if (threadIdx.x == 0) {
        st->done = 0;
        st->status = 0;
    }
}

// ---------------------------------------------------------------------------
// V-cycle driver
// ---------------------------------------------------------------------------

// Launch tile of a level's kernels over n_rows rows: 2 elements per lane
// when the row stride allows; 4 in FP32 over at least 2^18 elements (16-byte
// lanes where the launch streams; on smaller launches, which wait on
// latency, the wider lanes left too few threads and were slower), not on a
// level whose planes are merged (its restriction takes one plane pair per
// lane); enough lanes per row to cover k in one pass (at most 64), 256
// threads, XCD-aware order, one row tile per workgroup.
fvx_tile level_tile(const fvx_op *op, int64_t n_rows, size_t es, bool merge) {
    fvx_tile t{};
    const bool wide = es == 4 && !merge && op->ld % 4 == 0 && n_rows * op->ld >= (int64_t(1) << 18);
    t.vec = wide ? 4 : (op->ld % 2 == 0 ? 2 : 1);
    t.lanes_per_row = std::min(64, next_pow2(int(ceil_div(op->k, t.vec))));
    t.block = 256;
    t.xcd_remap = 1;
    t.max_blocks = 0;
    return t;
}

template <typename T>
struct LevelLaunch {
    RowArgs<T> a;
    dim3 grid, block;
    int vec;
};

template <typename T>
LevelLaunch<T> level_launch(const fvx_op *op, int64_t n_rows, bool merge) {
    LevelLaunch<T> L;
    const fvx_tile t = level_tile(op, n_rows, sizeof(T), merge);
    RowGrid g;
    L.a = row_args<T>(op, n_rows, g, t);
    L.grid = dim3(unsigned(g.n_blocks));
    L.block = dim3(unsigned(t.block));
    L.vec = t.vec;
    return L;
}

template <typename T, typename F>
void by_v_only(int vec, F &&f) {
    by_vec<T>(vec, false, [&](auto Vt, auto) { f(Vt); });
}

template <typename T>
const T *pinv_of(const fvx_amg *h);
template <>
const double *pinv_of<double>(const fvx_amg *h) { return h->pinv64; }
template <>
const float *pinv_of<float>(const fvx_amg *h) { return h->pinv32; }

// Chebyshev step j (1 <= j < degree) on one level, buffers as in the CG:
// gathers z_j from zin, writes z_{j+1} over z_{j-1} in zio.  mode 0: z_j =
// z_1 from r; 1: z_{j-1} = z_1 from r; 2: z_{j-1} read from zio.
template <typename T>
void cheb_step(const RowArgs<T> &a, dim3 grid, dim3 block, int vec, const fvx_op *op, const CgDev &d, int mode,
               bool last, const T *r, const T *zin, T *zio, const fvx_amg *h, int j, hipStream_t s) {
    const T c1 = T(h->c1[j]), c2 = T(h->c2[j]), ith = T(h->inv_theta);
    by_vec<T>(vec, op->zfaces, [&](auto Vt, auto Zt) {
        constexpr int V = decltype(Vt)::value;
        constexpr bool Z = decltype(Zt)::value;
        by_width(op->W, [&](auto Wt) {
            constexpr int WT = decltype(Wt)::value;
            auto go = [&](auto Mt, auto Lt) {
                hipLaunchKernelGGL((k_amg_cheb<T, V, Z, WT, decltype(Mt)::value, decltype(Lt)::value>), grid, block,
                                   0, s, a, d, r, zin, zio, c1, c2, ith);
            };
            auto with_last = [&](auto Mt) {
                if (last)
                    go(Mt, std::true_type{});
                else
                    go(Mt, std::false_type{});
            };
            if (mode == 0)
                with_last(std::integral_constant<int, 0>{});
            else if (mode == 1)
                with_last(std::integral_constant<int, 1>{});
            else
                with_last(std::integral_constant<int, 2>{});
        });
    });
}

}  // namespace

namespace {
template <typename T>
AmgWork<T> carve_work(const fvx_amg *h, char *base, size_t *bytes) {
    AmgWork<T> w;
    size_t off = 0;
    auto take = [&](size_t b) {
        char *p = base ? base + off : nullptr;
        off += align256(b);
        return p;
    };
    w.st = reinterpret_cast<CgState *>(take(sizeof(CgState)));
    const int nl = int(h->lv.size());
    for (int l = 0; l < nl; ++l) {
        const fvx_op *op = h->lv[l].op;
        const size_t nv = sizeof(T) * size_t(op->n_b) * op->ld;
        auto &v = w.lv[l];
        if (l > 0) v.r = reinterpret_cast<T *>(take(nv));
        if (l + 1 < nl) {
            v.s[0] = reinterpret_cast<T *>(take(nv));
            v.s[1] = reinterpret_cast<T *>(take(nv));
            v.q[0] = reinterpret_cast<T *>(take(nv));
            v.q[1] = reinterpret_cast<T *>(take(nv));
        } else {
            v.q[0] = reinterpret_cast<T *>(take(nv));
        }
    }
    if (h->modes) {
        const fvx_op *op = h->lv[nl - 1].op;
        const size_t nm = 8 * size_t(op->n_b) * op->k;
        w.mr = reinterpret_cast<double *>(take(nm));
        w.mz = reinterpret_cast<double *>(take(nm));
    }
    if (bytes) *bytes = off;
    return w;
}
}  // namespace

size_t amg_work_bytes(const fvx_amg *h, int dtype) {
    size_t b = 0;
    if (dtype == FVX_F32)
        carve_work<float>(h, nullptr, &b);
    else
        carve_work<double>(h, nullptr, &b);
    return b;
}

template <typename T>
AmgWork<T> amg_carve(const fvx_amg *h, char *base) {
    return carve_work<T>(h, base, nullptr);
}
template AmgWork<double> amg_carve<double>(const fvx_amg *, char *);
template AmgWork<float> amg_carve<float>(const fvx_amg *, char *);

// z_degree of the post-smoother sits in q[(degree - 2) & 1] (q[0] on the
// coarsest level).
template <typename T>
T *amg_output(const fvx_amg *h, const AmgWork<T> &w) {
    return h->lv.size() == 1 ? w.lv[0].q[0] : w.lv[0].q[(h->o.degree - 2) & 1];
}
template double *amg_output<double>(const fvx_amg *, const AmgWork<double> &);
template float *amg_output<float>(const fvx_amg *, const AmgWork<float> &);

template <typename T>
void amg_vcycle(const fvx_amg *h, const T *r0, const AmgWork<T> &w, const CgDev &d, const AmgFinal<T> *fin,
                hipStream_t s) {
    const int nl = int(h->lv.size());
    const int deg = h->o.degree;
    CgDev dn{};
    dn.st = d.st;  // the "done" flag only; partials are written by the final step alone
    auto rhs = [&](int l) { return l == 0 ? r0 : static_cast<const T *>(w.lv[l].r); };
    // Down: pre-smooth, restrict.
    for (int l = 0; l + 1 < nl; ++l) {
        const fvx_op *op = h->lv[l].op;
        const LevelLaunch<T> L = level_launch<T>(op, op->n_b, h->lv[l].kind == 2);
        const T *r = rhs(l);
        const auto &v = w.lv[l];
        for (int j = 1; j < deg; ++j)
            cheb_step<T>(L.a, L.grid, L.block, L.vec, op, dn, j == 1 ? 0 : (j == 2 ? 1 : 2), false, r, v.s[j & 1],
                         v.s[(j - 1) & 1], h, j, s);
        const T *zs = v.s[(deg - 2) & 1];
        const fvx_op *nop = h->lv[l + 1].op;
        if (h->lv[l].kind == 1) {
            const LevelLaunch<T> R = level_launch<T>(op, nop->n_b, false);
            by_vec<T>(R.vec, op->zfaces, [&](auto Vt, auto Zt) {
                constexpr int V = decltype(Vt)::value;
                constexpr bool Z = decltype(Zt)::value;
                by_width(op->W, [&](auto Wt) {
                    constexpr int WT = decltype(Wt)::value;
                    // a grid of at most one block per CU is latency-bound: take
                    // four members per step (not at width 8, where it spills)
                    if (WT != 8 && int(R.grid.x) <= kCoarseGridBlocks)
                        hipLaunchKernelGGL((k_amg_restrict<T, V, Z, WT, WT == 8 ? 2 : 4>), R.grid, R.block, 0, s,
                                           R.a, d.st, h->lv[l].mem_ptr, h->lv[l].mem_idx, r, zs, w.lv[l + 1].r);
                    else
                        hipLaunchKernelGGL((k_amg_restrict<T, V, Z, WT, 2>), R.grid, R.block, 0, s, R.a, d.st,
                                           h->lv[l].mem_ptr, h->lv[l].mem_idx, r, zs, w.lv[l + 1].r);
                });
            });
        } else {
            FVX_REQUIRE(L.vec == 2, FVX_E_ARG, "plane merging needs an even row stride");
            by_width(op->W, [&](auto Wt) {
                constexpr int WT = decltype(Wt)::value;
                hipLaunchKernelGGL((k_amg_restrict_z<T, true, WT>), L.grid, L.block, 0, s, L.a, d.st, r, zs,
                                   w.lv[l + 1].r, nop->ld);
            });
        }
        FVX_HIP(hipGetLastError());
    }
    // Coarsest: dense pseudo-inverse, or per plane mode.
    {
        const fvx_op *op = h->lv[nl - 1].op;
        const int64_t outs = op->n_b * int64_t(op->k);
        if (h->modes) {
            const dim3 tgrid(unsigned(ceil_div(outs, kDenseBlock)));
            const int units = h->coupled ? h->modes : (op->k + 1) / 2;
            const dim3 sgrid(unsigned(ceil_div(int64_t(units) * ((op->n_b + 1) / 2), kDenseBlock / 64)));
            const bool lds = h->phi && op->k <= kModeLdsK;
            const dim3 lgrid(lds ? unsigned(ceil_div(op->n_b, kDenseBlock / op->k)) : 1u);
            if (lds)
                hipLaunchKernelGGL(k_amg_modes_fwd_lds<T>, lgrid, dim3(kDenseBlock), 0, s, d.st, h->phi_t,
                                   int(op->n_b), op->k, op->ld, rhs(nl - 1), w.mr);
            else
                hipLaunchKernelGGL(k_amg_modes_fwd<T>, tgrid, dim3(kDenseBlock), 0, s, d.st, h->phi_t,
                                   int(op->n_b), op->k, op->ld, rhs(nl - 1), w.mr);
            if (op->n_b % 2 == 0)
                hipLaunchKernelGGL((k_amg_modes_solve<T, true>), sgrid, dim3(kDenseBlock), 0, s, d.st, pinv_of<T>(h),
                                   int(op->n_b), op->k, units, int(!h->coupled), static_cast<const double *>(w.mr),
                                   w.mz);
            else
                hipLaunchKernelGGL((k_amg_modes_solve<T, false>), sgrid, dim3(kDenseBlock), 0, s, d.st,
                                   pinv_of<T>(h), int(op->n_b), op->k, units, int(!h->coupled),
                                   static_cast<const double *>(w.mr), w.mz);
            if (lds)
                hipLaunchKernelGGL(k_amg_modes_inv_lds<T>, lgrid, dim3(kDenseBlock), 0, s, d.st, h->phi,
                                   int(op->n_b), op->k, op->ld, static_cast<const double *>(w.mz), w.lv[nl - 1].q[0]);
            else
                hipLaunchKernelGGL(k_amg_modes_inv<T>, tgrid, dim3(kDenseBlock), 0, s, d.st, h->phi,
                                   int(op->n_b), op->k, op->ld, static_cast<const double *>(w.mz), w.lv[nl - 1].q[0]);
        } else {
            const unsigned dense_grid = unsigned(h->coupled ? outs : ceil_div(outs, kDenseBlock / 64));
            hipLaunchKernelGGL(k_amg_dense<T>, dim3(dense_grid), dim3(kDenseBlock), 0, s, d.st, pinv_of<T>(h),
                               int(op->n_b), op->k, op->ld, int(h->coupled), rhs(nl - 1), w.lv[nl - 1].q[0]);
        }
        FVX_HIP(hipGetLastError());
        if (nl == 1 && fin) {
            by_v_only<T>(fin->vec, [&](auto Vt) {
                constexpr int V = decltype(Vt)::value;
                hipLaunchKernelGGL((k_amg_rz<T, V>), fin->grid, fin->block, 0, s, fin->a, d, r0, w.lv[0].q[0]);
            });
            FVX_HIP(hipGetLastError());
        }
    }
    // Up: prolongate + first post step, remaining post steps.
    for (int l = nl - 2; l >= 0; --l) {
        const fvx_op *op = h->lv[l].op;
        const LevelLaunch<T> L = level_launch<T>(op, op->n_b, h->lv[l].kind == 2);
        const T *r = rhs(l);
        const auto &v = w.lv[l];
        const fvx_op *nop = h->lv[l + 1].op;
        const T *e = l + 2 == nl ? w.lv[l + 1].q[0] : w.lv[l + 1].q[(deg - 2) & 1];
        const T *zs = v.s[(deg - 2) & 1];
        by_vec<T>(L.vec, op->zfaces, [&](auto Vt, auto Zt) {
            constexpr int V = decltype(Vt)::value;
            constexpr bool Z = decltype(Zt)::value;
            by_width(op->W, [&](auto Wt) {
                constexpr int WT = decltype(Wt)::value;
                if (h->lv[l].kind == 1)
                    hipLaunchKernelGGL((k_amg_prolong<T, V, Z, WT, 1>), L.grid, L.block, 0, s, L.a, d.st,
                                       h->lv[l].agg_dev, zs, e, nop->ld, r, v.q[0], v.q[1], T(h->inv_theta));
                else
                    hipLaunchKernelGGL((k_amg_prolong<T, V, Z, WT, 2>), L.grid, L.block, 0, s, L.a, d.st,
                                       h->lv[l].agg_dev, zs, e, nop->ld, r, v.q[0], v.q[1], T(h->inv_theta));
            });
        });
        for (int j = 1; j < deg; ++j) {
            const bool last = l == 0 && j == deg - 1 && fin;
            if (last)
                cheb_step<T>(fin->a, fin->grid, fin->block, fin->vec, op, d, 2, true, r, v.q[j & 1],
                             v.q[(j - 1) & 1], h, j, s);
            else
                cheb_step<T>(L.a, L.grid, L.block, L.vec, op, dn, 2, false, r, v.q[j & 1], v.q[(j - 1) & 1], h, j,
                             s);
        }
        FVX_HIP(hipGetLastError());
    }
}

template void amg_vcycle<double>(const fvx_amg *, const double *, const AmgWork<double> &, const CgDev &,
                                  const AmgFinal<double> *, hipStream_t);
template void amg_vcycle<float>(const fvx_amg *, const float *, const AmgWork<float> &, const CgDev &,
                                 const AmgFinal<float> *, hipStream_t);

void amg_check_solve(const fvx_amg *h, const fvx_op *op, bool mixed) {
    FVX_REQUIRE(h, FVX_E_ARG, "AMG preconditioner without a hierarchy (opts.amg is NULL)");
    FVX_REQUIRE(h->lv[0].op == op, FVX_E_ARG, "the multigrid hierarchy was built for another operator");
    FVX_REQUIRE(!mixed || op->has_f32, FVX_E_ARG, "mixed precision needs FP32 copies");
}

}  // namespace fvx

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using fvx::guard;

extern "C" {

int fvx_amg_opts_default(fvx_amg_opts *o) {
    if (!o) return FVX_E_ARG;
    o->degree = 2;
    o->ratio = 8.0;
    o->beta = 0.75;
    o->z_rule = 1.0;
    o->coarse_max = 2048;
    o->max_levels = 16;
    o->mode_cells = 2048;
    return FVX_OK;
}

int fvx_amg_bytes(const fvx_mesh *m, const fvx_op *op, const fvx_amg_opts *o, size_t *bytes) {
    return guard([&] {
        FVX_REQUIRE(bytes, FVX_E_ARG, "NULL bytes");
        const fvx::Plan P = fvx::make_plan(m, op, o, false);
        *bytes = fvx::plan_bytes(P, op->has_f32);
        return FVX_OK;
    });
}

int fvx_amg_create(const fvx_mesh *m, const fvx_op *op, const fvx_amg_opts *o, void *dev_mem, size_t bytes,
                   void *stream, fvx_amg **out) {
    return guard([&] {
        FVX_REQUIRE(out && dev_mem, FVX_E_ARG, "NULL output or device buffer");
        FVX_REQUIRE(reinterpret_cast<uintptr_t>(dev_mem) % 256 == 0, FVX_E_ARG,
                    "device buffer must be 256-byte aligned");
        const fvx::Plan P = fvx::make_plan(m, op, o, true);
        FVX_REQUIRE(P.pinv.size() == P.pinv_terms && P.phi.size() == P.phi_terms, FVX_E_ARG,
                    "coarsest solve sizes disagree with the plan");
        const bool f32 = op->has_f32;
        const size_t need = fvx::plan_bytes(P, f32);
        FVX_REQUIRE(bytes >= need, FVX_E_NOMEM, "multigrid buffer too small: need " + std::to_string(need));
        hipStream_t s = fvx::as_stream(stream);
        char *base = static_cast<char *>(dev_mem);
        size_t off = 0;
        auto take = [&](size_t b) {
            char *p = base + off;
            off += fvx::align256(b);
            return p;
        };
        auto h = std::make_unique<fvx_amg>();
        h->o = *o;
        h->coupled = P.coupled;
        h->n_d = P.n_d;
        h->modes = P.modes;
        const size_t nl = P.L.size();
        h->lv.resize(nl);
        h->lv[0].op = op;
        for (size_t l = 1; l < nl; ++l) {
            fvx_op *lop = nullptr;
            char *mem = take(P.op_bytes[l - 1]);
            const int rc = fvx_op_create(&P.meshes[l - 1], &P.descs[l - 1], mem, P.op_bytes[l - 1], stream, &lop);
            FVX_REQUIRE(rc == FVX_OK, rc, std::string("coarse level operator: ") + fvx_last_error());
            h->lv[l].own.reset(lop);
            h->lv[l].op = lop;
        }
        std::vector<std::vector<int32_t>> keep;
        for (size_t l = 0; l < nl; ++l) {
            const fvx::HostLevel &L = P.L[l];
            auto &lv = h->lv[l];
            lv.kind = L.kind;
            if (L.kind != 1) continue;
            lv.agg = L.agg;
            std::vector<int32_t> mptr(L.nc + 1, 0), midx(L.n);
            for (int64_t i = 0; i < L.n; ++i) ++mptr[L.agg[i] + 1];
            for (int64_t c = 0; c < L.nc; ++c) mptr[c + 1] += mptr[c];
            std::vector<int32_t> fill(mptr.begin(), mptr.end() - 1);
            for (int64_t i = 0; i < L.n; ++i) midx[fill[L.agg[i]]++] = int32_t(i);  // ascending within each
            char *pa = take(4 * size_t(L.n));
            char *pp = take(4 * size_t(L.nc + 1));
            char *pi = take(4 * size_t(L.n));
            FVX_HIP(hipMemcpyAsync(pa, lv.agg.data(), 4 * size_t(L.n), hipMemcpyHostToDevice, s));
            FVX_HIP(hipMemcpyAsync(pp, mptr.data(), 4 * mptr.size(), hipMemcpyHostToDevice, s));
            FVX_HIP(hipMemcpyAsync(pi, midx.data(), 4 * midx.size(), hipMemcpyHostToDevice, s));
            lv.agg_dev = reinterpret_cast<const int32_t *>(pa);
            lv.mem_ptr = reinterpret_cast<const int32_t *>(pp);
            lv.mem_idx = reinterpret_cast<const int32_t *>(pi);
            keep.push_back(std::move(mptr));
            keep.push_back(std::move(midx));
        }
        const size_t nd2 = P.pinv.size();
        char *p64 = take(8 * nd2);
        FVX_HIP(hipMemcpyAsync(p64, P.pinv.data(), 8 * nd2, hipMemcpyHostToDevice, s));
        h->pinv64 = reinterpret_cast<const double *>(p64);
        std::vector<float> p32;
        if (f32) {
            p32.assign(P.pinv.begin(), P.pinv.end());
            char *q = take(4 * nd2);
            FVX_HIP(hipMemcpyAsync(q, p32.data(), 4 * nd2, hipMemcpyHostToDevice, s));
            h->pinv32 = reinterpret_cast<const float *>(q);
        }
        std::vector<double> phi_t;
        if (!P.phi.empty()) {
            const int kc = P.L.back().k;
            phi_t.resize(P.phi.size());
            for (int j = 0; j < kc; ++j)
                for (int l = 0; l < kc; ++l) phi_t[size_t(l) * kc + j] = P.phi[size_t(j) * kc + l];
            char *a = take(8 * P.phi.size());
            char *b = take(8 * phi_t.size());
            FVX_HIP(hipMemcpyAsync(a, P.phi.data(), 8 * P.phi.size(), hipMemcpyHostToDevice, s));
            FVX_HIP(hipMemcpyAsync(b, phi_t.data(), 8 * phi_t.size(), hipMemcpyHostToDevice, s));
            h->phi = reinterpret_cast<const double *>(a);
            h->phi_t = reinterpret_cast<const double *>(b);
        }
        // Smoother coefficients on [2 / ratio, 2] (Saad, Algorithm 12.1).
        const double b = 2.0, a = b / o->ratio;
        const double theta = 0.5 * (b + a), delta = 0.5 * (b - a), sigma = theta / delta;
        h->inv_theta = 1.0 / theta;
        double rho = 1.0 / sigma;
        for (int j = 1; j < o->degree; ++j) {
            const double rn = 1.0 / (2.0 * sigma - rho);
            h->c1[j] = rn * rho;
            h->c2[j] = 2.0 * rn / delta;
            rho = rn;
        }
        FVX_HIP(hipStreamSynchronize(s));
        *out = h.release();
        return FVX_OK;
    });
}

int fvx_amg_destroy(fvx_amg *h) {
    delete h;
    return FVX_OK;
}

int fvx_amg_n_levels(const fvx_amg *h, int32_t *n) {
    return guard([&] {
        FVX_REQUIRE(h && n, FVX_E_ARG, "NULL argument");
        *n = int32_t(h->lv.size());
        return FVX_OK;
    });
}

int fvx_amg_level(const fvx_amg *h, int32_t level, int64_t *n_b, int32_t *k, int64_t *nnz_b, int32_t *kind,
                  const fvx_op **op) {
    return guard([&] {
        FVX_REQUIRE(h && level >= 0 && level < int32_t(h->lv.size()), FVX_E_ARG, "bad level");
        const auto &lv = h->lv[level];
        if (n_b) *n_b = lv.op->n_b;
        if (k) *k = lv.op->k;
        if (nnz_b) *nnz_b = lv.op->nnz_b;
        if (kind) *kind = lv.kind;
        if (op) *op = lv.op;
        return FVX_OK;
    });
}

int fvx_amg_aggregates(const fvx_amg *h, int32_t level, int32_t *agg) {
    return guard([&] {
        FVX_REQUIRE(h && agg && level >= 0 && level < int32_t(h->lv.size()), FVX_E_ARG, "bad argument");
        FVX_REQUIRE(h->lv[level].kind == 1, FVX_E_ARG, "level is not coarsened by aggregation");
        std::copy(h->lv[level].agg.begin(), h->lv[level].agg.end(), agg);
        return FVX_OK;
    });
}

int fvx_amg_coarsest_modes(const fvx_amg *h, int32_t *modes) {
    return guard([&] {
        FVX_REQUIRE(h && modes, FVX_E_ARG, "NULL argument");
        *modes = int32_t(h->modes);
        return FVX_OK;
    });
}

int fvx_amg_apply_bytes(const fvx_amg *h, int dtype, size_t *bytes) {
    return guard([&] {
        FVX_REQUIRE(h && bytes && (dtype == FVX_F64 || dtype == FVX_F32), FVX_E_ARG, "bad argument");
        *bytes = fvx::amg_work_bytes(h, dtype);
        return FVX_OK;
    });
}

int fvx_amg_apply(const fvx_amg *h, int dtype, const void *R, void *Z, void *ws, size_t ws_bytes, void *stream) {
    return guard([&] {
        FVX_REQUIRE(h && R && Z && ws, FVX_E_ARG, "NULL argument");
        FVX_REQUIRE(dtype == FVX_F64 || dtype == FVX_F32, FVX_E_ARG, "dtype must be FVX_F64 or FVX_F32");
        const fvx_op *op = h->lv[0].op;
        FVX_REQUIRE(dtype == FVX_F64 || op->has_f32, FVX_E_ARG, "operator has no FP32 copies");
        FVX_REQUIRE(reinterpret_cast<uintptr_t>(ws) % 256 == 0, FVX_E_ARG, "ws must be 256-byte aligned");
        FVX_REQUIRE(reinterpret_cast<uintptr_t>(R) % 16 == 0 && reinterpret_cast<uintptr_t>(Z) % 16 == 0, FVX_E_ARG,
                    "R and Z must be 16-byte aligned");
        FVX_REQUIRE(ws_bytes >= fvx::amg_work_bytes(h, dtype), FVX_E_NOMEM, "workspace too small");
        const size_t es = dtype == FVX_F32 ? 4 : 8;
        const size_t nbytes = es * size_t(op->n_b) * op->ld;
        const char *r0 = static_cast<const char *>(R), *z0 = static_cast<const char *>(Z);
        FVX_REQUIRE(r0 + nbytes <= z0 || z0 + nbytes <= r0, FVX_E_ARG, "R and Z overlap");
        hipStream_t s = fvx::as_stream(stream);
        auto run = [&](auto tag) {
            using T = decltype(tag);
            const fvx::AmgWork<T> w = fvx::amg_carve<T>(h, static_cast<char *>(ws));
            hipLaunchKernelGGL(fvx::k_amg_clear_state, dim3(1), dim3(64), 0, s, w.st);
            fvx::CgDev d{};
            d.st = w.st;
            fvx::amg_vcycle<T>(h, static_cast<const T *>(R), w, d, nullptr, s);
            FVX_HIP(hipMemcpyAsync(Z, fvx::amg_output<T>(h, w), nbytes, hipMemcpyDeviceToDevice, s));
        };
        if (dtype == FVX_F32)
            run(float{});
        else
            run(double{});
        FVX_HIP(hipGetLastError());
        return FVX_OK;
    });
}

}  // extern "C"
