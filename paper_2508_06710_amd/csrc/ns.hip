// One time step of the incompressible Navier-Stokes equations on the
// extruded mesh with the operators of this library (Section 3, Eqs. 8-9, and
// Section 4: Heun's third-order Runge-Kutta scheme with a projection at every
// stage).  Velocities are cell-centred (three multivectors u, v, w of k
// columns) with face velocities u_s for the mass fluxes; in semi-discrete form
//   Omega du/dt = -C(u_s) u + nu L u - Omega Gamma_sc G p,   M u_s = 0,
// with C(u_s) = M U_s Pi (fvx_convect), L = M G (fvx_lap), the cell-to-face
// interpolation u_s = Gamma_cs u (normal component of the midpoint value)
// and its volume-weighted adjoint Gamma_sc = Omega^-1 Gamma_cs^T Omega_s.
//
// A stage with velocity u* is projected by solving L phi = M Gamma_cs u* /
// (c dt) (fvx_poisson_solve) and setting u_s = Gamma_cs u* - c dt G phi,
// u = u* - c dt Gamma_sc G phi.  Heun's scheme (nodes 0, 1/3, 2/3; weights
// 1/4, 0, 3/4):
//   u2* = u^n + dt/3 R(u^n),              projected with c = 1/3
//   u3* = u^n + 2 dt/3 R(u2),             projected with c = 2/3
//   u^{n+1}* = u^n + dt (R(u^n)/4 + 3 R(u3)/4), projected with c = 1,
// R(u) = Omega^-1 (-C(u_s) u + nu L_v u) per component.
#include <chrono>

#include "kernels.h"

namespace fvx {
namespace {

// Cell -> face: rows [0, F_b) are in-plane faces, u_s = n_f . (u_c1 + u_c2)/2;
// rows [F_b, F_b + n_b) are the faces above each plane, w_s = (w_l + w_{l+1})/2.
template <typename T, int V, bool Z>
__global__ __launch_bounds__(1024) void k_c2f(RowArgs<T> a, const T *__restrict__ U, const T *__restrict__ Vv,
                                              const T *__restrict__ W, T *__restrict__ Uf, T *__restrict__ Wz) {
    const int lpr = a.lpr;
    const int sub = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const bool single = lpr * V >= a.k;
    const T half = T(0.5);
    const int64_t t0 = logical_block(a.remap) * a.tiles_per_block;
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        if (row < a.F_b) {
            const int64_t c1 = a.A.f_c1[row], c2 = a.A.f_c2[row];
            const T nx = a.A.fnx[row] * half, ny = a.A.fny[row] * half;
            for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
                const vec_t<T, V> su = ldv<T, V>(U + c1 * a.ld + c0) + ldv<T, V>(U + c2 * a.ld + c0);
                const vec_t<T, V> sv = ldv<T, V>(Vv + c1 * a.ld + c0) + ldv<T, V>(Vv + c2 * a.ld + c0);
                stv_masked<T, V>(Uf + row * a.ld + c0, nx * su + ny * sv, a.k - c0);
            }
        } else if constexpr (Z) {
            const int64_t i = row - a.F_b;
            for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
                const vec_t<T, V> wo = ldv<T, V>(W + i * a.ld + c0);
                const auto nb = neighbours_of<T, V>(wo, PlainLoad<T, V>{W, a.ld}, i, c0, sub, lpr, a.k, single);
                vec_t<T, V> g;
#pragma unroll
                for (int q = 0; q < V; ++q) g[q] = half * (wo[q] + right_of<T, V>(wo, nb, q, c0 + q, a.k));
                stv_masked<T, V>(Wz + i * a.ld + c0, g, a.k - c0);
            }
        }
    }
}

// Face -> cell, accumulated: (u, v, w) += alpha Gamma_sc (Gf, Gz), with
// (Gamma_sc g)_c = sum_f (len_f dist_f / (2 area_c)) n_f g_f in the plane and
// (g_{l-1} + g_l) / 2 from the faces below and above.
template <typename T, int V, bool Z, int WT>
__global__ __launch_bounds__(1024) void k_f2c(RowArgs<T> a, const T *__restrict__ Gf, const T *__restrict__ Gz,
                                              T alpha, T *__restrict__ U, T *__restrict__ Vv, T *__restrict__ W) {
    const int lpr = a.lpr;
    const int sub = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const bool single = lpr * V >= a.k;
    const int64_t t0 = logical_block(a.remap) * a.tiles_per_block;
    for (int64_t t = t0; t < t0 + a.tiles_per_block; ++t) {
        const int64_t row = t * a.rows_per_tile + grp;
        if (row >= a.n_rows) break;
        const T sc = alpha * a.A.inv_area[row];
        for (int c0 = sub * V; c0 < a.k; c0 += lpr * V) {
            vec_t<T, V> gx = 0, gy = 0;
            auto face = [&](int64_t f, T cf) {
                if (cf == T(0)) return;  // padding entry
                const vec_t<T, V> g = ldv<T, V>(Gf + f * a.ld + c0);
                gx += a.A.gsx[f] * g;
                gy += a.A.gsy[f] * g;
            };
            if constexpr (WT > 0) {
#pragma unroll
                for (int e = 0; e < WT; ++e) face(a.A.cf_face[e * a.n_b + row], a.A.cf_coef[e * a.n_b + row]);
            } else {
                for (int e = 0; e < a.Wd; ++e) face(a.A.cf_face[e * a.n_b + row], a.A.cf_coef[e * a.n_b + row]);
            }
            const int64_t o = row * a.ld + c0;
            stv_masked<T, V>(U + o, ldv<T, V>(U + o) + sc * gx, a.k - c0);
            stv_masked<T, V>(Vv + o, ldv<T, V>(Vv + o) + sc * gy, a.k - c0);
            if constexpr (Z) {
                const vec_t<T, V> go = ldv<T, V>(Gz + o);
                const auto nb = neighbours_of<T, V>(go, PlainLoad<T, V>{Gz, a.ld}, row, c0, sub, lpr, a.k, single);
                vec_t<T, V> gz;
#pragma unroll
                for (int q = 0; q < V; ++q) gz[q] = T(0.5) * (left_of<T, V>(go, nb, q) + go[q]);
                stv_masked<T, V>(W + o, ldv<T, V>(W + o) + alpha * gz, a.k - c0);
            }
        }
    }
}

// out = s_row * (a0 X0 + a1 X1 + a2 X2) over [n_b][ld] (X1, X2 may be NULL;
// s_row = rowscale[row] * colfac, or 1 when rowscale is NULL).
template <typename T>
__global__ __launch_bounds__(256) void k_lincomb(int64_t n_b, int k, int ld, const T *__restrict__ X0, T a0,
                                                 const T *__restrict__ X1, T a1, const T *__restrict__ X2, T a2,
                                                 const T *__restrict__ rowscale, T colfac, T *__restrict__ out) {
    const int64_t n = n_b * k;
    for (int64_t idx = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; idx < n;
         idx += int64_t(gridDim.x) * blockDim.x) {
        const int64_t r = idx / k;
        const int64_t o = r * ld + idx % k;
        T v = a0 * X0[o];
        if (X1) v += a1 * X1[o];
        if (X2) v += a2 * X2[o];
        if (rowscale) v *= rowscale[r] * colfac;
        out[o] = v;
    }
}

void lincomb(const fvx_op *op, const double *X0, double a0, const double *X1, double a1, const double *X2, double a2,
             const double *rowscale, double colfac, double *out, hipStream_t s) {
    const int64_t n = op->n_b * op->k;
    const int blocks = int(std::min<int64_t>(std::max<int64_t>(1, ceil_div(n, 256)), 8192));
    hipLaunchKernelGGL(k_lincomb<double>, dim3(blocks), dim3(256), 0, s, op->n_b, op->k, op->ld, X0, a0, X1, a1, X2,
                       a2, rowscale, colfac, out);
}

void cell_to_face(const fvx_op *op, double *const U[3], double *Uf, double *Wz, hipStream_t s) {
    RowGrid g;
    const fvx_tile &t = op->tile[FVX_F64];
    auto a = row_args<double>(op, op->F_b + (op->zfaces ? op->n_b : 0), g, t);
    by_vec<double>(t.vec, op->zfaces, [&](auto V, auto Z) {
        hipLaunchKernelGGL((k_c2f<double, decltype(V)::value, decltype(Z)::value>), dim3(g.n_blocks), dim3(t.block), 0,
                           s, a, U[0], U[1], U[2], Uf, Wz);
    });
}

void face_to_cell_axpy(const fvx_op *op, const double *Gf, const double *Gz, double alpha, double *const U[3],
                       hipStream_t s) {
    RowGrid g;
    const fvx_tile &t = op->tile[FVX_F64];
    auto a = row_args<double>(op, op->n_b, g, t);
    by_vec<double>(t.vec, op->zfaces, [&](auto V, auto Z) {
        by_width(op->Wd, [&](auto Wt) {
            hipLaunchKernelGGL((k_f2c<double, decltype(V)::value, decltype(Z)::value, decltype(Wt)::value>),
                               dim3(g.n_blocks), dim3(t.block), 0, s, a, Gf, Gz, alpha, U[0], U[1], U[2]);
        });
    });
}

struct NsWork {
    double *un[3], *r1[3], *r2[3], *us[3];
    double *conv, *lap, *rhs, *phi, *gz, *wz_star;
    double *uf_star, *gf;
    char *solve_ws;
    size_t solve_bytes, bytes;
};

NsWork carve_ns(void *ws, const fvx_op *op, size_t solve_bytes) {
    NsWork w{};
    char *base = static_cast<char *>(ws);
    size_t off = 0;
    const size_t nv = size_t(op->n_b) * op->ld, nf = size_t(std::max<int64_t>(op->F_b, 1)) * op->ld;
    auto take = [&](size_t n) {
        double *p = base ? reinterpret_cast<double *>(base + off) : nullptr;
        off += (8 * n + 255) / 256 * 256;
        return p;
    };
    for (int d = 0; d < 3; ++d) {
        w.un[d] = take(nv);
        w.r1[d] = take(nv);
        w.r2[d] = take(nv);
        w.us[d] = take(nv);
    }
    w.conv = take(nv);
    w.lap = take(nv);
    w.rhs = take(nv);
    w.phi = take(nv);
    w.gz = take(nv);
    w.wz_star = take(nv);
    w.uf_star = take(nf);
    w.gf = take(nf);
    w.solve_ws = base ? base + off : nullptr;
    w.solve_bytes = solve_bytes;
    off += (solve_bytes + 255) / 256 * 256;
    w.bytes = off;
    return w;
}

void check_ns(const fvx_op *op, const fvx_solve_opts *o) {
    FVX_REQUIRE(op && o, FVX_E_ARG, "NULL op or options");
    FVX_REQUIRE(op->d64.fnx != nullptr, FVX_E_UNSUPPORTED,
                "the time step needs face normals (Cartesian or triangle base meshes)");
    FVX_REQUIRE(o->precision == FVX_F64, FVX_E_UNSUPPORTED, "the time step runs in FP64");
}

}  // namespace
}  // namespace fvx

using fvx::guard;

extern "C" {

int fvx_ns_step_bytes(const fvx_op *op, const fvx_solve_opts *opts, size_t *bytes) {
    return guard([&]() -> int {
        fvx::check_ns(op, opts);
        FVX_REQUIRE(bytes, FVX_E_ARG, "bytes is NULL");
        size_t sb = 0;
        const int rc = fvx_solve_bytes(op, opts, &sb);
        if (rc != FVX_OK) return rc;
        *bytes = fvx::carve_ns(nullptr, op, sb).bytes;
        return FVX_OK;
    });
}

int fvx_ns_step(const fvx_op *op, const fvx_op *visc, double *const U[3], double *Uf, double *Wz, double *P,
                double dt, double nu, const fvx_solve_opts *opts, void *ws, size_t ws_bytes, fvx_solve_stats *stats,
                void *stream) {
    return guard([&]() -> int {
        using namespace fvx;
        const auto t_start = std::chrono::steady_clock::now();
        check_ns(op, opts);
        FVX_REQUIRE(U && U[0] && U[1] && U[2] && Uf && P && ws, FVX_E_ARG, "NULL argument");
        FVX_REQUIRE(!op->zfaces || Wz, FVX_E_ARG, "Wz is required when the planes are coupled");
        FVX_REQUIRE(dt > 0 && std::isfinite(dt) && nu >= 0 && std::isfinite(nu), FVX_E_ARG, "dt > 0 and nu >= 0");
        FVX_REQUIRE(reinterpret_cast<uintptr_t>(ws) % 256 == 0, FVX_E_ARG, "ws must be 256-byte aligned");
        const fvx_op *vop = visc ? visc : op;
        FVX_REQUIRE(vop->n_b == op->n_b && vop->k == op->k && vop->ld == op->ld && vop->F_b == op->F_b &&
                        vop->zfaces == op->zfaces && vop->stencil == 7,
                    FVX_E_ARG, "visc must be a 7-point operator on the same mesh, planes and coupling");
        size_t sb = 0;
        int rc = fvx_solve_bytes(op, opts, &sb);
        if (rc != FVX_OK) return rc;
        const NsWork w = carve_ns(ws, op, sb);
        FVX_REQUIRE(ws_bytes >= w.bytes, FVX_E_NOMEM, "workspace too small: need " + std::to_string(w.bytes));
        hipStream_t s = as_stream(stream);
        const double *inv_area = op->d64.inv_area;
        const double inv_dz = 1.0 / op->dz;
        const size_t vb = sizeof(double) * size_t(op->n_b) * op->ld;
        for (int d = 0; d < 3; ++d) FVX_HIP(hipMemcpyAsync(w.un[d], U[d], vb, hipMemcpyDeviceToDevice, s));

        // R(u) = Omega^-1 (-C(u_s) u + nu L_v u) per component, with the current u_s.
        auto rhs = [&](double *const u[3], const double *uf, const double *wz, double *const r[3]) {
            for (int d = 0; d < 3; ++d) {
                launch_convect<double>(op, uf, wz, u[d], w.conv, s);
                launch_lap<double>(vop, u[d], w.lap, nullptr, s);
                lincomb(op, w.conv, -1.0, w.lap, nu, nullptr, 0.0, inv_area, inv_dz, r[d], s);
            }
        };
        int iters = 0, status = FVX_OK;
        fvx_solve_stats last{};
        // Projection of the stage velocity u* (in `u`) with factor c dt; u_s
        // ends in (Uf, Wz) and phi in P.
        auto project = [&](double *const u[3], double cdt) {
            cell_to_face(op, u, w.uf_star, w.wz_star, s);
            launch_div<double>(op, w.uf_star, op->zfaces ? w.wz_star : nullptr, w.rhs, s);
            lincomb(op, w.rhs, 1.0 / cdt, nullptr, 0.0, nullptr, 0.0, nullptr, 1.0, w.rhs, s);
            fvx_solve_opts o = *opts;
            const int src = fvx_poisson_solve(op, w.rhs, P, &o, w.solve_ws, w.solve_bytes, &last, stream);
            if (src < 0) throw Error(src, std::string("projection solve: ") + fvx_last_error());
            if (src > 0 && status == FVX_OK) status = src;
            iters += last.iters;
            // u_s = u_s* - c dt G phi;  u = u* - c dt Gamma_sc G phi
            FVX_HIP(hipMemcpyAsync(Uf, w.uf_star, sizeof(double) * size_t(op->F_b) * op->ld, hipMemcpyDeviceToDevice,
                                   s));
            if (op->zfaces) FVX_HIP(hipMemcpyAsync(Wz, w.wz_star, vb, hipMemcpyDeviceToDevice, s));
            launch_grad<double>(op, P, Uf, op->zfaces ? Wz : nullptr, s, -cdt, true);
            launch_grad<double>(op, P, w.gf, op->zfaces ? w.gz : nullptr, s, 1.0, false);
            face_to_cell_axpy(op, w.gf, w.gz, -cdt, u, s);
        };
        double *const *un = w.un;
        double *const *r1 = w.r1, *const *r2 = w.r2, *const *ust = w.us;
        // Stage 1: R1 = R(u^n, u_s^n).
        rhs(un, Uf, Wz, r1);
        // Stage 2.
        for (int d = 0; d < 3; ++d) lincomb(op, un[d], 1.0, r1[d], dt / 3.0, nullptr, 0.0, nullptr, 1.0, ust[d], s);
        project(ust, dt / 3.0);
        rhs(ust, Uf, Wz, r2);
        // Stage 3.
        for (int d = 0; d < 3; ++d)
            lincomb(op, un[d], 1.0, r2[d], 2.0 * dt / 3.0, nullptr, 0.0, nullptr, 1.0, ust[d], s);
        project(ust, 2.0 * dt / 3.0);
        rhs(ust, Uf, Wz, r2);  // R3 (R2 is no longer needed)
        // Final combination and projection into the caller's arrays.
        for (int d = 0; d < 3; ++d)
            lincomb(op, un[d], 1.0, r1[d], 0.25 * dt, r2[d], 0.75 * dt, nullptr, 1.0, U[d], s);
        project(U, dt);
        FVX_HIP(hipGetLastError());
        FVX_HIP(hipStreamSynchronize(s));
        if (stats) {
            *stats = last;
            stats->iters = iters;
            stats->status = status;
            stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        }
        return status;
    });
}

}  // extern "C"
