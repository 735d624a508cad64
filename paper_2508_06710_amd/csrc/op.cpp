// Host operator builder: base mesh + k -> the base block A_b, the plane
// coupling weights, the divergence incidence M_b and the gradient G_b, stored
// once on the device (Section 3.1: operators are stored as for one system,
// only the fields grow with the number of planes).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

#include "common.h"

namespace fvx {

namespace {

// Host image of the operator in FP64, before it is laid out on the device.
struct HostOp {
    int64_t n_b = 0, F_b = 0, nnz_b = 0;
    int W = 0, Wd = 0;
    std::vector<double> diag, w, ell_val, area, cf_coef, f_invd;
    std::vector<double> ell_v1, w2;  // structured 13/27-point operators only
    std::vector<double> fnx, fny, gsx, gsy, inv_area;  // velocity interpolation (meshes with face normals)
    std::vector<int32_t> ell_col, cf_face, f_c1, f_c2;
    // FP32 copies: diagonal rebuilt in FP32 so that rows sum to zero up to
    // FP32 rounding of that sum.
    std::vector<float> diag32;
    // Cartesian 5-point record [n_b][8] (diag, w, S, W, E, N, 0, 0); empty
    // when the base is not such a grid.
    std::vector<double> cart;
    int nx = 0, ny = 0, px = 0, py = 0;
    // structured 13/27-point operators: 1 when every row's 8 ELL entries are
    // stored in the fixed direction order of stencil_dirs (an absent
    // neighbour, past a wall, being the row itself with value 0)
    int sdir = 0;
    // and then each row's coefficients packed [n_b][srec_width]: the 8 entries,
    // diagonal, w, then the 8 neighbouring-plane entries (27-point) or w2 and a
    // pad (13-point), so that a row's coefficients are one contiguous record
    std::vector<double> srec;
};

// One axis of a Cartesian base: cell centres and, when periodic, the period.
struct Axis {
    int n;
    bool periodic;
    std::vector<double> c;
    double period;
    Axis(const std::vector<double> &faces, bool per) : n(int(faces.size()) - 1), periodic(per) {
        for (int i = 0; i < n; ++i) c.push_back(0.5 * (faces[i] + faces[i + 1]));
        period = faces[n] - faces[0];
    }
    // index i + d on the axis (wrapped when periodic), or -1 past a wall
    int at(int i, int d) const {
        const int v = i + d;
        if (periodic) return ((v % n) + n) % n;
        return v >= 0 && v < n ? v : -1;
    }
    // distance from centre i forward to centre i + d (d >= 1, across the period if needed)
    double ahead(int i, int d) const {
        double s = 0.0;
        for (int q = 0; q < d; ++q) {
            const int u = (i + q) % n;
            s += u + 1 < n ? c[u + 1] - c[u] : c[0] + period - c[u];
        }
        return s;
    }
    // Row i of the 1D element stiffness K and consistent mass M on the centres
    // (linear elements between consecutive centres; node -> (K, M)).
    std::map<int, std::pair<double, double>> km(int i) const {
        std::map<int, std::pair<double, double>> r;
        std::vector<int> elems;
        if (periodic) {
            elems.push_back(((i - 1) % n + n) % n);
            if (elems[0] != i) elems.push_back(i);
        } else {
            if (i >= 1) elems.push_back(i - 1);
            if (i + 1 < n) elems.push_back(i);
        }
        for (int e : elems) {
            const int u = e, v = (e + 1) % n;
            const double s = ahead(e, 1);
            for (int side = 0; side < 2; ++side) {
                const int me = side == 0 ? u : v, other = side == 0 ? v : u;
                if (me != i) continue;
                r[i].first += 1.0 / s;
                r[other].first -= 1.0 / s;
                r[i].second += s / 3.0;
                r[other].second += s / 6.0;
            }
        }
        return r;
    }
};

// The fixed order of the 8 in-plane entries of a structured operator row,
// as (dj, di) offsets: 27-point SW, S, SE, W, E, NW, N, NE; 13-point SS, S,
// WW, W, E, EE, N, NN -- the column order of an interior row.
const int (*stencil_dirs(int stencil))[2] {
    static const int d27[8][2] = {{-1, -1}, {-1, 0}, {-1, 1}, {0, -1}, {0, 1}, {1, -1}, {1, 0}, {1, 1}};
    static const int d13[8][2] = {{-2, 0}, {-1, 0}, {0, -2}, {0, -1}, {0, 1}, {0, 2}, {1, 0}, {2, 0}};
    return stencil == 27 ? d27 : d13;
}

// The structured 13- and 27-point operators (Section 4.1) on a Cartesian
// base repeated in periodic planes: in-plane entries (shift 0 and, for 27,
// planes l +- 1 of each neighbour), the row's own planes l +- 1 and (13)
// l +- 2.  Neighbours that meet at one cell (short periodic axes) are merged;
// a neighbour that is the row itself joins the diagonal.
HostOp build_host_stencil(const fvx_mesh &m, const fvx_op_desc &d) {
    HostOp h;
    const int nx = m.grid_nx, ny = m.grid_ny;
    const int64_t nb = int64_t(nx) * ny;
    const double dz = d.dz;
    h.n_b = nb;
    h.F_b = m.n_faces;
    const Axis ax(m.xf, m.periodic_x), ay(m.yf, m.periodic_y);
    std::vector<std::map<int32_t, std::pair<double, double>>> nbr(nb);  // col -> (shift 0, planes +-1)
    h.diag.assign(nb, 0.0);
    h.w.assign(nb, 0.0);
    h.w2.assign(nb, 0.0);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const int32_t r = j * nx + i;
            const double hx = m.xf[i + 1] - m.xf[i], hy = m.yf[j + 1] - m.yf[j];
            if (d.stencil == 27) {
                // planes: M = 2dz/3 (same plane), dz/6 (l +- 1); K = 2/dz, -1/dz
                const double mz0 = 2.0 * dz / 3.0, mz1 = dz / 6.0, kz0 = 2.0 / dz, kz1 = -1.0 / dz;
                for (const auto &X : ax.km(i))
                    for (const auto &Y : ay.km(j)) {
                        const double kx = X.second.first, mx = X.second.second;
                        const double ky = Y.second.first, my = Y.second.second;
                        const double v0 = -(kx * my * mz0 + mx * ky * mz0 + mx * my * kz0);
                        const double v1 = -(kx * my * mz1 + mx * ky * mz1 + mx * my * kz1);
                        const int32_t c = Y.first * nx + X.first;
                        if (c == r) {
                            h.diag[r] += v0;
                            h.w[r] += v1;
                        } else {
                            nbr[r][c].first += v0;
                            nbr[r][c].second += v1;
                        }
                    }
            } else {
                double off = 0.0;
                for (int dd = 1; dd <= 2; ++dd) {
                    const double wt = dd == 1 ? 4.0 / 3.0 : -1.0 / 6.0;
                    for (int sgn : {-1, 1}) {
                        const int I = ax.at(i, sgn * dd), J = ay.at(j, sgn * dd);
                        if (I >= 0) {
                            const double dist = sgn > 0 ? ax.ahead(i, dd) : ax.ahead(I, dd);
                            const double cf = wt * hy * dz / dist;
                            const int32_t c = j * nx + I;
                            off += cf;
                            if (c == r)
                                h.diag[r] += cf;
                            else
                                nbr[r][c].first += cf;
                        }
                        if (J >= 0) {
                            const double dist = sgn > 0 ? ay.ahead(j, dd) : ay.ahead(J, dd);
                            const double cf = wt * hx * dz / dist;
                            const int32_t c = J * nx + i;
                            off += cf;
                            if (c == r)
                                h.diag[r] += cf;
                            else
                                nbr[r][c].first += cf;
                        }
                    }
                }
                const double area = hx * hy;
                h.w[r] = (4.0 / 3.0) * area / dz;
                h.w2[r] = -(1.0 / 6.0) * area / (2.0 * dz);
                h.diag[r] -= off + 2.0 * h.w[r] + 2.0 * h.w2[r];
            }
        }
    h.W = 8;  // the 8 in-plane neighbours (fewer on short periodic axes, padded)
    for (int64_t i = 0; i < nb; ++i) FVX_REQUIRE(nbr[i].size() <= 8, FVX_E_MESH, "structured stencil row too wide");
    h.ell_col.assign(size_t(h.W) * nb, 0);
    h.ell_val.assign(size_t(h.W) * nb, 0.0);
    if (d.stencil == 27) h.ell_v1.assign(size_t(h.W) * nb, 0.0);
    if (d.stencil != 13) h.w2.clear();
    // Entry order: the fixed direction order when every direction of every
    // row is a distinct cell or past a wall (axes of at least 3 cells for the
    // 27-point operator, 5 for the 13-point one), else by column index.
    const int (*dirs)[2] = stencil_dirs(d.stencil);
    const int reach = d.stencil == 27 ? 1 : 2;
    h.sdir = nx >= 2 * reach + 1 && ny >= 2 * reach + 1;
    h.nnz_b = nb;
    for (int j = 0; j < ny && h.sdir; ++j)
        for (int i = 0; i < nx; ++i) {
            const int64_t r = int64_t(j) * nx + i;
            size_t found = 0;
            for (int e = 0; e < 8; ++e) {
                const int J = ay.at(j, dirs[e][0]), I = ax.at(i, dirs[e][1]);
                if (I >= 0 && J >= 0 && nbr[r].count(J * nx + I)) ++found;
            }
            if (found != nbr[r].size()) h.sdir = 0;
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const int64_t r = int64_t(j) * nx + i;
            int e = 0;
            if (h.sdir) {
                for (; e < 8; ++e) {
                    const int J = ay.at(j, dirs[e][0]), I = ax.at(i, dirs[e][1]);
                    const auto it = (I >= 0 && J >= 0) ? nbr[r].find(J * nx + I) : nbr[r].end();
                    h.ell_col[size_t(e) * nb + r] = it == nbr[r].end() ? int32_t(r) : it->first;
                    if (it == nbr[r].end()) continue;  // past a wall: the row itself, value 0
                    h.ell_val[size_t(e) * nb + r] = it->second.first;
                    if (!h.ell_v1.empty()) h.ell_v1[size_t(e) * nb + r] = it->second.second;
                }
                h.nnz_b += int64_t(nbr[r].size());
                continue;
            }
            for (const auto &kv : nbr[r]) {
                h.ell_col[size_t(e) * nb + r] = kv.first;
                h.ell_val[size_t(e) * nb + r] = kv.second.first;
                if (!h.ell_v1.empty()) h.ell_v1[size_t(e) * nb + r] = kv.second.second;
                ++e;
            }
            h.nnz_b += e;
            for (; e < h.W; ++e) h.ell_col[size_t(e) * nb + r] = int32_t(r);  // padding: self, value 0
        }
    h.nx = nx;
    h.ny = ny;
    h.px = m.periodic_x;
    h.py = m.periodic_y;
    h.diag32.assign(nb, 0.0f);
    for (int64_t i = 0; i < nb; ++i) h.diag32[i] = float(h.diag[i]);
    if (h.sdir) {
        const int wd = fvx::srec_width(d.stencil);
        h.srec.assign(size_t(wd) * nb, 0.0);
        for (int64_t r = 0; r < nb; ++r) {
            double *o = &h.srec[size_t(r) * wd];
            for (int e = 0; e < 8; ++e) o[e] = h.ell_val[size_t(e) * nb + r];
            o[8] = h.diag[r];
            o[9] = h.w[r];
            if (d.stencil == 27)
                for (int e = 0; e < 8; ++e) o[10 + e] = h.ell_v1[size_t(e) * nb + r];
            else
                o[10] = h.w2[r];
        }
    }
    return h;
}

// The divergence and gradient data of the face graph (all operators).
void build_div_grad(const fvx_mesh &m, const fvx_op_desc &d, HostOp &h);

HostOp build_host(const fvx_mesh &m, const fvx_op_desc &d) {
    if (d.stencil == 13 || d.stencil == 27) {
        HostOp h = build_host_stencil(m, d);
        build_div_grad(m, d, h);
        return h;
    }
    HostOp h;
    const int64_t nb = m.n_cells;
    h.n_b = nb;
    h.F_b = m.n_faces;
    const bool zf = d.coupling == FVX_COUPLING_PERIODIC_Z && d.k >= 2;
    const double dz = d.dz;

    // Off-diagonal neighbours per row, duplicates (two faces between the same
    // cells, as on a two-cell periodic ring) merged.
    std::vector<std::map<int32_t, double>> nbr(nb);
    h.diag.assign(nb, 0.0);
    for (int f = 0; f < m.n_faces; ++f) {
        const int a = m.c1[f], b = m.c2[f];
        if (a == b) continue;  // a face from a cell to itself carries no net flux
        const double coef = m.len[f] * dz / m.dist[f];
        nbr[a][b] += coef;
        nbr[b][a] += coef;
        h.diag[a] -= coef;
        h.diag[b] -= coef;
    }
    h.w.assign(nb, 0.0);
    if (zf)
        for (int64_t c = 0; c < nb; ++c) {
            h.w[c] = m.area[c] / dz;
            h.diag[c] -= h.w[c];
            h.diag[c] -= h.w[c];
        }
    std::vector<double> wall(nb, 0.0);
    if (d.wall_bc == FVX_WALL_DIRICHLET)
        for (int i = 0; i < m.n_walls; ++i) {
            const double t = m.wlen[i] * dz / m.wdist[i];
            wall[m.wcell[i]] -= t;
            h.diag[m.wcell[i]] -= t;
        }

    h.W = 0;
    for (int64_t i = 0; i < nb; ++i) h.W = std::max<int>(h.W, int(nbr[i].size()));
    h.W = ell_width(h.W);
    h.ell_col.assign(size_t(h.W) * nb, 0);
    h.ell_val.assign(size_t(h.W) * nb, 0.0);
    h.diag32.assign(nb, 0.0f);
    h.nnz_b = nb;
    for (int64_t i = 0; i < nb; ++i) {
        int e = 0;
        float s32 = 0.0f;
        for (const auto &kv : nbr[i]) {
            h.ell_col[size_t(e) * nb + i] = kv.first;
            h.ell_val[size_t(e) * nb + i] = kv.second;
            s32 += float(kv.second);
            ++e;
        }
        h.nnz_b += e;
        for (; e < h.W; ++e) {
            h.ell_col[size_t(e) * nb + i] = int32_t(i);
            h.ell_val[size_t(e) * nb + i] = 0.0;
        }
        if (zf) {
            s32 += float(h.w[i]);
            s32 += float(h.w[i]);
        }
        h.diag32[i] = -s32 + float(wall[i]);
    }
    build_div_grad(m, d, h);
    return h;
}

void build_div_grad(const fvx_mesh &m, const fvx_op_desc &d, HostOp &h) {
    const int64_t nb = m.n_cells;
    const double dz = d.dz;
    // Divergence: cell -> face incidence.
    std::vector<std::vector<std::pair<int32_t, double>>> inc(nb);
    for (int f = 0; f < m.n_faces; ++f) {
        const int a = m.c1[f], b = m.c2[f];
        if (a == b) continue;
        const double s = m.len[f] * dz;
        inc[a].push_back({f, +s});
        inc[b].push_back({f, -s});
    }
    h.Wd = 0;
    for (int64_t i = 0; i < nb; ++i) h.Wd = std::max<int>(h.Wd, int(inc[i].size()));
    h.Wd = ell_width(h.Wd);
    h.cf_face.assign(size_t(h.Wd) * nb, 0);
    h.cf_coef.assign(size_t(h.Wd) * nb, 0.0);
    for (int64_t i = 0; i < nb; ++i)
        for (size_t e = 0; e < inc[i].size(); ++e) {
            h.cf_face[e * nb + i] = inc[i][e].first;
            h.cf_coef[e * nb + i] = inc[i][e].second;
        }
    h.area = m.area;
    h.f_c1 = m.c1;
    h.f_c2 = m.c2;
    h.f_invd.resize(m.n_faces);
    for (int f = 0; f < m.n_faces; ++f) h.f_invd[f] = 1.0 / m.dist[f];
    if (m.n_faces > 0 && m.fnx.size() == size_t(m.n_faces)) {
        h.fnx = m.fnx;
        h.fny = m.fny;
        h.gsx.resize(m.n_faces);
        h.gsy.resize(m.n_faces);
        for (int f = 0; f < m.n_faces; ++f) {
            h.gsx[f] = 0.5 * m.len[f] * m.dist[f] * m.fnx[f];
            h.gsy[f] = 0.5 * m.len[f] * m.dist[f] * m.fny[f];
        }
        h.inv_area.resize(m.n_cells);
        for (int c = 0; c < m.n_cells; ++c) h.inv_area[c] = 1.0 / m.area[c];
    }
}

// Byte layout of the device image; every array starts on a 256-byte boundary.
struct Layout {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    }
};

struct Offsets {
    size_t ell_col, cf_face, f_c1, f_c2, cart[2];
    size_t diag[2], ell_val[2], w[2], cf_coef[2], area[2], f_invd[2], ell_v1[2], w2[2], dinv[2], srec[2];
    size_t fnx[2], fny[2], gsx[2], gsy[2], inv_area[2];
    size_t total;
};

Offsets layout(const HostOp &h, bool f32) {
    Layout L;
    Offsets o{};
    const size_t nb = size_t(h.n_b), fb = size_t(h.F_b);
    o.ell_col = L.take(sizeof(int32_t) * h.W * nb);
    o.cf_face = L.take(sizeof(int32_t) * h.Wd * nb);
    o.f_c1 = L.take(sizeof(int32_t) * fb);
    o.f_c2 = L.take(sizeof(int32_t) * fb);
    for (int p = 0; p < (f32 ? 2 : 1); ++p) {
        const size_t v = p == 0 ? 8 : 4;
        o.diag[p] = L.take(v * nb);
        o.ell_val[p] = L.take(v * h.W * nb);
        o.w[p] = L.take(v * nb);
        o.cf_coef[p] = L.take(v * h.Wd * nb);
        o.area[p] = L.take(v * nb);
        o.f_invd[p] = L.take(v * fb);
        o.ell_v1[p] = L.take(v * h.ell_v1.size());
        o.w2[p] = L.take(v * h.w2.size());
        o.dinv[p] = L.take(v * nb);
        o.fnx[p] = L.take(v * h.fnx.size());
        o.fny[p] = L.take(v * h.fny.size());
        o.gsx[p] = L.take(v * h.gsx.size());
        o.gsy[p] = L.take(v * h.gsy.size());
        o.inv_area[p] = L.take(v * h.inv_area.size());
        o.cart[p] = L.take(v * h.cart.size());
        o.srec[p] = L.take(v * h.srec.size());
    }
    o.total = L.off;
    return o;
}

void check_desc(const fvx_mesh *m, const fvx_op_desc *d) {
    FVX_REQUIRE(m && d, FVX_E_ARG, "NULL mesh or descriptor");
    FVX_REQUIRE(d->k >= 1, FVX_E_ARG, "k must be >= 1");
    FVX_REQUIRE(d->coupling == FVX_COUPLING_NONE || d->coupling == FVX_COUPLING_PERIODIC_Z,
                FVX_E_ARG, "unknown coupling");
    FVX_REQUIRE(d->dz > 0 && std::isfinite(d->dz), FVX_E_ARG, "dz must be > 0");
    FVX_REQUIRE(d->wall_bc == FVX_WALL_NEUMANN || d->wall_bc == FVX_WALL_DIRICHLET, FVX_E_ARG,
                "unknown wall_bc");
    FVX_REQUIRE(m->n_cells < (1 << 30) && m->n_faces < (1 << 30), FVX_E_ARG, "mesh too large for int32 indices");
    FVX_REQUIRE(d->stencil == 0 || d->stencil == 7 || d->stencil == 13 || d->stencil == 27, FVX_E_ARG,
                "stencil must be 0, 7, 13 or 27");
    if (d->stencil == 13 || d->stencil == 27) {
        FVX_REQUIRE(m->grid_nx > 0 && m->grid_ny > 0, FVX_E_ARG, "13/27-point operators need a Cartesian base mesh");
        FVX_REQUIRE(d->coupling == FVX_COUPLING_PERIODIC_Z, FVX_E_ARG, "13/27-point operators need PERIODIC_Z");
        FVX_REQUIRE(d->wall_bc == FVX_WALL_NEUMANN, FVX_E_ARG, "13/27-point operators have zero-flux walls");
        FVX_REQUIRE(d->k <= 64 || (d->k <= 128 && d->k % 2 == 0), FVX_E_UNSUPPORTED,
                    "13/27-point operators support k <= 64, or even k <= 128 (one pass of a row group)");
    }
}

// The Cartesian record of a 7-point operator on an nx x ny grid: every ELL
// entry of row (i, j) must be exactly one of its S, W, E, N neighbours
// (periodic axes need at least 3 cells, so that no two directions meet the
// same cell, and the ELL width is 4); otherwise no record is built.  With a
// record, the ELL rows are stored in that direction order too (an absent
// neighbour as padding in its place), so that every kernel sums a row's
// entries in the same order.
void build_cart(const fvx_mesh &m, HostOp &h) {
    const int nx = m.grid_nx, ny = m.grid_ny;
    if (nx <= 0 || ny <= 0 || int64_t(nx) * ny != h.n_b || h.W != 4) return;
    const bool px = m.periodic_x, py = m.periodic_y;
    if ((px && nx < 3) || (py && ny < 3)) return;
    const int64_t nb = h.n_b;
    std::vector<double> rec(size_t(nb) * 8, 0.0);
    for (int64_t row = 0; row < nb; ++row) {
        const int64_t i = row % nx, j = row / nx;
        const int64_t dir[4] = {j > 0 ? row - nx : (py ? row + int64_t(nx) * (ny - 1) : -1),
                                i > 0 ? row - 1 : (px ? row + nx - 1 : -1),
                                i < nx - 1 ? row + 1 : (px ? row - (nx - 1) : -1),
                                j < ny - 1 ? row + nx : (py ? row - int64_t(nx) * (ny - 1) : -1)};
        double *r = &rec[size_t(row) * 8];
        r[0] = h.diag[row];
        r[1] = h.w[row];
        bool seen[4] = {false, false, false, false};
        for (int e = 0; e < h.W; ++e) {
            const int64_t c = h.ell_col[size_t(e) * nb + row];
            const double v = h.ell_val[size_t(e) * nb + row];
            if (c == row && v == 0.0) continue;  // padding
            int d = 0;
            while (d < 4 && dir[d] != c) ++d;
            if (d == 4 || seen[d]) return;
            seen[d] = true;
            r[2 + d] = v;
        }
    }
    for (int64_t row = 0; row < nb; ++row) {
        const int64_t i = row % nx, j = row / nx;
        const int64_t dir[4] = {j > 0 ? row - nx : (py ? row + int64_t(nx) * (ny - 1) : row),
                                i > 0 ? row - 1 : (px ? row + nx - 1 : row),
                                i < nx - 1 ? row + 1 : (px ? row - (nx - 1) : row),
                                j < ny - 1 ? row + nx : (py ? row - int64_t(nx) * (ny - 1) : row)};
        for (int d = 0; d < 4; ++d) {
            h.ell_col[size_t(d) * nb + row] = int32_t(dir[d]);
            h.ell_val[size_t(d) * nb + row] = rec[size_t(row) * 8 + 2 + d];
        }
    }
    h.cart = std::move(rec);
    h.nx = nx;
    h.ny = ny;
    h.px = px;
    h.py = py;
}

template <typename T>
std::vector<T> cast(const std::vector<double> &v) {
    return std::vector<T>(v.begin(), v.end());
}

}  // namespace

fvx_tile default_tile(const fvx_op *op, int dtype) {
    fvx_tile t{};
    const int vmax = dtype == FVX_F32 ? 4 : 2;
    int v = 1;
    for (int c = vmax; c >= 1; c >>= 1)
        if (op->ld % c == 0 && (op->stencil == 7 || op->k % c == 0)) {
            v = c;
            break;
        }
    t.vec = v;
    t.lanes_per_row = std::min(64, next_pow2(int(ceil_div(op->k, v))));
    t.block = 256;
    t.xcd_remap = 1;
    t.max_blocks = 0;
    t.stage_lds = 0;
    t.nt_store = 0;
    return t;
}

void check_tile(const fvx_op *op, int dtype, const fvx_tile &t) {
    const int vmax = dtype == FVX_F32 ? 4 : 2;
    FVX_REQUIRE(t.vec == 1 || t.vec == 2 || t.vec == 4, FVX_E_ARG, "tile.vec must be 1, 2 or 4");
    FVX_REQUIRE(t.vec <= vmax, FVX_E_ARG, "tile.vec exceeds 16 bytes for this precision");
    FVX_REQUIRE(op->ld % t.vec == 0, FVX_E_ARG, "tile.vec must divide ld");
    FVX_REQUIRE(t.lanes_per_row >= 1 && t.lanes_per_row <= 64 &&
                    (t.lanes_per_row & (t.lanes_per_row - 1)) == 0,
                FVX_E_ARG, "tile.lanes_per_row must be a power of two in 1..64");
    FVX_REQUIRE(t.block >= 64 && t.block <= 1024 && t.block % 64 == 0, FVX_E_ARG,
                "tile.block must be a multiple of 64 in 64..1024");
    FVX_REQUIRE(t.block >= t.lanes_per_row, FVX_E_ARG, "tile.block must hold one row group");
    FVX_REQUIRE(t.max_blocks >= 0, FVX_E_ARG, "tile.max_blocks must be >= 0");
    FVX_REQUIRE(t.stage_lds == 0 || t.stage_lds == 1, FVX_E_ARG, "tile.stage_lds must be 0 or 1");
    FVX_REQUIRE(!t.stage_lds || t.block / t.lanes_per_row <= kMaxStageRows, FVX_E_ARG,
                "tile.stage_lds needs at most 64 rows per tile");
    FVX_REQUIRE(t.nt_store == 0 || t.nt_store == 1, FVX_E_ARG, "tile.nt_store must be 0 or 1");
    if (op->stencil != 7) {
        const int span = t.lanes_per_row * t.vec;
        const bool one = span >= op->k && op->k % t.vec == 0;
        const bool multi = span >= 2 && t.block <= 512 && (op->k == 2 * span || op->k == 4 * span);
        FVX_REQUIRE(one || multi, FVX_E_ARG,
                    "13/27-point operators need one pass of a row group over k with vec dividing k, or exactly 2 or 4 "
                    "passes (block <= 512)");
        FVX_REQUIRE(!t.stage_lds, FVX_E_ARG, "13/27-point operators do not stage rows in LDS");
    }
}

RowGrid row_grid(int64_t n_rows, const fvx_tile &t, int max_blocks) {
    RowGrid g;
    g.n_rows = n_rows;
    g.rows_per_tile = t.block / t.lanes_per_row;
    const int64_t tiles = std::max<int64_t>(1, ceil_div(n_rows, g.rows_per_tile));
    const int64_t nb = std::min<int64_t>(tiles, max_blocks);
    g.tiles_per_block = ceil_div(tiles, nb);
    g.n_blocks = int(ceil_div(tiles, g.tiles_per_block));
    return g;
}

void expand_csr(const fvx_mesh &m, const fvx_op_desc &d, std::vector<int32_t> &ptr, std::vector<int32_t> &col,
                std::vector<double> &val) {
    check_desc(&m, &d);
    const HostOp h = build_host(m, d);
    const int64_t nb = h.n_b, N = nb * int64_t(d.k);
    FVX_REQUIRE(N < (int64_t(1) << 31), FVX_E_ARG, "expanded matrix too large for int32 indices");
    const bool structured = d.stencil == 13 || d.stencil == 27;
    const bool zf = (d.coupling == FVX_COUPLING_PERIODIC_Z && d.k >= 2) || structured;
    auto plane = [&](int l, int s) { return int64_t(((l + s) % d.k + d.k) % d.k) * nb; };
    ptr.assign(size_t(N) + 1, 0);
    col.clear();
    val.clear();
    std::vector<std::pair<int32_t, double>> row;
    for (int l = 0; l < d.k; ++l) {
        const int64_t off = int64_t(l) * nb;
        for (int64_t i = 0; i < nb; ++i) {
            row.clear();
            row.push_back({int32_t(off + i), h.diag[i]});
            for (int e = 0; e < h.W; ++e) {
                const int32_t j = h.ell_col[size_t(e) * nb + i];
                if (j == i) continue;  // padding
                row.push_back({int32_t(off + j), h.ell_val[size_t(e) * nb + i]});
                if (!h.ell_v1.empty())
                    for (int sgn : {1, -1}) row.push_back({int32_t(plane(l, sgn) + j), h.ell_v1[size_t(e) * nb + i]});
            }
            if (zf)
                for (int sgn : {1, -1}) row.push_back({int32_t(plane(l, sgn) + i), h.w[i]});
            if (!h.w2.empty())
                for (int sgn : {2, -2}) row.push_back({int32_t(plane(l, sgn) + i), h.w2[i]});
            std::sort(row.begin(), row.end(), [](auto &a, auto &b) { return a.first < b.first; });
            for (size_t e = 0; e < row.size(); ++e) {
                if (!col.empty() && int64_t(col.size()) > ptr[off + i] && col.back() == row[e].first)
                    val.back() += row[e].second;
                else {
                    col.push_back(row[e].first);
                    val.push_back(row[e].second);
                }
            }
            FVX_REQUIRE(col.size() < (size_t(1) << 31), FVX_E_ARG, "expanded matrix too large for int32 indices");
            ptr[off + i + 1] = int32_t(col.size());
        }
    }
}

}  // namespace fvx

using fvx::guard;

extern "C" {

int fvx_op_bytes(const fvx_mesh *m, const fvx_op_desc *d, size_t *bytes) {
    return guard([&] {
        fvx::check_desc(m, d);
        FVX_REQUIRE(bytes, FVX_E_ARG, "bytes is NULL");
        auto h = fvx::build_host(*m, *d);
        if (d->stencil != 13 && d->stencil != 27) fvx::build_cart(*m, h);
        *bytes = fvx::layout(h, d->with_f32 != 0).total;
        return FVX_OK;
    });
}

int fvx_op_create(const fvx_mesh *m, const fvx_op_desc *d, void *dev_mem, size_t bytes, void *stream,
                  fvx_op **out) {
    return guard([&] {
        fvx::check_desc(m, d);
        FVX_REQUIRE(out && dev_mem, FVX_E_ARG, "NULL output or device buffer");
        FVX_REQUIRE(reinterpret_cast<uintptr_t>(dev_mem) % 256 == 0, FVX_E_ARG,
                    "device buffer must be 256-byte aligned");
        const bool f32 = d->with_f32 != 0;
        auto h = fvx::build_host(*m, *d);
        if (d->stencil != 13 && d->stencil != 27) fvx::build_cart(*m, h);
        auto o = fvx::layout(h, f32);
        FVX_REQUIRE(bytes >= o.total, FVX_E_NOMEM,
                    "operator buffer too small: need " + std::to_string(o.total));
        hipStream_t s = fvx::as_stream(stream);
        char *base = static_cast<char *>(dev_mem);
        auto put = [&](size_t off, const void *src, size_t n) {
            if (n) FVX_HIP(hipMemcpyAsync(base + off, src, n, hipMemcpyHostToDevice, s));
        };
        const size_t nb = size_t(h.n_b), fb = size_t(h.F_b);
        put(o.ell_col, h.ell_col.data(), 4 * h.ell_col.size());
        put(o.cf_face, h.cf_face.data(), 4 * h.cf_face.size());
        put(o.f_c1, h.f_c1.data(), 4 * fb);
        put(o.f_c2, h.f_c2.data(), 4 * fb);
        put(o.diag[0], h.diag.data(), 8 * nb);
        put(o.ell_val[0], h.ell_val.data(), 8 * h.ell_val.size());
        put(o.w[0], h.w.data(), 8 * nb);
        put(o.cf_coef[0], h.cf_coef.data(), 8 * h.cf_coef.size());
        put(o.area[0], h.area.data(), 8 * nb);
        put(o.f_invd[0], h.f_invd.data(), 8 * fb);
        put(o.ell_v1[0], h.ell_v1.data(), 8 * h.ell_v1.size());
        put(o.w2[0], h.w2.data(), 8 * h.w2.size());
        std::vector<double> dinv(nb);
        std::vector<float> dinv32(nb);
        for (size_t i = 0; i < nb; ++i) {
            dinv[i] = h.diag[i] != 0.0 ? 1.0 / -h.diag[i] : 1.0;
            dinv32[i] = h.diag32[i] != 0.0f ? float(1.0 / -double(h.diag32[i])) : 1.0f;
        }
        put(o.dinv[0], dinv.data(), 8 * nb);
        put(o.cart[0], h.cart.data(), 8 * h.cart.size());
        put(o.srec[0], h.srec.data(), 8 * h.srec.size());
        for (auto pr : {std::make_pair(o.fnx[0], &h.fnx), std::make_pair(o.fny[0], &h.fny),
                        std::make_pair(o.gsx[0], &h.gsx), std::make_pair(o.gsy[0], &h.gsy),
                        std::make_pair(o.inv_area[0], &h.inv_area)})
            put(pr.first, pr.second->data(), 8 * pr.second->size());
        std::vector<float> nv32[5];
        std::vector<float> ev32, w32, cf32, ar32, fi32, v132, w232, cart32, srec32;
        if (f32) {
            cart32 = fvx::cast<float>(h.cart);
            for (size_t r = 0; r < cart32.size() / 8; ++r) cart32[r * 8] = h.diag32[r];  // the FP32 diagonal
            put(o.cart[1], cart32.data(), 4 * cart32.size());
            srec32 = fvx::cast<float>(h.srec);
            if (!h.srec.empty()) {
                const size_t wd = h.srec.size() / nb;
                for (size_t r = 0; r < nb; ++r) srec32[r * wd + 8] = h.diag32[r];  // the FP32 diagonal
            }
            put(o.srec[1], srec32.data(), 4 * srec32.size());
            v132 = fvx::cast<float>(h.ell_v1);
            w232 = fvx::cast<float>(h.w2);
            put(o.ell_v1[1], v132.data(), 4 * v132.size());
            put(o.w2[1], w232.data(), 4 * w232.size());
            ev32 = fvx::cast<float>(h.ell_val);
            w32 = fvx::cast<float>(h.w);
            cf32 = fvx::cast<float>(h.cf_coef);
            ar32 = fvx::cast<float>(h.area);
            fi32 = fvx::cast<float>(h.f_invd);
            put(o.diag[1], h.diag32.data(), 4 * nb);
            put(o.ell_val[1], ev32.data(), 4 * ev32.size());
            put(o.w[1], w32.data(), 4 * nb);
            put(o.cf_coef[1], cf32.data(), 4 * cf32.size());
            put(o.area[1], ar32.data(), 4 * nb);
            put(o.f_invd[1], fi32.data(), 4 * fb);
            put(o.dinv[1], dinv32.data(), 4 * nb);
            const std::vector<double> *src[5] = {&h.fnx, &h.fny, &h.gsx, &h.gsy, &h.inv_area};
            const size_t dst[5] = {o.fnx[1], o.fny[1], o.gsx[1], o.gsy[1], o.inv_area[1]};
            for (int q = 0; q < 5; ++q) {
                nv32[q] = fvx::cast<float>(*src[q]);
                put(dst[q], nv32[q].data(), 4 * nv32[q].size());
            }
        }
        FVX_HIP(hipStreamSynchronize(s));

        auto op = std::make_unique<fvx_op>();
        op->n_b = h.n_b;
        op->F_b = h.F_b;
        op->nnz_b = h.nnz_b;
        op->k = d->k;
        op->ld = fvx::ld_for_k(d->k);
        op->coupling = d->coupling;
        op->zfaces = d->coupling == FVX_COUPLING_PERIODIC_Z && d->k >= 2;
        op->singular = !(d->wall_bc == FVX_WALL_DIRICHLET && m->n_walls > 0);
        op->percol = d->coupling == FVX_COUPLING_NONE && d->k > 1;
        op->dz = d->dz;
        op->W = h.W;
        op->Wd = h.Wd;
        op->has_f32 = f32;
        op->grid_nx = m->grid_nx;
        op->grid_ny = m->grid_ny;
        op->stencil = (d->stencil == 13 || d->stencil == 27) ? d->stencil : 7;
        op->grid_px = m->periodic_x;
        op->grid_py = m->periodic_y;
        op->stencil_dir = op->stencil != 7 && h.sdir;
        FVX_HIP(hipGetDevice(&op->device));
        auto fill = [&](auto &D, int p, auto tag) {
            using T = decltype(tag);
            D.diag = reinterpret_cast<const T *>(base + o.diag[p]);
            D.ell_col = reinterpret_cast<const int32_t *>(base + o.ell_col);
            D.ell_val = reinterpret_cast<const T *>(base + o.ell_val[p]);
            D.w = reinterpret_cast<const T *>(base + o.w[p]);
            D.cf_face = reinterpret_cast<const int32_t *>(base + o.cf_face);
            D.cf_coef = reinterpret_cast<const T *>(base + o.cf_coef[p]);
            D.area = reinterpret_cast<const T *>(base + o.area[p]);
            D.f_c1 = reinterpret_cast<const int32_t *>(base + o.f_c1);
            D.f_c2 = reinterpret_cast<const int32_t *>(base + o.f_c2);
            D.f_invd = reinterpret_cast<const T *>(base + o.f_invd[p]);
            D.inv_dz = T(1.0 / d->dz);
            D.ell_v1 = h.ell_v1.empty() ? nullptr : reinterpret_cast<const T *>(base + o.ell_v1[p]);
            D.w2 = h.w2.empty() ? nullptr : reinterpret_cast<const T *>(base + o.w2[p]);
            D.srec = h.srec.empty() ? nullptr : reinterpret_cast<const T *>(base + o.srec[p]);
            D.dinv = reinterpret_cast<const T *>(base + o.dinv[p]);
            if (!h.cart.empty()) {
                D.cart = reinterpret_cast<const T *>(base + o.cart[p]);
                D.cart_nx = h.nx;
                D.cart_ny = h.ny;
                D.cart_px = h.px;
                D.cart_py = h.py;
            }
            if (!h.fnx.empty()) {
                D.fnx = reinterpret_cast<const T *>(base + o.fnx[p]);
                D.fny = reinterpret_cast<const T *>(base + o.fny[p]);
                D.gsx = reinterpret_cast<const T *>(base + o.gsx[p]);
                D.gsy = reinterpret_cast<const T *>(base + o.gsy[p]);
                D.inv_area = reinterpret_cast<const T *>(base + o.inv_area[p]);
            }
        };
        fill(op->d64, 0, double{});
        if (f32) fill(op->d32, 1, float{});
        op->tile[0] = fvx::default_tile(op.get(), FVX_F64);
        op->tile[1] = fvx::default_tile(op.get(), FVX_F32);
        *out = op.release();
        return FVX_OK;
    });
}

int fvx_op_destroy(fvx_op *op) {
    delete op;
    return FVX_OK;
}

int fvx_op_shape(const fvx_op *op, int64_t *n_b, int64_t *F_b, int32_t *k, int32_t *ld, int64_t *nnz_b) {
    return guard([&] {
        FVX_REQUIRE(op, FVX_E_ARG, "op is NULL");
        if (n_b) *n_b = op->n_b;
        if (F_b) *F_b = op->F_b;
        if (k) *k = op->k;
        if (ld) *ld = op->ld;
        if (nnz_b) *nnz_b = op->nnz_b;
        return FVX_OK;
    });
}

int fvx_op_singular(const fvx_op *op) { return op && op->singular ? 1 : 0; }

int fvx_op_get_tile(const fvx_op *op, int dtype, fvx_tile *tile) {
    return guard([&] {
        FVX_REQUIRE(op && tile, FVX_E_ARG, "NULL argument");
        FVX_REQUIRE(dtype == FVX_F64 || dtype == FVX_F32, FVX_E_ARG, "dtype must be F64 or F32");
        *tile = op->tile[dtype];
        return FVX_OK;
    });
}

int fvx_op_set_tile(fvx_op *op, int dtype, const fvx_tile *tile) {
    return guard([&] {
        FVX_REQUIRE(op && tile, FVX_E_ARG, "NULL argument");
        FVX_REQUIRE(dtype == FVX_F64 || dtype == FVX_F32, FVX_E_ARG, "dtype must be F64 or F32");
        fvx::check_tile(op, dtype, *tile);
        op->tile[dtype] = *tile;
        return FVX_OK;
    });
}

int fvx_expand_csr(const fvx_mesh *m, const fvx_op_desc *d, int64_t *nnz, int32_t *ptr, int32_t *col,
                   double *val) {
    return guard([&] {
        FVX_REQUIRE(m && d && nnz, FVX_E_ARG, "NULL argument");
        std::vector<int32_t> p, c;
        std::vector<double> v;
        fvx::expand_csr(*m, *d, p, c, v);
        *nnz = int64_t(c.size());
        if (ptr) std::memcpy(ptr, p.data(), sizeof(int32_t) * p.size());
        if (col) std::memcpy(col, c.data(), sizeof(int32_t) * c.size());
        if (val) std::memcpy(val, v.data(), sizeof(double) * v.size());
        return FVX_OK;
    });
}

}  // extern "C"
