// Base meshes: 2D finite-volume face graphs (host side), plus the library's
// error handling.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <utility>
#include <vector>

#include "common.h"

namespace fvx {

static thread_local std::string g_last_error;

void set_last_error(const std::string &s) { g_last_error = s; }

int guard(const std::function<int()> &f) {
    try {
        int rc = f();
        if (rc >= 0) g_last_error.clear();
        return rc;
    } catch (const Error &e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return FVX_E_NOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return FVX_E_ARG;
    } catch (...) {
        g_last_error = "unknown error";
        return FVX_E_ARG;
    }
}

static void validate(const fvx_mesh &m) {
    FVX_REQUIRE(m.n_cells >= 1, FVX_E_MESH, "mesh has no cells");
    for (int c = 0; c < m.n_cells; ++c)
        FVX_REQUIRE(m.area[c] > 0.0 && std::isfinite(m.area[c]), FVX_E_MESH,
                    "cell " + std::to_string(c) + " has non-positive area");
    for (int f = 0; f < m.n_faces; ++f) {
        FVX_REQUIRE(m.c1[f] >= 0 && m.c1[f] < m.n_cells && m.c2[f] >= 0 && m.c2[f] < m.n_cells,
                    FVX_E_MESH, "face " + std::to_string(f) + " cell index out of range");
        FVX_REQUIRE(m.len[f] > 0.0 && m.dist[f] > 0.0 && std::isfinite(m.len[f]) &&
                        std::isfinite(m.dist[f]),
                    FVX_E_MESH, "face " + std::to_string(f) + " has non-positive length or distance");
    }
    for (int w = 0; w < m.n_walls; ++w) {
        FVX_REQUIRE(m.wcell[w] >= 0 && m.wcell[w] < m.n_cells, FVX_E_MESH,
                    "wall " + std::to_string(w) + " cell index out of range");
        FVX_REQUIRE(m.wlen[w] > 0.0 && m.wdist[w] > 0.0, FVX_E_MESH,
                    "wall " + std::to_string(w) + " has non-positive length or distance");
    }
}

}  // namespace fvx

using fvx::Error;
using fvx::guard;

extern "C" {

const char *fvx_status_str(int s) {
    switch (s) {
        case FVX_OK: return "ok";
        case FVX_NOT_CONVERGED: return "not converged";
        case FVX_E_ARG: return "invalid argument";
        case FVX_E_MESH: return "invalid mesh";
        case FVX_E_NOMEM: return "buffer too small";
        case FVX_E_HIP: return "HIP runtime error";
        case FVX_E_BREAKDOWN: return "CG breakdown";
        case FVX_E_NONFINITE: return "non-finite input";
        case FVX_E_UNSUPPORTED: return "unsupported";
        case FVX_E_IO: return "file input/output error";
        default: return "unknown status";
    }
}

const char *fvx_last_error(void) { return fvx::g_last_error.c_str(); }

int fvx_version(void) { return 10000; }

}  // extern "C"

namespace {

// Cartesian face graph from the face coordinates of both axes: cell (i, j) is
// j * nx + i; x-faces first, then y-faces; walls where an axis is not
// periodic.
fvx_mesh *cartesian_from_faces(const std::vector<double> &xf, const std::vector<double> &yf, int periodic_x,
                               int periodic_y) {
    const int nx = int(xf.size()) - 1, ny = int(yf.size()) - 1;
    auto m = new fvx_mesh();
    {
        const int nc = nx * ny;
        m->n_cells = nc;
        m->grid_nx = nx;
        m->grid_ny = ny;
        m->xf = xf;
        m->yf = yf;
        m->periodic_x = periodic_x != 0;
        m->periodic_y = periodic_y != 0;
        m->area.resize(nc);
        m->cx.resize(nc);
        m->cy.resize(nc);
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int c = j * nx + i;
                m->area[c] = (xf[i + 1] - xf[i]) * (yf[j + 1] - yf[j]);
                m->cx[c] = 0.5 * (xf[i] + xf[i + 1]);
                m->cy[c] = 0.5 * (yf[j] + yf[j + 1]);
            }
        auto add_face = [&](int a, int b, double l, double d, double nxv, double nyv) {
            m->c1.push_back(a);
            m->c2.push_back(b);
            m->len.push_back(l);
            m->dist.push_back(d);
            m->fnx.push_back(nxv);
            m->fny.push_back(nyv);
        };
        auto half = [](const std::vector<double> &f, int i) { return 0.5 * (f[i + 1] - f[i]); };
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                if (i == nx - 1 && !periodic_x) continue;
                const int ip = (i + 1) % nx;
                add_face(j * nx + i, j * nx + ip, yf[j + 1] - yf[j], half(xf, i) + half(xf, ip), 1.0, 0.0);
            }
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                if (j == ny - 1 && !periodic_y) continue;
                const int jp = (j + 1) % ny;
                add_face(j * nx + i, jp * nx + i, xf[i + 1] - xf[i], half(yf, j) + half(yf, jp), 0.0, 1.0);
            }
        m->n_faces = int(m->c1.size());
        auto add_wall = [&](int c, double l, double d) {
            m->wcell.push_back(c);
            m->wlen.push_back(l);
            m->wdist.push_back(d);
        };
        if (!periodic_x)
            for (int j = 0; j < ny; ++j) {
                add_wall(j * nx, yf[j + 1] - yf[j], half(xf, 0));
                add_wall(j * nx + nx - 1, yf[j + 1] - yf[j], half(xf, nx - 1));
            }
        if (!periodic_y)
            for (int i = 0; i < nx; ++i) {
                add_wall(i, xf[i + 1] - xf[i], half(yf, 0));
                add_wall((ny - 1) * nx + i, xf[i + 1] - xf[i], half(yf, ny - 1));
            }
        m->n_walls = int(m->wcell.size());
    }
    return m;
}

// Centres of an axis and the coarse-centre interpolation of a point x:
// (index, weight) pairs.  Between two centres: linear weights; past the first
// or last centre of a wall-bounded axis: the end centre with weight 1; a
// periodic axis wraps across the period.
void axis_weights(const std::vector<double> &f, bool periodic, double x, std::vector<std::pair<int, double>> &out) {
    const int n = int(f.size()) - 1;
    out.clear();
    std::vector<double> c(n);
    for (int i = 0; i < n; ++i) c[i] = 0.5 * (f[i] + f[i + 1]);
    if (n == 1) {
        out.push_back({0, 1.0});
        return;
    }
    const int hi = int(std::upper_bound(c.begin(), c.end(), x) - c.begin());  // first centre > x
    if (hi > 0 && hi < n) {
        const double t = (x - c[hi - 1]) / (c[hi] - c[hi - 1]);
        out.push_back({hi - 1, 1.0 - t});
        out.push_back({hi, t});
        return;
    }
    if (!periodic) {
        out.push_back({hi == 0 ? 0 : n - 1, 1.0});
        return;
    }
    const double period = f[n] - f[0];
    const double left = c[n - 1] - period, right = c[0] + period;  // images across the period
    if (hi == 0) {
        const double t = (x - left) / (c[0] - left);
        out.push_back({n - 1, 1.0 - t});
        out.push_back({0, t});
    } else {
        const double t = (x - c[n - 1]) / (right - c[n - 1]);
        out.push_back({n - 1, 1.0 - t});
        out.push_back({0, t});
    }
}

}  // namespace

extern "C" {

int fvx_mesh_cartesian(int nx, int ny, double x0, double Lx, double y0, double y1, double stretch,
                       int periodic_x, int periodic_y, fvx_mesh **out) {
    return guard([&] {
        FVX_REQUIRE(out, FVX_E_ARG, "out is NULL");
        FVX_REQUIRE(nx >= 1 && ny >= 1, FVX_E_ARG, "nx and ny must be >= 1");
        FVX_REQUIRE(Lx > 0 && y1 > y0 && std::isfinite(stretch) && stretch >= 0, FVX_E_ARG,
                    "empty extent or bad stretch");
        std::vector<double> xf(nx + 1), yf(ny + 1);
        for (int i = 0; i <= nx; ++i) xf[i] = x0 + Lx * double(i) / double(nx);
        for (int j = 0; j <= ny; ++j) {
            double t = double(j) / double(ny);
            yf[j] = stretch == 0.0
                        ? y0 + (y1 - y0) * t
                        : y0 + (y1 - y0) * 0.5 * (1.0 + std::tanh(stretch * (2.0 * t - 1.0)) / std::tanh(stretch));
        }
        *out = cartesian_from_faces(xf, yf, periodic_x, periodic_y);
        return FVX_OK;
    });
}

int fvx_mesh_refine(const fvx_mesh *coarse, int rf, fvx_mesh **fine) {
    return guard([&] {
        FVX_REQUIRE(coarse && fine, FVX_E_ARG, "NULL argument");
        FVX_REQUIRE(coarse->grid_nx > 0, FVX_E_UNSUPPORTED, "refinement needs a Cartesian base mesh");
        FVX_REQUIRE(rf >= 1 && rf <= 16, FVX_E_ARG, "rf must be in 1..16");
        auto split = [&](const std::vector<double> &f) {
            std::vector<double> g;
            for (size_t i = 0; i + 1 < f.size(); ++i)
                for (int a = 0; a < rf; ++a) g.push_back(f[i] + (f[i + 1] - f[i]) * double(a) / double(rf));
            g.push_back(f.back());
            return g;
        };
        *fine = cartesian_from_faces(split(coarse->xf), split(coarse->yf), coarse->periodic_x, coarse->periodic_y);
        return FVX_OK;
    });
}

int fvx_refine_prolongation(const fvx_mesh *coarse, int rf, int64_t *nnz, int32_t *ptr, int32_t *col,
                            double *val) {
    return guard([&] {
        FVX_REQUIRE(coarse && nnz, FVX_E_ARG, "NULL argument");
        FVX_REQUIRE(coarse->grid_nx > 0, FVX_E_UNSUPPORTED, "refinement needs a Cartesian base mesh");
        FVX_REQUIRE(rf >= 1 && rf <= 16, FVX_E_ARG, "rf must be in 1..16");
        const int nx = coarse->grid_nx, ny = coarse->grid_ny, NX = nx * rf, NY = ny * rf;
        std::vector<std::pair<int, double>> wx, wy;
        std::vector<std::map<int32_t, double>> rows(size_t(NX) * NY);
        for (int J = 0; J < NY; ++J) {
            const int j = J / rf, b = J % rf;
            const double hy = coarse->yf[j + 1] - coarse->yf[j];
            axis_weights(coarse->yf, coarse->periodic_y, coarse->yf[j] + hy * (b + 0.5) / rf, wy);
            for (int I = 0; I < NX; ++I) {
                const int i = I / rf, a = I % rf;
                const double hx = coarse->xf[i + 1] - coarse->xf[i];
                axis_weights(coarse->xf, coarse->periodic_x, coarse->xf[i] + hx * (a + 0.5) / rf, wx);
                auto &row = rows[size_t(J) * NX + I];
                for (const auto &py : wy)
                    for (const auto &px : wx) row[py.first * nx + px.first] += py.second * px.second;
            }
        }
        int64_t total = 0;
        for (const auto &r : rows) total += int64_t(r.size());
        *nnz = total;
        if (!ptr && !col && !val) return FVX_OK;
        FVX_REQUIRE(ptr && col && val, FVX_E_ARG, "ptr, col and val must all be given");
        int64_t e = 0;
        ptr[0] = 0;
        for (size_t r = 0; r < rows.size(); ++r) {
            for (const auto &kv : rows[r]) {
                col[e] = kv.first;
                val[e] = kv.second;
                ++e;
            }
            ptr[r + 1] = int32_t(e);
        }
        return FVX_OK;
    });
}

int fvx_mesh_triangles(int n_pts, const double *xy, int n_tri, const int32_t *tri, fvx_mesh **out) {
    return guard([&] {
        FVX_REQUIRE(out && xy && tri, FVX_E_ARG, "NULL argument");
        FVX_REQUIRE(n_pts >= 3 && n_tri >= 1, FVX_E_ARG, "need >= 3 points and >= 1 triangle");
        auto m = std::make_unique<fvx_mesh>();
        m->n_cells = n_tri;
        m->area.resize(n_tri);
        m->cx.resize(n_tri);
        m->cy.resize(n_tri);
        for (int t = 0; t < n_tri; ++t) {
            for (int s = 0; s < 3; ++s)
                FVX_REQUIRE(tri[3 * t + s] >= 0 && tri[3 * t + s] < n_pts, FVX_E_MESH,
                            "triangle " + std::to_string(t) + " vertex out of range");
            const double *a = xy + 2 * tri[3 * t], *b = xy + 2 * tri[3 * t + 1], *c = xy + 2 * tri[3 * t + 2];
            const double cr = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
            m->area[t] = 0.5 * std::fabs(cr);
            FVX_REQUIRE(m->area[t] > 0.0, FVX_E_MESH, "degenerate triangle " + std::to_string(t));
            m->cx[t] = (a[0] + b[0] + c[0]) / 3.0;
            m->cy[t] = (a[1] + b[1] + c[1]) / 3.0;
        }
        // Edge key (lo, hi, triangle); sorting groups the two sides of a face.
        std::vector<std::tuple<int, int, int>> e;
        e.reserve(size_t(3) * n_tri);
        for (int t = 0; t < n_tri; ++t)
            for (int s = 0; s < 3; ++s) {
                int u = tri[3 * t + s], v = tri[3 * t + (s + 1) % 3];
                FVX_REQUIRE(u != v, FVX_E_MESH, "repeated vertex in triangle " + std::to_string(t));
                e.emplace_back(std::min(u, v), std::max(u, v), t);
            }
        std::sort(e.begin(), e.end());
        for (size_t i = 0; i < e.size();) {
            size_t j = i;
            while (j < e.size() && std::get<0>(e[j]) == std::get<0>(e[i]) &&
                   std::get<1>(e[j]) == std::get<1>(e[i]))
                ++j;
            FVX_REQUIRE(j - i <= 2, FVX_E_MESH, "edge shared by more than two triangles");
            const double *pa = xy + 2 * std::get<0>(e[i]), *pb = xy + 2 * std::get<1>(e[i]);
            const double tx = pb[0] - pa[0], ty = pb[1] - pa[1];
            const double l = std::sqrt(tx * tx + ty * ty);
            const double nxv = ty / l, nyv = -tx / l;
            const int ta = std::get<2>(e[i]);
            if (j - i == 2) {
                const int tb = std::get<2>(e[i + 1]);
                const double dn = nxv * (m->cx[tb] - m->cx[ta]) + nyv * (m->cy[tb] - m->cy[ta]);
                const double d = std::fabs(dn);
                FVX_REQUIRE(d > 0.0, FVX_E_MESH, "zero centroid distance across a face");
                m->c1.push_back(ta);
                m->c2.push_back(tb);
                m->len.push_back(l);
                m->dist.push_back(d);
                m->fnx.push_back(dn > 0 ? nxv : -nxv);  // oriented from ta to tb
                m->fny.push_back(dn > 0 ? nyv : -nyv);
            } else {
                m->wcell.push_back(ta);
                m->wlen.push_back(l);
                m->wdist.push_back(std::fabs(nxv * (m->cx[ta] - pa[0]) + nyv * (m->cy[ta] - pa[1])));
            }
            i = j;
        }
        m->n_faces = int(m->c1.size());
        m->n_walls = int(m->wcell.size());
        *out = m.release();
        return FVX_OK;
    });
}

int fvx_mesh_from_faces(int n_cells, const double *area, const double *cx, const double *cy,
                        int n_faces, const int32_t *c1, const int32_t *c2, const double *len,
                        const double *dist, int n_walls, const int32_t *wcell, const double *wlen,
                        const double *wdist, fvx_mesh **out) {
    return guard([&] {
        FVX_REQUIRE(out && area, FVX_E_ARG, "NULL argument");
        FVX_REQUIRE(n_cells >= 1 && n_faces >= 0 && n_walls >= 0, FVX_E_ARG, "bad sizes");
        FVX_REQUIRE(n_faces == 0 || (c1 && c2 && len && dist), FVX_E_ARG, "NULL face array");
        FVX_REQUIRE(n_walls == 0 || (wcell && wlen && wdist), FVX_E_ARG, "NULL wall array");
        auto m = std::make_unique<fvx_mesh>();
        m->n_cells = n_cells;
        m->n_faces = n_faces;
        m->n_walls = n_walls;
        m->area.assign(area, area + n_cells);
        m->cx = cx ? std::vector<double>(cx, cx + n_cells) : std::vector<double>(n_cells, 0.0);
        m->cy = cy ? std::vector<double>(cy, cy + n_cells) : std::vector<double>(n_cells, 0.0);
        if (n_faces) {
            m->c1.assign(c1, c1 + n_faces);
            m->c2.assign(c2, c2 + n_faces);
            m->len.assign(len, len + n_faces);
            m->dist.assign(dist, dist + n_faces);
        }
        if (n_walls) {
            m->wcell.assign(wcell, wcell + n_walls);
            m->wlen.assign(wlen, wlen + n_walls);
            m->wdist.assign(wdist, wdist + n_walls);
        }
        fvx::validate(*m);
        *out = m.release();
        return FVX_OK;
    });
}

namespace {

// Distance along the Hilbert curve that fills the 2^bits x 2^bits grid, of
// grid point (x, y): per level from the coarsest, the quadrant contributes
// s^2 times its digit (3 rx) xor ry along the curve, then the point is
// reflected and transposed into the sub-square's standard orientation.
uint64_t hilbert_distance(uint32_t x, uint32_t y, int bits) {
    const uint32_t n = 1u << bits;
    uint64_t d = 0;
    for (uint32_t s = n >> 1; s > 0; s >>= 1) {
        const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
        d += uint64_t(s) * s * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = n - 1 - x;
                y = n - 1 - y;
            }
            std::swap(x, y);
        }
    }
    return d;
}

}  // namespace

int fvx_hilbert_order(int64_t n, const double *x, const double *y, int32_t *perm) {
    return guard([&] {
        FVX_REQUIRE(n >= 0 && n <= INT32_MAX, FVX_E_ARG, "n out of range");
        if (n == 0) return FVX_OK;
        FVX_REQUIRE(x && y && perm, FVX_E_ARG, "NULL argument");
        double lo[2] = {x[0], y[0]}, hi[2] = {x[0], y[0]};
        for (int64_t i = 0; i < n; ++i) {
            FVX_REQUIRE(std::isfinite(x[i]) && std::isfinite(y[i]), FVX_E_ARG, "non-finite coordinate");
            lo[0] = std::min(lo[0], x[i]);
            hi[0] = std::max(hi[0], x[i]);
            lo[1] = std::min(lo[1], y[i]);
            hi[1] = std::max(hi[1], y[i]);
        }
        constexpr int kBits = 16;
        constexpr double kTop = double((1u << kBits) - 1);
        auto grid = [&](double v, int a) -> uint32_t {
            const double w = hi[a] - lo[a];
            if (!(w > 0.0)) return 0;
            const double g = std::floor((v - lo[a]) / w * kTop);
            return uint32_t(std::min(std::max(g, 0.0), kTop));
        };
        std::vector<std::pair<uint64_t, int32_t>> key(static_cast<size_t>(n));
        for (int64_t i = 0; i < n; ++i) key[size_t(i)] = {hilbert_distance(grid(x[i], 0), grid(y[i], 1), kBits), int32_t(i)};
        std::sort(key.begin(), key.end());  // ties: ascending index
        for (int64_t i = 0; i < n; ++i) perm[i] = key[size_t(i)].second;
        return FVX_OK;
    });
}

int fvx_mesh_info(const fvx_mesh *m, int64_t *n_cells, int64_t *n_faces, int64_t *n_walls) {
    return guard([&] {
        FVX_REQUIRE(m, FVX_E_ARG, "mesh is NULL");
        if (n_cells) *n_cells = m->n_cells;
        if (n_faces) *n_faces = m->n_faces;
        if (n_walls) *n_walls = m->n_walls;
        return FVX_OK;
    });
}

int fvx_mesh_centroids(const fvx_mesh *m, double *cx, double *cy) {
    return guard([&] {
        FVX_REQUIRE(m, FVX_E_ARG, "mesh is NULL");
        if (cx) std::memcpy(cx, m->cx.data(), sizeof(double) * m->n_cells);
        if (cy) std::memcpy(cy, m->cy.data(), sizeof(double) * m->n_cells);
        return FVX_OK;
    });
}

int fvx_mesh_faces(const fvx_mesh *m, double *area, int32_t *c1, int32_t *c2, double *len,
                   double *dist) {
    return guard([&] {
        FVX_REQUIRE(m, FVX_E_ARG, "mesh is NULL");
        if (area) std::memcpy(area, m->area.data(), sizeof(double) * m->n_cells);
        if (c1 && m->n_faces) std::memcpy(c1, m->c1.data(), sizeof(int32_t) * m->n_faces);
        if (c2 && m->n_faces) std::memcpy(c2, m->c2.data(), sizeof(int32_t) * m->n_faces);
        if (len && m->n_faces) std::memcpy(len, m->len.data(), sizeof(double) * m->n_faces);
        if (dist && m->n_faces) std::memcpy(dist, m->dist.data(), sizeof(double) * m->n_faces);
        return FVX_OK;
    });
}

int fvx_mesh_destroy(fvx_mesh *m) {
    delete m;
    return FVX_OK;
}

}  // extern "C"
