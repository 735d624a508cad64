/*
 * Plain CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * What it follows:
 *  - The staggered symmetry-preserving finite-volume operators of Section 3
 *    (Eq. 9): the integrated divergence M (cells x faces), the face volumes
 *    Omega_s, the gradient G = -Omega_s^{-1} M^T, and the Laplacian L = M G.
 *  - The repeated-block structure of Section 2 (Eq. 1) and Section 3.1
 *    (Eq. 10) is deliberately NOT used: every 3D face of the extruded mesh is
 *    visited and assembled on its own, including the periodic faces between
 *    planes, so the matrices here are the plain assembled ones.
 *  - SpMV is the textbook CSR row loop; CG is the textbook Hestenes-Stiefel
 *    loop on the SPD matrix -L.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ERR_ARG (-1)
#define ERR_MESH (-2)
#define ERR_NOMEM (-3)

/* ====================================================================== */
/* Base geometry                                                          */
/* ====================================================================== */

int orc_cart_sizes(int nx, int ny, int periodic_x, int periodic_y,
                   int *n_cells, int *n_faces, int *n_walls)
{
    if (nx < 1 || ny < 1) return ERR_ARG;
    int fx = periodic_x ? nx * ny : (nx - 1) * ny;
    int fy = periodic_y ? nx * ny : nx * (ny - 1);
    *n_cells = nx * ny;
    *n_faces = fx + fy;
    *n_walls = (periodic_x ? 0 : 2 * ny) + (periodic_y ? 0 : 2 * nx);
    return 0;
}

/* Face coordinate j of the wall-clustered direction. */
static double stretched(int j, int n, double a, double b, double s)
{
    double t = (double)j / (double)n;
    if (s == 0.0) return a + (b - a) * t;
    return a + (b - a) * 0.5 * (1.0 + tanh(s * (2.0 * t - 1.0)) / tanh(s));
}

int orc_cart_geometry(int nx, int ny, double x0, double Lx, double y0, double y1,
                      double stretch, int periodic_x, int periodic_y,
                      double *area, double *cx, double *cy,
                      int *c1, int *c2, double *len, double *dist,
                      int *wcell, double *wlen, double *wdist)
{
    if (nx < 1 || ny < 1 || !(Lx > 0.0) || !(y1 > y0)) return ERR_ARG;
    double *xf = malloc(sizeof(double) * (nx + 1));
    double *yf = malloc(sizeof(double) * (ny + 1));
    if (!xf || !yf) { free(xf); free(yf); return ERR_NOMEM; }
    for (int i = 0; i <= nx; ++i) xf[i] = x0 + Lx * (double)i / (double)nx;
    for (int j = 0; j <= ny; ++j) yf[j] = stretched(j, ny, y0, y1, stretch);

    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int c = j * nx + i;
            area[c] = (xf[i + 1] - xf[i]) * (yf[j + 1] - yf[j]);
            cx[c] = 0.5 * (xf[i] + xf[i + 1]);
            cy[c] = 0.5 * (yf[j] + yf[j + 1]);
        }

    int f = 0;
    /* faces normal to x: between (i, j) and (i+1, j) */
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (i == nx - 1 && !periodic_x) continue;
            int ip = (i + 1) % nx;
            c1[f] = j * nx + i;
            c2[f] = j * nx + ip;
            len[f] = yf[j + 1] - yf[j];
            if (i == nx - 1) /* wrap: half cell on each side of the period */
                dist[f] = 0.5 * (xf[nx] - xf[nx - 1]) + 0.5 * (xf[1] - xf[0]);
            else
                dist[f] = 0.5 * (xf[i + 2] - xf[i]);
            ++f;
        }
    /* faces normal to y: between (i, j) and (i, j+1) */
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (j == ny - 1 && !periodic_y) continue;
            int jp = (j + 1) % ny;
            c1[f] = j * nx + i;
            c2[f] = jp * nx + i;
            len[f] = xf[i + 1] - xf[i];
            if (j == ny - 1)
                dist[f] = 0.5 * (yf[ny] - yf[ny - 1]) + 0.5 * (yf[1] - yf[0]);
            else
                dist[f] = 0.5 * (yf[j + 2] - yf[j]);
            ++f;
        }
    int w = 0;
    if (!periodic_x)
        for (int j = 0; j < ny; ++j) {
            int ends[2] = {0, nx - 1};
            for (int e = 0; e < 2; ++e) {
                int i = ends[e];
                wcell[w] = j * nx + i;
                wlen[w] = yf[j + 1] - yf[j];
                wdist[w] = 0.5 * (xf[i + 1] - xf[i]);
                ++w;
            }
        }
    if (!periodic_y)
        for (int i = 0; i < nx; ++i) {
            int ends[2] = {0, ny - 1};
            for (int e = 0; e < 2; ++e) {
                int j = ends[e];
                wcell[w] = j * nx + i;
                wlen[w] = xf[i + 1] - xf[i];
                wdist[w] = 0.5 * (yf[j + 1] - yf[j]);
                ++w;
            }
        }
    free(xf);
    free(yf);
    return 0;
}

/* Triangle edges in canonical order: sorted by (lower vertex, higher vertex,
 * triangle).  An edge seen twice is an interior face whose c1 is the lower
 * triangle index; an edge seen once is a wall. */
typedef struct { int a, b, t; } edge_rec;

static int edge_cmp(const void *p, const void *q)
{
    const edge_rec *x = p, *y = q;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    if (x->t != y->t) return x->t < y->t ? -1 : 1;
    return 0;
}

static edge_rec *sorted_edges(int n_pts, int n_tri, const int *tri, int *err)
{
    edge_rec *e = malloc(sizeof(edge_rec) * 3 * (size_t)n_tri);
    if (!e) { *err = ERR_NOMEM; return NULL; }
    for (int t = 0; t < n_tri; ++t)
        for (int s = 0; s < 3; ++s) {
            int u = tri[3 * t + s], v = tri[3 * t + (s + 1) % 3];
            if (u < 0 || v < 0 || u >= n_pts || v >= n_pts || u == v) {
                free(e);
                *err = ERR_MESH;
                return NULL;
            }
            e[3 * t + s].a = u < v ? u : v;
            e[3 * t + s].b = u < v ? v : u;
            e[3 * t + s].t = t;
        }
    qsort(e, 3 * (size_t)n_tri, sizeof(edge_rec), edge_cmp);
    *err = 0;
    return e;
}

int orc_tri_sizes(int n_pts, const double *xy, int n_tri, const int *tri,
                  int *n_faces, int *n_walls)
{
    (void)xy;
    if (n_pts < 3 || n_tri < 1) return ERR_ARG;
    int err;
    edge_rec *e = sorted_edges(n_pts, n_tri, tri, &err);
    if (!e) return err;
    int nf = 0, nw = 0;
    size_t m = 3 * (size_t)n_tri;
    for (size_t i = 0; i < m;) {
        size_t j = i;
        while (j < m && e[j].a == e[i].a && e[j].b == e[i].b) ++j;
        if (j - i == 1) ++nw;
        else if (j - i == 2) ++nf;
        else { free(e); return ERR_MESH; }
        i = j;
    }
    free(e);
    *n_faces = nf;
    *n_walls = nw;
    return 0;
}

int orc_tri_geometry(int n_pts, const double *xy, int n_tri, const int *tri,
                     double *area, double *cx, double *cy,
                     int *c1, int *c2, double *len, double *dist,
                     int *wcell, double *wlen, double *wdist)
{
    if (n_pts < 3 || n_tri < 1) return ERR_ARG;
    for (int t = 0; t < n_tri; ++t) {
        const double *p0 = xy + 2 * tri[3 * t], *p1 = xy + 2 * tri[3 * t + 1],
                     *p2 = xy + 2 * tri[3 * t + 2];
        double cr = (p1[0] - p0[0]) * (p2[1] - p0[1]) - (p1[1] - p0[1]) * (p2[0] - p0[0]);
        area[t] = 0.5 * fabs(cr);
        if (!(area[t] > 0.0)) return ERR_MESH;
        cx[t] = (p0[0] + p1[0] + p2[0]) / 3.0;
        cy[t] = (p0[1] + p1[1] + p2[1]) / 3.0;
    }
    int err;
    edge_rec *e = sorted_edges(n_pts, n_tri, tri, &err);
    if (!e) return err;
    int nf = 0, nw = 0;
    size_t m = 3 * (size_t)n_tri;
    for (size_t i = 0; i < m;) {
        size_t j = i;
        while (j < m && e[j].a == e[i].a && e[j].b == e[i].b) ++j;
        const double *pa = xy + 2 * e[i].a, *pb = xy + 2 * e[i].b;
        double tx = pb[0] - pa[0], ty = pb[1] - pa[1];
        double l = sqrt(tx * tx + ty * ty);
        double nx = ty / l, ny = -tx / l; /* unit normal of the edge line */
        if (j - i == 2) {
            int ta = e[i].t, tb = e[i + 1].t; /* sorted: ta < tb */
            c1[nf] = ta;
            c2[nf] = tb;
            len[nf] = l;
            dist[nf] = fabs(nx * (cx[tb] - cx[ta]) + ny * (cy[tb] - cy[ta]));
            if (!(dist[nf] > 0.0)) { free(e); return ERR_MESH; }
            ++nf;
        } else if (j - i == 1) {
            int ta = e[i].t;
            wcell[nw] = ta;
            wlen[nw] = l;
            wdist[nw] = fabs(nx * (cx[ta] - pa[0]) + ny * (cy[ta] - pa[1]));
            ++nw;
        } else {
            free(e);
            return ERR_MESH;
        }
        i = j;
    }
    free(e);
    return 0;
}

/* ====================================================================== */
/* 3D assembly                                                            */
/* ====================================================================== */

static int has_zfaces(const orc_mesh3d *m) { return m->coupling == 1 && m->k >= 2; }

int64_t orc_n_faces3d(const orc_mesh3d *m)
{
    int64_t n = (int64_t)m->k * m->n_faces;
    if (has_zfaces(m)) n += (int64_t)m->k * m->n_cells;
    return n;
}

/* One 3D face: its two cells (c2 < 0: wall), its area and its centre-to-centre
 * (or centre-to-wall) distance.  Every face of the extruded mesh is produced
 * by this routine from the base geometry and the plane spacing. */
typedef struct { int64_t c1, c2; double area, dist; } face3d;

static face3d get_face(const orc_mesh3d *m, int64_t f3)
{
    face3d F;
    int64_t nb = m->n_cells, fb = m->n_faces;
    if (f3 < (int64_t)m->k * fb) {
        int64_t l = f3 / fb, f = f3 % fb;
        F.c1 = l * nb + m->c1[f];
        F.c2 = l * nb + m->c2[f];
        F.area = m->len[f] * m->dz;
        F.dist = m->dist[f];
    } else {
        int64_t z = f3 - (int64_t)m->k * fb;
        int64_t l = z / nb, c = z % nb;
        F.c1 = l * nb + c;
        F.c2 = ((l + 1) % m->k) * nb + c;
        F.area = m->area[c];
        F.dist = m->dz;
    }
    return F;
}

typedef struct { int64_t r; int32_t c; double v; } trip;

static int trip_cmp(const void *p, const void *q)
{
    const trip *x = p, *y = q;
    if (x->r != y->r) return x->r < y->r ? -1 : 1;
    if (x->c != y->c) return x->c < y->c ? -1 : 1;
    return 0;
}

/* Sort triplets by (row, column) -- stable order of insertion is kept for
 * equal keys by tagging -- and sum duplicates into CSR. */
typedef struct { trip t; int64_t order; } trip_o;

static int trip_o_cmp(const void *p, const void *q)
{
    const trip_o *x = p, *y = q;
    int c = trip_cmp(&x->t, &y->t);
    if (c) return c;
    return x->order < y->order ? -1 : (x->order > y->order);
}

static int to_csr(trip_o *T, int64_t nt, int64_t n_rows, int64_t *ptr, int32_t *col,
                  double *val, int64_t *nnz)
{
    qsort(T, (size_t)nt, sizeof(trip_o), trip_o_cmp);
    int64_t k = 0;
    for (int64_t r = 0; r <= n_rows; ++r) ptr[r] = 0;
    for (int64_t i = 0; i < nt;) {
        int64_t j = i;
        double s = 0.0;
        while (j < nt && T[j].t.r == T[i].t.r && T[j].t.c == T[i].t.c) {
            s += T[j].t.v;
            ++j;
        }
        col[k] = T[i].t.c;
        val[k] = s;
        ptr[T[i].t.r + 1]++;
        ++k;
        i = j;
    }
    for (int64_t r = 0; r < n_rows; ++r) ptr[r + 1] += ptr[r];
    *nnz = k;
    return 0;
}

static int check_mesh(const orc_mesh3d *m)
{
    if (m->k < 1 || !(m->dz > 0.0) || m->n_cells < 1 || m->n_faces < 0) return ERR_ARG;
    if (m->coupling != 0 && m->coupling != 1) return ERR_ARG;
    for (int f = 0; f < m->n_faces; ++f) {
        if (m->c1[f] < 0 || m->c1[f] >= m->n_cells || m->c2[f] < 0 || m->c2[f] >= m->n_cells)
            return ERR_MESH;
        if (!(m->len[f] > 0.0) || !(m->dist[f] > 0.0)) return ERR_MESH;
    }
    for (int c = 0; c < m->n_cells; ++c)
        if (!(m->area[c] > 0.0)) return ERR_MESH;
    if (m->dirichlet)
        for (int w = 0; w < m->n_walls; ++w) {
            if (m->wcell[w] < 0 || m->wcell[w] >= m->n_cells) return ERR_MESH;
            if (!(m->wlen[w] > 0.0) || !(m->wdist[w] > 0.0)) return ERR_MESH;
        }
    return 0;
}

int64_t orc_lap_max_nnz(const orc_mesh3d *m)
{
    int64_t n3 = (int64_t)m->k * m->n_cells;
    return n3 + 2 * orc_n_faces3d(m);
}

/* L = M G = -M Omega_s^{-1} M^T, assembled face by face: a face of area a and
 * distance d adds -a/d to both diagonals and +a/d to both off-diagonals.
 * Dirichlet walls add -a_w/d_w to the wall cell's diagonal (p = 0 at the wall,
 * d_w = distance from the cell centre to the wall). */
int orc_assemble_lap(const orc_mesh3d *m, int64_t *ptr, int32_t *col, double *val, int64_t *nnz)
{
    int e = check_mesh(m);
    if (e) return e;
    int64_t n3 = (int64_t)m->k * m->n_cells, f3 = orc_n_faces3d(m);
    int64_t nw3 = m->dirichlet ? (int64_t)m->k * m->n_walls : 0;
    int64_t nt = 4 * f3 + nw3 + n3;
    trip_o *T = malloc(sizeof(trip_o) * (size_t)(nt > 0 ? nt : 1));
    if (!T) return ERR_NOMEM;
    int64_t t = 0;
    /* an explicit zero on each diagonal keeps every diagonal entry present */
    for (int64_t g = 0; g < n3; ++g) { T[t].t = (trip){g, (int32_t)g, 0.0}; T[t].order = t; ++t; }
    for (int64_t f = 0; f < f3; ++f) {
        face3d F = get_face(m, f);
        double coef = F.area / F.dist;
        T[t].t = (trip){F.c1, (int32_t)F.c1, -coef}; T[t].order = t; ++t;
        T[t].t = (trip){F.c1, (int32_t)F.c2, +coef}; T[t].order = t; ++t;
        T[t].t = (trip){F.c2, (int32_t)F.c2, -coef}; T[t].order = t; ++t;
        T[t].t = (trip){F.c2, (int32_t)F.c1, +coef}; T[t].order = t; ++t;
    }
    if (m->dirichlet)
        for (int l = 0; l < m->k; ++l)
            for (int w = 0; w < m->n_walls; ++w) {
                int64_t g = (int64_t)l * m->n_cells + m->wcell[w];
                double a = m->wlen[w] * m->dz;
                T[t].t = (trip){g, (int32_t)g, -a / m->wdist[w]}; T[t].order = t; ++t;
            }
    int r = to_csr(T, t, n3, ptr, col, val, nnz);
    free(T);
    return r;
}

int64_t orc_div_max_nnz(const orc_mesh3d *m) { return 2 * orc_n_faces3d(m); }

/* M: (M u)_c = sum over faces of c of (+area if c is the face's c1, -area if
 * c2) times u_f -- the integrated outward flux (Eq. 9a). */
int orc_assemble_div(const orc_mesh3d *m, int64_t *ptr, int32_t *col, double *val, int64_t *nnz)
{
    int e = check_mesh(m);
    if (e) return e;
    int64_t n3 = (int64_t)m->k * m->n_cells, f3 = orc_n_faces3d(m);
    trip_o *T = malloc(sizeof(trip_o) * (size_t)(2 * f3 > 0 ? 2 * f3 : 1));
    if (!T) return ERR_NOMEM;
    int64_t t = 0;
    for (int64_t f = 0; f < f3; ++f) {
        face3d F = get_face(m, f);
        T[t].t = (trip){F.c1, (int32_t)f, +F.area}; T[t].order = t; ++t;
        T[t].t = (trip){F.c2, (int32_t)f, -F.area}; T[t].order = t; ++t;
    }
    int r = to_csr(T, t, n3, ptr, col, val, nnz);
    free(T);
    return r;
}

int orc_face_volumes(const orc_mesh3d *m, double *omega_s)
{
    int64_t f3 = orc_n_faces3d(m);
    for (int64_t f = 0; f < f3; ++f) {
        face3d F = get_face(m, f);
        omega_s[f] = F.area * F.dist;
    }
    return 0;
}

int orc_cell_volumes(const orc_mesh3d *m, double *omega_c)
{
    for (int l = 0; l < m->k; ++l)
        for (int c = 0; c < m->n_cells; ++c)
            omega_c[(int64_t)l * m->n_cells + c] = m->area[c] * m->dz;
    return 0;
}

/* G = -Omega_s^{-1} M^T, computed from M's entries and the face volumes. */
int orc_assemble_grad(const orc_mesh3d *m, int64_t *ptr, int32_t *col, double *val, int64_t *nnz)
{
    int e = check_mesh(m);
    if (e) return e;
    int64_t f3 = orc_n_faces3d(m);
    trip_o *T = malloc(sizeof(trip_o) * (size_t)(2 * f3 > 0 ? 2 * f3 : 1));
    if (!T) return ERR_NOMEM;
    int64_t t = 0;
    for (int64_t f = 0; f < f3; ++f) {
        face3d F = get_face(m, f);
        double os = F.area * F.dist;
        T[t].t = (trip){f, (int32_t)F.c1, -(+F.area) / os}; T[t].order = t; ++t;
        T[t].t = (trip){f, (int32_t)F.c2, -(-F.area) / os}; T[t].order = t; ++t;
    }
    int r = to_csr(T, t, f3, ptr, col, val, nnz);
    free(T);
    return r;
}

/* ====================================================================== */
/* Dense brute force                                                      */
/* ====================================================================== */

int orc_dense_lap(const orc_mesh3d *m, double *L)
{
    int e = check_mesh(m);
    if (e) return e;
    int64_t n3 = (int64_t)m->k * m->n_cells, f3 = orc_n_faces3d(m);
    memset(L, 0, sizeof(double) * (size_t)(n3 * n3));
    for (int64_t f = 0; f < f3; ++f) {
        face3d F = get_face(m, f);
        double a = F.area / F.dist;
        L[F.c1 * n3 + F.c1] -= a;
        L[F.c1 * n3 + F.c2] += a;
        L[F.c2 * n3 + F.c2] -= a;
        L[F.c2 * n3 + F.c1] += a;
    }
    if (m->dirichlet)
        for (int l = 0; l < m->k; ++l)
            for (int w = 0; w < m->n_walls; ++w) {
                int64_t g = (int64_t)l * m->n_cells + m->wcell[w];
                L[g * n3 + g] -= m->wlen[w] * m->dz / m->wdist[w];
            }
    return 0;
}

int orc_dense_div(const orc_mesh3d *m, double *M)
{
    int e = check_mesh(m);
    if (e) return e;
    int64_t n3 = (int64_t)m->k * m->n_cells, f3 = orc_n_faces3d(m);
    memset(M, 0, sizeof(double) * (size_t)(n3 * f3));
    for (int64_t f = 0; f < f3; ++f) {
        face3d F = get_face(m, f);
        M[F.c1 * f3 + f] += F.area;
        M[F.c2 * f3 + f] -= F.area;
    }
    return 0;
}

int orc_dense_grad(const orc_mesh3d *m, double *G)
{
    int e = check_mesh(m);
    if (e) return e;
    int64_t n3 = (int64_t)m->k * m->n_cells, f3 = orc_n_faces3d(m);
    memset(G, 0, sizeof(double) * (size_t)(n3 * f3));
    for (int64_t f = 0; f < f3; ++f) {
        face3d F = get_face(m, f);
        /* gradient along the normal from c1 to c2 */
        G[f * n3 + F.c2] += 1.0 / F.dist;
        G[f * n3 + F.c1] -= 1.0 / F.dist;
    }
    return 0;
}

int orc_dense_solve(int n, const double *L, const double *b, double *x, int n_groups)
{
    if (n < 1) return ERR_ARG;
    if (n_groups > 0 && n % n_groups) return ERR_ARG;
    double *A = malloc(sizeof(double) * (size_t)n * n);
    double *y = malloc(sizeof(double) * (size_t)n);
    if (!A || !y) { free(A); free(y); return ERR_NOMEM; }
    int gs = n_groups > 0 ? n / n_groups : n;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double v = -L[(size_t)i * n + j];
            if (n_groups > 0 && i / gs == j / gs) v += 1.0; /* pins 1^T x = 0 per group */
            A[(size_t)i * n + j] = v;
        }
    /* Cholesky A = R^T R, R upper triangular, stored in the upper triangle */
    for (int j = 0; j < n; ++j) {
        double s = A[(size_t)j * n + j];
        for (int p = 0; p < j; ++p) s -= A[(size_t)p * n + j] * A[(size_t)p * n + j];
        if (!(s > 0.0)) { free(A); free(y); return ERR_MESH; }
        double rjj = sqrt(s);
        A[(size_t)j * n + j] = rjj;
        for (int i = j + 1; i < n; ++i) {
            double t = A[(size_t)j * n + i];
            for (int p = 0; p < j; ++p) t -= A[(size_t)p * n + j] * A[(size_t)p * n + i];
            A[(size_t)j * n + i] = t / rjj;
        }
    }
    /* R^T y = -b, then R x = y (we solve -L x = -b) */
    for (int i = 0; i < n; ++i) {
        double t = -b[i];
        for (int p = 0; p < i; ++p) t -= A[(size_t)p * n + i] * y[p];
        y[i] = t / A[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double t = y[i];
        for (int p = i + 1; p < n; ++p) t -= A[(size_t)i * n + p] * x[p];
        x[i] = t / A[(size_t)i * n + i];
    }
    free(A);
    free(y);
    return 0;
}

/* ====================================================================== */
/* SpMV and CG                                                            */
/* ====================================================================== */

void orc_spmv(int64_t n_rows, const int64_t *ptr, const int32_t *col, const double *val,
              const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t j = ptr[i]; j < ptr[i + 1]; ++j) s += val[j] * x[col[j]];
        y[i] = s;
    }
}

/* Dot product summed in fixed chunks, then the chunk sums in order, so the
 * result does not depend on the number of threads. */
#define DOT_CHUNK 4096
static double dot(int64_t n, const double *a, const double *b)
{
    int64_t nc = (n + DOT_CHUNK - 1) / DOT_CHUNK;
    double *part = malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double s = 0.0;
        int64_t e = (c + 1) * DOT_CHUNK < n ? (c + 1) * DOT_CHUNK : n;
        for (int64_t i = c * DOT_CHUNK; i < e; ++i) s += a[i] * b[i];
        part[c] = s;
    }
    double s = 0.0;
    for (int64_t c = 0; c < nc; ++c) s += part[c];
    free(part);
    return s;
}

static void project_mean(int64_t n, double *v)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += v[i];
    double mean = s / (double)n;
    for (int64_t i = 0; i < n; ++i) v[i] -= mean;
}

/* y = L x restricted to rows [row0, row0+n), columns shifted by row0. */
static void spmv_block(int64_t row0, int64_t n, const int64_t *ptr, const int32_t *col,
                       const double *val, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = ptr[row0 + i]; j < ptr[row0 + i + 1]; ++j)
            s += val[j] * x[col[j] - row0];
        y[i] = s;
    }
}

int orc_cg(int64_t row0, int64_t n, const int64_t *ptr, const int32_t *col, const double *val,
           const double *b_in, double *x, int x_given, double tol, int max_iter, int singular,
           orc_cg_stats *st)
{
    if (n < 1 || max_iter < 0 || !(tol >= 0.0)) return ERR_ARG;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = ptr[row0 + i]; j < ptr[row0 + i + 1]; ++j)
            if (col[j] < row0 || col[j] >= row0 + n) return ERR_ARG;
    double *b = malloc(sizeof(double) * n), *r = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    if (!b || !r || !p || !q) { free(b); free(r); free(p); free(q); return ERR_NOMEM; }
    memcpy(b, b_in, sizeof(double) * n);
    if (singular) project_mean(n, b);
    double bnorm = sqrt(dot(n, b, b));
    st->bnorm = bnorm;
    st->iters = 0;
    st->status = 0;
    if (!x_given)
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        st->relres_rec = st->relres_true = 0.0;
        free(b); free(r); free(p); free(q);
        return 0;
    }
    /* CG on A = -L with right-hand side -b:  r = -b - A x = L x - b */
    spmv_block(row0, n, ptr, col, val, x, q);
    for (int64_t i = 0; i < n; ++i) r[i] = q[i] - b[i];
    for (int64_t i = 0; i < n; ++i) p[i] = r[i];
    double rho = dot(n, r, r);
    int it = 0;
    st->status = 1;
    if (sqrt(rho) <= tol * bnorm) st->status = 0;
    while (st->status == 1 && it < max_iter) {
        spmv_block(row0, n, ptr, col, val, p, q);     /* q = L p */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) q[i] = -q[i]; /* q = A p */
        double pq = dot(n, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { st->status = -5; break; }
        double alpha = rho / pq;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        double rho_new = dot(n, r, r);
        ++it;
        if (sqrt(rho_new) <= tol * bnorm) { rho = rho_new; st->status = 0; break; }
        double beta = rho_new / rho;
        rho = rho_new;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
    }
    st->iters = it;
    st->relres_rec = sqrt(rho) / bnorm;
    if (singular) project_mean(n, x);
    spmv_block(row0, n, ptr, col, val, x, q);
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += (b[i] - q[i]) * (b[i] - q[i]);
    st->relres_true = sqrt(s) / bnorm;
    free(b); free(r); free(p); free(q);
    return st->status == -5 ? -5 : 0;
}

/* Threads the OpenMP loops above use (1 without OpenMP). */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of threads of the OpenMP loops above (n >= 1; ignored
 * without OpenMP). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}


/* ---- higher-order structured operators (13- and 27-point) --------------
 *
 * The paper tests its SpMM with 7-, 13- and 27-point Laplacian stencils
 * (Section 4.1, the discretisation figure): first neighbours; first and
 * second neighbours along each axis; all 26 neighbours.  Here they are
 * written for a Cartesian base (the same face coordinates as
 * orc_cart_geometry) repeated in k periodic planes of spacing dz, with the
 * unknowns at the cell centres:
 *
 *  27-point: minus the tensor-product (trilinear finite-element) stiffness on
 *    the centre nodes, A = -(Kx My Mz + Mx Ky Mz + Mx My Kz).  Along one axis,
 *    every element joins two consecutive centres a, b at distance s and adds
 *    [1 -1; -1 1]/s to K and [2 1; 1 2] s/6 to M at (a, b).  A periodic axis
 *    closes the loop with an element across the period; a wall axis has none
 *    beyond its end centres (zero flux).
 *  13-point: A = (4/3) L1 - (1/6) L2.  L1 is the 7-point finite-volume form:
 *    off-diagonal len*dz/dist between face neighbours (len the face length,
 *    dist the centre distance) and area/dz between neighbouring planes.  L2
 *    has the same form between second neighbours along each axis (the face
 *    length over the distance of the two centres, area/(2 dz) between planes
 *    l and l +- 2).  Each has diagonal minus its off-diagonal row sum.  On a
 *    uniform grid this is the cell volume times the fourth-order central
 *    difference (-1/12, 4/3, -5/2, 4/3, -1/12)/h^2 along each axis.
 *
 * Rows and columns are 3D cells l*n_b + j*nx + i.  Entries that meet at one
 * column (short periodic axes) are summed.
 */
typedef struct {
    int n, periodic;
    double *c;        /* centres */
    double period;    /* length of the period (periodic axes) */
} axis1d;

static int make_axis(axis1d *a, int n, int periodic, const double *faces)
{
    a->n = n;
    a->periodic = periodic;
    a->c = malloc(sizeof(double) * (size_t)n);
    if (!a->c) return ERR_NOMEM;
    for (int i = 0; i < n; ++i) a->c[i] = 0.5 * (faces[i] + faces[i + 1]);
    a->period = faces[n] - faces[0];
    return 0;
}

/* centre distance from node i to node i + d (d = 1, 2), walking forward */
static double fwd_dist(const axis1d *a, int i, int d)
{
    double s = 0.0;
    for (int q = 0; q < d; ++q) {
        int u = (i + q) % a->n, v = (i + q + 1) % a->n;
        s += (u + 1 < a->n) ? a->c[v] - a->c[u] : a->c[v] + a->period - a->c[u];
    }
    return s;
}

/* dense 1D stiffness K and mass M (n x n, row-major) of an axis */
static int axis_km(const axis1d *a, double **K, double **M)
{
    int n = a->n;
    *K = calloc((size_t)n * n, sizeof(double));
    *M = calloc((size_t)n * n, sizeof(double));
    if (!*K || !*M) return ERR_NOMEM;
    int ne = a->periodic ? n : n - 1;
    for (int e = 0; e < ne; ++e) {
        int u = e, v = (e + 1) % n;
        double s = fwd_dist(a, e, 1);
        (*K)[u * n + u] += 1.0 / s;  (*K)[v * n + v] += 1.0 / s;
        (*K)[u * n + v] -= 1.0 / s;  (*K)[v * n + u] -= 1.0 / s;
        (*M)[u * n + u] += s / 3.0;  (*M)[v * n + v] += s / 3.0;
        (*M)[u * n + v] += s / 6.0;  (*M)[v * n + u] += s / 6.0;
    }
    return 0;
}

/* distinct indices among i-1, i, i+1 on an axis (periodic wrap or bounded) */
static int near3(const axis1d *a, int i, int *out)
{
    int m = 0;
    for (int d = -1; d <= 1; ++d) {
        int v = i + d;
        if (a->periodic) v = ((v % a->n) + a->n) % a->n;
        else if (v < 0 || v >= a->n) continue;
        int dup = 0;
        for (int q = 0; q < m; ++q) dup |= out[q] == v;
        if (!dup) out[m++] = v;
    }
    return m;
}

int64_t orc_stencil_max_nnz(int nx, int ny, int k, int stencil)
{
    int64_t n3 = (int64_t)nx * ny * k;
    return n3 * (stencil == 27 ? 27 : 14);
}

int orc_assemble_stencil(int nx, int ny, double x0, double Lx, double y0, double y1, double stretch,
                         int periodic_x, int periodic_y, int k, double dz, int stencil,
                         int64_t *ptr, int32_t *col, double *val, int64_t *nnz)
{
    if (nx < 1 || ny < 1 || k < 1 || !(dz > 0.0) || !(Lx > 0.0) || !(y1 > y0)) return ERR_ARG;
    if (stencil != 13 && stencil != 27) return ERR_ARG;
    double *xf = malloc(sizeof(double) * (nx + 1)), *yf = malloc(sizeof(double) * (ny + 1));
    double *zf = malloc(sizeof(double) * (k + 1));
    if (!xf || !yf || !zf) { free(xf); free(yf); free(zf); return ERR_NOMEM; }
    for (int i = 0; i <= nx; ++i) xf[i] = x0 + Lx * (double)i / (double)nx;
    for (int j = 0; j <= ny; ++j) yf[j] = stretched(j, ny, y0, y1, stretch);
    for (int l = 0; l <= k; ++l) zf[l] = dz * l;
    axis1d ax, ay, az;
    int e = make_axis(&ax, nx, periodic_x, xf);
    if (!e) e = make_axis(&ay, ny, periodic_y, yf);
    if (!e) e = make_axis(&az, k, 1, zf);
    if (e) return e;
    const int64_t nb = (int64_t)nx * ny, n3 = nb * k;
    int64_t cap = orc_stencil_max_nnz(nx, ny, k, stencil);
    trip_o *T = malloc(sizeof(trip_o) * (size_t)cap);
    if (!T) return ERR_NOMEM;
    int64_t t = 0;
#define PUT(R, C, V) do { T[t].t = (trip){(R), (int32_t)(C), (V)}; T[t].order = t; ++t; } while (0)
    if (stencil == 27) {
        double *Kx, *Mx, *Ky, *My, *Kz, *Mz;
        e = axis_km(&ax, &Kx, &Mx);
        if (!e) e = axis_km(&ay, &Ky, &My);
        if (!e) e = axis_km(&az, &Kz, &Mz);
        if (e) { free(T); return e; }
        for (int l = 0; l < k; ++l)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    int64_t r = (int64_t)l * nb + (int64_t)j * nx + i;
                    int ni[3], nj[3], nl[3];
                    int mi = near3(&ax, i, ni), mj = near3(&ay, j, nj), ml = near3(&az, l, nl);
                    for (int a = 0; a < ml; ++a)
                        for (int b = 0; b < mj; ++b)
                            for (int c = 0; c < mi; ++c) {
                                int I = ni[c], J = nj[b], Lz = nl[a];
                                double v = Kx[i * nx + I] * My[j * ny + J] * Mz[l * k + Lz]
                                         + Mx[i * nx + I] * Ky[j * ny + J] * Mz[l * k + Lz]
                                         + Mx[i * nx + I] * My[j * ny + J] * Kz[l * k + Lz];
                                PUT(r, (int64_t)Lz * nb + (int64_t)J * nx + I, -v);
                            }
                }
        free(Kx); free(Mx); free(Ky); free(My); free(Kz); free(Mz);
    } else {
        for (int l = 0; l < k; ++l)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    int64_t r = (int64_t)l * nb + (int64_t)j * nx + i;
                    double hx = xf[i + 1] - xf[i], hy = yf[j + 1] - yf[j];
                    double area = hx * hy, diag = 0.0;
                    for (int d = 1; d <= 2; ++d) {
                        double w = d == 1 ? 4.0 / 3.0 : -1.0 / 6.0;
                        for (int sgn = -1; sgn <= 1; sgn += 2) {
                            /* x */
                            int I = i + sgn * d;
                            if (periodic_x || (I >= 0 && I < nx)) {
                                int Iw = ((I % nx) + nx) % nx;
                                double dist = sgn > 0 ? fwd_dist(&ax, i, d) : fwd_dist(&ax, Iw, d);
                                double cf = w * hy * dz / dist;
                                PUT(r, (int64_t)l * nb + (int64_t)j * nx + Iw, cf);
                                diag -= cf;
                            }
                            /* y */
                            int J = j + sgn * d;
                            if (periodic_y || (J >= 0 && J < ny)) {
                                int Jw = ((J % ny) + ny) % ny;
                                double dist = sgn > 0 ? fwd_dist(&ay, j, d) : fwd_dist(&ay, Jw, d);
                                double cf = w * hx * dz / dist;
                                PUT(r, (int64_t)l * nb + (int64_t)Jw * nx + i, cf);
                                diag -= cf;
                            }
                            /* z (periodic planes) */
                            int Lz = (((l + sgn * d) % k) + k) % k;
                            double cf = w * area / (d * dz);
                            PUT(r, (int64_t)Lz * nb + (int64_t)j * nx + i, cf);
                            diag -= cf;
                        }
                    }
                    PUT(r, r, diag);
                }
    }
#undef PUT
    free(xf); free(yf); free(zf); free(ax.c); free(ay.c); free(az.c);
    int rc = to_csr(T, t, n3, ptr, col, val, nnz);
    free(T);
    return rc;
}
