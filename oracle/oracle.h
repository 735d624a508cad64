/*
 * Plain CPU oracle for the repeated-block finite-volume operators.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP library: it assembles the full 3D matrices face by face, with
 * no block reuse, and applies them with a plain row-sequential CSR SpMV and a
 * textbook conjugate-gradient loop.
 *
 * Numbering.  Base cells c = 0..n_b-1 and base faces f = 0..F_b-1 come from the
 * geometry routines.  3D cell (c, plane l) is g = l*n_b + c (plane-major, the
 * stacked vector of Section 2, Eq. 1).  3D faces: in-plane face f on plane l is
 * l*F_b + f; the z-face between (c, l) and (c, (l+1) mod k) is k*F_b + l*n_b + c.
 * z-faces exist only for coupling 1 (periodic along the repeated direction)
 * and k >= 2.
 *
 * All routines return 0 on success and a negative code on bad input.
 */
#ifndef FVX_ORACLE_H
#define FVX_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- base geometry ---------------------------------------------------- */
int orc_cart_sizes(int nx, int ny, int periodic_x, int periodic_y,
                   int *n_cells, int *n_faces, int *n_walls);
int orc_cart_geometry(int nx, int ny, double x0, double Lx, double y0, double y1,
                      double stretch, int periodic_x, int periodic_y,
                      double *area, double *cx, double *cy,
                      int *c1, int *c2, double *len, double *dist,
                      int *wcell, double *wlen, double *wdist);
int orc_tri_sizes(int n_pts, const double *xy, int n_tri, const int *tri,
                  int *n_faces, int *n_walls);
int orc_tri_geometry(int n_pts, const double *xy, int n_tri, const int *tri,
                     double *area, double *cx, double *cy,
                     int *c1, int *c2, double *len, double *dist,
                     int *wcell, double *wlen, double *wdist);

/* ---- 3D assembly (CSR, int64 row pointers, duplicates summed) ---------- */
typedef struct {
    int n_cells, n_faces, n_walls;
    const double *area;
    const int *c1, *c2;
    const double *len, *dist;
    const int *wcell;
    const double *wlen, *wdist;
    int k;          /* number of repeated planes */
    double dz;      /* plane spacing */
    int coupling;   /* 0: independent planes, 1: periodic z-faces */
    int dirichlet;  /* 1: walls impose p = 0 at the wall */
} orc_mesh3d;

int64_t orc_n_faces3d(const orc_mesh3d *m);
int64_t orc_lap_max_nnz(const orc_mesh3d *m);
int orc_assemble_lap(const orc_mesh3d *m, int64_t *ptr, int32_t *col, double *val, int64_t *nnz);
int64_t orc_div_max_nnz(const orc_mesh3d *m);
int orc_assemble_div(const orc_mesh3d *m, int64_t *ptr, int32_t *col, double *val, int64_t *nnz);
int orc_assemble_grad(const orc_mesh3d *m, int64_t *ptr, int32_t *col, double *val, int64_t *nnz);
int orc_face_volumes(const orc_mesh3d *m, double *omega_s);
int orc_cell_volumes(const orc_mesh3d *m, double *omega_c);

/* ---- higher-order structured operators (13- and 27-point) -------------- */
/* A Cartesian base (as orc_cart_geometry) repeated in k periodic planes;
 * stencil 13 or 27 (definitions in oracle.c).  CSR as orc_assemble_lap. */
int64_t orc_stencil_max_nnz(int nx, int ny, int k, int stencil);
int orc_assemble_stencil(int nx, int ny, double x0, double Lx, double y0, double y1, double stretch,
                         int periodic_x, int periodic_y, int k, double dz, int stencil,
                         int64_t *ptr, int32_t *col, double *val, int64_t *nnz);

/* ---- dense brute force (tiny meshes) ---------------------------------- */
int orc_dense_lap(const orc_mesh3d *m, double *L);   /* N x N row-major */
int orc_dense_div(const orc_mesh3d *m, double *M);   /* N x F3 */
int orc_dense_grad(const orc_mesh3d *m, double *G);  /* F3 x N */
/* Solve L x = b by Cholesky of -L (+ sum of group indicator outer products
 * when singular).  n_groups = 0: L nonsingular; otherwise the null space is
 * spanned by the indicators of n_groups equal consecutive index ranges. */
int orc_dense_solve(int n, const double *L, const double *b, double *x, int n_groups);

/* ---- apply and solve --------------------------------------------------- */
void orc_spmv(int64_t n_rows, const int64_t *ptr, const int32_t *col, const double *val,
              const double *x, double *y);

typedef struct {
    int iters;
    int status;          /* 0 converged, 1 not converged, -5 breakdown */
    double bnorm;        /* norm of the projected right-hand side */
    double relres_rec;   /* recursive residual / bnorm at exit */
    double relres_true;  /* ||b - L x|| / bnorm at exit */
} orc_cg_stats;

/* Textbook CG on A = -L for rows [row0, row0+n) of a CSR matrix whose columns
 * in those rows also lie in [row0, row0+n).  b is projected to zero plain mean
 * first when singular != 0, and x is projected on exit.  x holds the initial
 * guess when x_given != 0 (else zero).  Stops when the recursive residual
 * satisfies ||r|| <= tol ||b||. */
int orc_cg(int64_t row0, int64_t n, const int64_t *ptr, const int32_t *col, const double *val,
           const double *b, double *x, int x_given, double tol, int max_iter, int singular,
           orc_cg_stats *st);

int orc_threads(void);
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
