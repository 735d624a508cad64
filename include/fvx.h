/*
 * fvx -- repeated-block finite-volume operators as sparse-times-multivector
 * products on MI355X (gfx950).
 *
 * The operators follow the staggered symmetry-preserving finite-volume
 * discretisation of Section 3 (Eq. 9): the integrated divergence M, the face
 * volumes Omega_s, the gradient G = -Omega_s^{-1} M^T and the Laplacian
 * L = M G.  A 2D base mesh is extruded into k planes.  The 3D Laplacian then
 * has the repeated-block form  L = I_k (x) A_b + C  (Section 2, Eq. 1, and the
 * k stacked systems of Section 3.1, Eq. 10): one base block A_b, identical on
 * every plane, plus C, the faces between neighbouring planes (periodic along
 * the repeated direction) when the planes are coupled.  Every product with
 * these operators is one sparse-times-multivector product (SpMM, Algorithm 1)
 * over the k columns.
 *
 * CONVENTIONS
 *  - Every call returns an int status: 0 = FVX_OK, > 0 = warning, < 0 = error
 *    (see fvx_status).  No call aborts, exits or throws.  The text of the last
 *    error on the calling thread is returned by fvx_last_error().
 *  - "host" pointers point to CPU memory, "device" pointers to GPU memory on
 *    the current HIP device.  The caller owns all memory it passes in.
 *  - Streams are hipStream_t values passed as void* (NULL = default stream).
 *    Operator applications are asynchronous on that stream.
 *  - Multivectors are row-major "array of structures" (the AoS layout of
 *    Algorithm 1): row r holds the k values of that cell (or face) for the k
 *    planes contiguously, at elements [r*ld, r*ld + k).  ld >= k is fixed per
 *    operator (fvx_op_shape); columns k..ld-1 are padding, never read for
 *    results and never written.  Base pointers must be 16-byte aligned.
 *  - Cell vectors have n_b rows; in-plane face vectors have F_b rows; the
 *    faces between planes (plane l to plane (l+1) mod k) form a cell-shaped
 *    vector with n_b rows whose column l is the face above plane l.
 *  - Plane-major vectors (the stacked vector of Section 2) hold cell c of
 *    plane l at l*n + c; fvx_pack / fvx_unpack convert.
 */
#ifndef FVX_H
#define FVX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ */
/* Status codes, precisions, options                                   */
/* ------------------------------------------------------------------ */
typedef enum fvx_status {
    FVX_OK = 0,
    FVX_NOT_CONVERGED = 1,   /* warning: X holds the last iterate, stats are filled */
    FVX_E_ARG = -1,          /* null pointer, size or enum out of range, misaligned */
    FVX_E_MESH = -2,         /* mesh index out of range, non-positive area/length/distance */
    FVX_E_NOMEM = -3,        /* caller buffer smaller than the size query returned */
    FVX_E_HIP = -4,          /* a HIP runtime call failed (text in fvx_last_error) */
    FVX_E_BREAKDOWN = -5,    /* CG breakdown: p.Ap <= 0 with nonzero residual, or non-finite */
    FVX_E_NONFINITE = -6,    /* NaN/Inf in the right-hand side or initial guess */
    FVX_E_UNSUPPORTED = -7,  /* valid request this build does not provide */
    FVX_E_IO = -8            /* a file could not be opened, read or written, or is not the expected format */
} fvx_status;

enum { FVX_F64 = 0, FVX_F32 = 1, FVX_MIXED = 2 };
enum { FVX_COUPLING_NONE = 0, FVX_COUPLING_PERIODIC_Z = 1 };
enum { FVX_WALL_NEUMANN = 0, FVX_WALL_DIRICHLET = 1 };
enum { FVX_GUESS_ZERO = 0, FVX_GUESS_GIVEN = 1 };
/* Reported by fvx_poisson_solve_net only: the network's guess was used. */
enum { FVX_GUESS_NET = 2 };

typedef struct fvx_mesh fvx_mesh;   /* host-side base mesh (face graph) */
typedef struct fvx_op fvx_op;       /* operator: base block on the device + launch tiles */
typedef struct fvx_sparse fvx_sparse; /* a general CSR matrix on the device (fvx_sparse_*) */
typedef struct fvx_net fvx_net;     /* learned initial-guess network (device parameters) */
typedef struct fvx_amg fvx_amg;     /* aggregation multigrid hierarchy of an operator (fvx_amg_*) */

/* Returns a static string naming a status code. */
const char *fvx_status_str(int status);
/* Detail of the last error on the calling thread ("" if none). */
const char *fvx_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int fvx_version(void);

/* ------------------------------------------------------------------ */
/* Base meshes (host).  A base mesh is a 2D finite-volume face graph:  */
/* cells with an area, interior faces with their two cells (normal     */
/* from c1 to c2), length and centre-to-centre distance, and wall      */
/* faces with their cell, length and centre-to-wall distance.          */
/* ------------------------------------------------------------------ */

/* Structured base: nx uniform cells on [x0, x0+Lx]; ny cells on [y0, y1]
 * clustered towards both ends by y_j = y0 + (y1-y0)(1 + tanh(s(2j/ny-1))/tanh s)/2
 * (s = stretch; s = 0 is uniform), the hyperbolic-tangent refinement of the
 * channel case (Section 4.1).  Non-periodic sides are walls.  Cell (i, j) is
 * c = j*nx + i.  Interior faces are numbered x-normal faces first (j outer, i
 * inner, face between (i, j) and (i+1 mod nx, j)), then y-normal faces (j
 * outer, i inner, face between (i, j) and (i, j+1 mod ny)).
 * Errors: FVX_E_ARG for nx, ny < 1 or an empty extent. */
int fvx_mesh_cartesian(int nx, int ny, double x0, double Lx, double y0, double y1,
                       double stretch, int periodic_x, int periodic_y, fvx_mesh **out);

/* Triangle base (cells = triangles, e.g. a Delaunay mesh around a body).
 * xy: host [n_pts][2]; tri: host [n_tri][3] vertex indices.  Cell area and
 * centroid from the vertices; face length = edge length; face distance =
 * |n . (centroid_c2 - centroid_c1)| with n the unit edge normal (two-point
 * flux).  Interior faces are the edges shared by two triangles, in ascending
 * order of (lower vertex, higher vertex), with c1 the lower triangle index;
 * edges of one triangle are walls.  Errors: FVX_E_MESH for a vertex index out
 * of range, a degenerate triangle or an edge shared by more than two. */
int fvx_mesh_triangles(int n_pts, const double *xy, int n_tri, const int32_t *tri,
                       fvx_mesh **out);

/* General face graph.  All arrays are host memory and are copied.
 * area [n_cells] > 0; c1, c2 [n_faces] in [0, n_cells); len, dist > 0;
 * wcell [n_walls], wlen, wdist > 0 (may be NULL when n_walls == 0).
 * cx, cy [n_cells] optional cell centres (NULL allowed). */
int fvx_mesh_from_faces(int n_cells, const double *area, const double *cx, const double *cy,
                        int n_faces, const int32_t *c1, const int32_t *c2,
                        const double *len, const double *dist,
                        int n_walls, const int32_t *wcell, const double *wlen,
                        const double *wdist, fvx_mesh **out);

/* Cell order for locality (host only, no device work): perm[i] = index of
 * the point visited i-th along a Hilbert curve over the points' bounding box
 * (each axis scaled to a 2^16 grid; points in one grid cell keep index
 * order).  x, y, perm: host arrays of n.  Numbering a base mesh's cells in
 * this order (e.g. the triangles of fvx_mesh_triangles by their centroids)
 * keeps the in-plane neighbours of a row close in memory, so the SpMM's
 * gathers of the input multivector hit the caches: the reads of X move from
 * the no-reuse case of Section 2, Eq. 3b, toward the read-once case of
 * Eq. 3a.  The operator's rows follow the mesh's cell order, so the caller
 * numbers its fields the same way.  FVX_E_ARG for NULL arrays (n > 0),
 * n < 0 or n > INT32_MAX, or a non-finite coordinate. */
int fvx_hilbert_order(int64_t n, const double *x, const double *y, int32_t *perm);

/* Sizes of a mesh (any pointer may be NULL). */
int fvx_mesh_info(const fvx_mesh *m, int64_t *n_cells, int64_t *n_faces, int64_t *n_walls);
/* Copies the cell centres (host arrays of n_cells). */
int fvx_mesh_centroids(const fvx_mesh *m, double *cx, double *cy);
/* Copies the face graph (host arrays sized by fvx_mesh_info; NULL skips). */
int fvx_mesh_faces(const fvx_mesh *m, double *area, int32_t *c1, int32_t *c2,
                   double *len, double *dist);
int fvx_mesh_destroy(fvx_mesh *m);

/* ------------------------------------------------------------------ */
/* Operators                                                           */
/* ------------------------------------------------------------------ */
typedef struct fvx_op_desc {
    int32_t k;          /* number of repeated planes (columns), >= 1 */
    int32_t coupling;   /* FVX_COUPLING_NONE: k independent systems (Section 3.1);
                           FVX_COUPLING_PERIODIC_Z: faces between planes l and
                           l+1 mod k (area = cell area, distance = dz) */
    double dz;          /* plane spacing (> 0); in-plane face area = len * dz */
    int32_t wall_bc;    /* FVX_WALL_NEUMANN: zero-flux walls (L singular, null
                           space = constants); FVX_WALL_DIRICHLET: p = 0 on walls */
    int32_t with_f32;   /* nonzero: also store FP32 copies (FVX_F32 and FVX_MIXED) */
    int32_t stencil;    /* Laplacian: 0 or 7 = the finite-volume operator of the face
                           graph (Section 3, Eq. 9); 13 or 27 = the higher-order
                           structured stencils of Section 4.1 on a Cartesian base
                           (fvx_mesh_cartesian), coupling PERIODIC_Z, zero-flux walls,
                           k <= 64 or even k <= 128:
                             27: minus the trilinear-element (Q1) stiffness on the
                                 cell centres, -(Kx My Mz + Mx Ky Mz + Mx My Kz);
                             13: (4/3) L1 - (1/6) L2, L1 the 7-point finite-volume
                                 form and L2 the same form between second neighbours
                                 along each axis (area/(2 dz) between planes l, l+-2):
                                 the fourth-order central difference on uniform grids.
                           div/grad stay the face-graph operators; solves and
                           fvx_lap's colscale need 7 (E_UNSUPPORTED / E_ARG). */
    int32_t reserved[3];
} fvx_op_desc;

/* Launch tile of the SpMM kernels: vec = elements per lane per load (FP64:
 * 1 or 2, FP32: 1, 2 or 4); lanes_per_row = lanes sharing one matrix row
 * (power of two, 1..64); block = threads per workgroup (64..1024, multiple of
 * 64); xcd_remap = nonzero maps consecutive row tiles to the same XCD;
 * max_blocks = cap on workgroups (each then walks several consecutive row
 * tiles), 0 = one tile per workgroup; on a Cartesian 5-point base whose
 * k columns one row group covers (lanes_per_row * vec == k, lanes_per_row
 * >= 8, no LDS staging) a cap below the tile count instead gives each row
 * group 2 or 4 grid lines along y, the fewest that fit under the cap (at
 * most ny), loaded together; stage_lds = nonzero stages each tile's
 * base-block rows (column indices, values, diagonal, coupling weight) in LDS
 * with coalesced loads, shared by all lanes of a row (needs at most 64 rows
 * per tile, i.e. block / lanes_per_row <= 64); nt_store = nonzero writes the
 * Laplacian SpMM's output with non-temporal stores (not re-read by the same
 * kernel).  When one row group covers the k columns in exactly 2 or 4 passes
 * (k = passes * lanes_per_row * vec, no LDS staging, block <= 512), every
 * pass's loads are issued before the arithmetic.  For the 13/27-point
 * operators a tile must cover k in one pass with vec dividing k, or in exactly
 * 2 or 4 passes (block <= 512), without LDS staging; with lanes_per_row = 64
 * their row metadata is read with scalar loads.  All tiles give bitwise the
 * same product. */
typedef struct fvx_tile {
    int32_t vec, lanes_per_row, block, xcd_remap, max_blocks, stage_lds, nt_store;
} fvx_tile;

/* Device bytes the operator needs (query before fvx_op_create). */
int fvx_op_bytes(const fvx_mesh *m, const fvx_op_desc *d, size_t *bytes);

/* Builds the operator.  dev_mem: device buffer of at least fvx_op_bytes bytes,
 * owned by the caller and kept alive until fvx_op_destroy.  The host builds
 * A_b, the plane-coupling weights, M_b and G_b once (their storage does not
 * grow with k) and copies them on `stream`; the call returns after the copy.
 * The op is immutable afterwards except for its tiles (fvx_op_set_tile). */
int fvx_op_create(const fvx_mesh *m, const fvx_op_desc *d, void *dev_mem, size_t bytes,
                  void *stream, fvx_op **out);
int fvx_op_destroy(fvx_op *op);

/* n_b cells, F_b in-plane faces, k planes, ld row stride of multivectors;
 * nnz_b = nnz(A_b).  Any pointer may be NULL. */
int fvx_op_shape(const fvx_op *op, int64_t *n_b, int64_t *F_b, int32_t *k, int32_t *ld,
                 int64_t *nnz_b);
/* 1 if L has the constant null space (solves project to zero mean). */
int fvx_op_singular(const fvx_op *op);

int fvx_op_get_tile(const fvx_op *op, int dtype, fvx_tile *tile);
/* Sets the SpMM tile for one precision.  FVX_E_ARG if the tile is invalid
 * for this operator (vec must divide ld, alignment, ranges above). */
int fvx_op_set_tile(fvx_op *op, int dtype, const fvx_tile *tile);

/* Autotuner.  Times the Laplacian SpMM of precision dtype on the device for
 * candidate tiles and sets the fastest on the op, in two stages: every row
 * mapping (vector width, lanes per row, workgroup size) with default launch
 * options, then every launch option (XCD remap, workgroup cap, LDS staging,
 * non-temporal stores) around the best mapping; on a Cartesian base whose k
 * columns one row group covers, also the caps of 1024 and 2048 (grid lines per
 * row group) at the other workgroup sizes.  Each candidate is timed with
 * HIP events over `reps` sweeps of up to 512 launches on rotating pairs.
 * scratch: device buffer for input/output pairs, at least
 * 2 * n_b * ld * sizeof(element) bytes; the more pairs fit, the colder the
 * caches (zero-filled here before timing).  results:
 * optional host array of max_results (tile, microseconds per launch) records,
 * *n_results receives the count tried.  Every candidate computes the same
 * product (the tiles are interchangeable); only the timing differs. */
typedef struct fvx_tune_result {
    fvx_tile tile;
    double us;
} fvx_tune_result;
int fvx_tune(fvx_op *op, int dtype, void *scratch, size_t scratch_bytes, int reps, void *stream,
             fvx_tune_result *results, int max_results, int *n_results);

/* Launch tile of the CG kernels (the fused direction+SpMM kernel and the
 * update kernel) per precision, separate from the SpMM tile: their partial
 * reductions make them sensitive to the workgroup size and the grid cap.
 * get: the tile in use (the one set or tuned, else the default: the SpMM
 * tile's vector width, 256 threads, XCD remap, at most 1024 workgroups),
 * with lanes per row widened so that one pass covers all k columns.
 * set: validated like fvx_op_set_tile, block at most 512 (256 with
 * independent planes); block 0 or tile NULL restores the default.
 * The solution of a solve depends on the CG tile only through the order of
 * its FP64 partial sums. */
int fvx_op_get_cg_tile(const fvx_op *op, int dtype, fvx_tile *tile);
int fvx_op_set_cg_tile(fvx_op *op, int dtype, const fvx_tile *tile);

/* CG autotuner: times `iters` CG iterations (FVX_F64: the FP64 solve; FVX_F32:
 * the FP32 inner CG of the mixed solve) of a fixed right-hand side for each
 * candidate (workgroup size 128/256/512, XCD remap on/off, grid cap
 * 512/1024/2048) and sets the fastest as the op's CG tile.  ws: device
 * workspace of fvx_tune_cg_bytes (256-byte aligned).  Synchronises
 * `stream`.  results/n_results as fvx_tune (microseconds per iteration). */
int fvx_tune_cg_bytes(const fvx_op *op, int dtype, size_t *bytes);
int fvx_tune_cg(fvx_op *op, int dtype, void *ws, size_t ws_bytes, int iters, void *stream,
                fvx_tune_result *results, int max_results, int *n_results);

/* The autotuners behind a tile cache file: the tile stored for this
 * operator's key is set without timing anything (*from_cache = 1); when the
 * key is absent (or its tile is not valid for this build) the tuner runs
 * (fvx_tune, fvx_tune_cg: same scratch/workspace and reps/iters arguments),
 * its choice is set and stored (*from_cache = 0).  *tile (may be NULL)
 * receives the tile in use.  Keys:
 *   "<arch>|<f64|f32>|k=<k>|ld=<ld>|n_b=<n_b>|nnz_b=<nnz_b>|stencil=<7|13|27>"
 *   "cg|<arch>|<f64|f32>|k=<k>|ld=<ld>|n_b=<n_b>|nnz_b=<nnz_b>|coupling=<0|1>"
 * with <arch> the device's architecture name ("gfx950").  The file is a JSON
 * object of entries {"tile": [vec, lanes_per_row, block, xcd_remap,
 * max_blocks, stage_lds, nt_store], "us" or "us_per_iter", "candidates",
 * ...}; other entries and members are kept when the file is rewritten (sorted
 * keys, one-space indentation, written to "<path>.tmp" and renamed over the
 * file).  cache_path NULL: tune without a cache.  Writers within one process
 * are serialised; processes sharing a file may each tune a key once.
 * FVX_E_IO for an unreadable or malformed file or a failed write. */
int fvx_tune_cached(fvx_op *op, int dtype, const char *cache_path, void *scratch, size_t scratch_bytes, int reps,
                    void *stream, fvx_tile *tile, int *from_cache);
int fvx_tune_cg_cached(fvx_op *op, int dtype, const char *cache_path, void *ws, size_t ws_bytes, int iters,
                       void *stream, fvx_tile *tile, int *from_cache);

/* Laplacian SpMM (Algorithm 1 with the plane coupling):
 *   Y[i][l] = s_l ( sum_j A_b[i][j] X[j][l] + w_i (X[i][l+1 mod k] + X[i][l-1 mod k]) )
 * dtype FVX_F64 (double X, Y) or FVX_F32 (float X, Y; needs with_f32).
 * X, Y: device [n_b][ld], must not overlap.  colscale: device double [k], the
 * per-column output scale c of Algorithm 1, or NULL (s_l = 1). */
int fvx_lap(const fvx_op *op, int dtype, const void *X, void *Y, const double *colscale,
            void *stream);

/* n Laplacian SpMMs back to back on one stream, Y[i] = L X[i] (e.g. the k
 * stacked fields of several time levels).  X, Y: host arrays of n device
 * pointers, each as in fvx_lap. */
int fvx_lap_many(const fvx_op *op, int dtype, int n, const void *const *X, void *const *Y, void *stream);

/* Divergence SpMM, integrated over cells (M u of Eq. 9a):
 *   D[i][l] = sum_{faces f of i} (+-) len_f dz Uf[f][l] + A_i (Wz[i][l] - Wz[i][l-1 mod k])
 * with + when i is the face's c1.  Uf: device [F_b][ld]; Wz: device [n_b][ld]
 * (faces between planes; ignored and may be NULL when there are none);
 * D: device [n_b][ld]. */
int fvx_div(const fvx_op *op, int dtype, const void *Uf, const void *Wz, void *D, void *stream);

/* Convective operator C(u_s) = M U_s Pi (Section 3.1: the divergence of the
 * face velocities times the face-interpolated cell values, Pi the midpoint
 * interpolation):
 *   Out[i][l] = sum_{faces f of i} (+-) len_f dz Uf[f][l] (Phi[i][l] + Phi[j][l]) / 2
 *             + A_i (Wz[i][l] (Phi[i][l] + Phi[i][l+1]) - Wz[i][l-1] (Phi[i][l-1] + Phi[i][l])) / 2
 * (j the cell across f; plane indices mod k).  Uf, Wz: face velocities as in
 * fvx_div; Phi, Out: device [n_b][ld] (Out must not overlap the inputs).  For
 * a divergence-free u_s (M u_s = 0) the operator is skew-symmetric, so it
 * neither creates nor destroys the discrete kinetic energy. */
int fvx_convect(const fvx_op *op, int dtype, const void *Uf, const void *Wz, const void *Phi, void *Out,
                void *stream);

/* Gradient SpMM, G = -Omega_s^{-1} M^T (Eq. 9b):
 *   Gf[f][l] = (P[c2][l] - P[c1][l]) / dist_f,   Gz[i][l] = (P[i][l+1 mod k] - P[i][l]) / dz
 * P: device [n_b][ld]; Gf: device [F_b][ld]; Gz: device [n_b][ld] (may be
 * NULL when there are no faces between planes). */
int fvx_grad(const fvx_op *op, int dtype, const void *P, void *Gf, void *Gz, void *stream);

/* Gradient update  Gf += alpha * (G_b P),  Gz += alpha * (G_z P)  -- e.g. the
 * projection step u <- u - G p with alpha = -1.  Arguments as fvx_grad. */
int fvx_grad_axpy(const fvx_op *op, int dtype, double alpha, const void *P, void *Gf, void *Gz, void *stream);

/* Plane-major <-> row-major conversion on the device.  n_rows = n_b or F_b.
 * src/dst: device; pack reads [k][n_rows] and writes [n_rows][ld]. */
int fvx_pack(const fvx_op *op, int dtype, int64_t n_rows, const void *src, void *dst, void *stream);
int fvx_unpack(const fvx_op *op, int dtype, int64_t n_rows, const void *src, void *dst, void *stream);

/* ------------------------------------------------------------------ */
/* Poisson solve  L x = b  (CG on the SPD operator -L)                  */
/* ------------------------------------------------------------------ */
typedef struct fvx_solve_opts {
    double rtol;          /* stop when ||b - L x|| <= rtol ||b|| (b after projection) */
    int32_t max_iter;     /* CG iteration cap (inner iterations summed for MIXED) */
    int32_t precision;    /* FVX_F64, or FVX_MIXED: FP32 SpMM and vectors inside CG,
                             FP64 dot products and scalars, FP64 outer defect correction */
    double inner_rtol;    /* MIXED: inner CG tolerance relative to the outer residual; a
                             correction that needs less (outer residual within
                             1/(2 inner_rtol) of rtol ||b||) stops at half its need */
    int32_t max_outer;    /* MIXED: cap on outer corrections */
    int32_t guess;        /* FVX_GUESS_ZERO or FVX_GUESS_GIVEN (X holds x0) */
    int32_t poll_every;   /* most iterations between host reads of the device flag (>= 1):
                             the first read comes after min(poll_every, 8), later
                             ones when the residual's decay since the previous
                             read predicts convergence (the iterates do not
                             depend on when the host reads) */
    int32_t precond;      /* FVX_PRECOND_NONE (plain CG), FVX_PRECOND_JACOBI or
                             FVX_PRECOND_CHEBYSHEV (see below) */
    int32_t cheb_degree;  /* CHEBYSHEV: steps of the semi-iteration per application
                             (1..16; 1 is Jacobi) */
    double cheb_ratio;    /* CHEBYSHEV: the polynomial targets the interval
                             [2 / cheb_ratio, 2] of the spectrum of D^-1 A (> 1) */
    const fvx_amg *amg;   /* AMG: the hierarchy built for this operator (fvx_amg_create);
                             NULL otherwise */
    int32_t launch;       /* FVX_LAUNCH_PHASES or FVX_LAUNCH_GRAPH (see below) */
} fvx_solve_opts;

/* How the CG iterations between two host polls are launched:
 *   PHASES: kernel by kernel (the direction kernel, the update kernel and
 *           the preconditioner's kernels of every iteration).
 *   GRAPH (the default of fvx_solve_opts_default):
 *           after the first poll, replayed from HIP graphs of 1, 2, 4, ...,
 *           64 iterations.  The graphs are captured on first use (on a
 *           library-owned stream of the device, default priority) and kept
 *           in a process-wide cache of the 16 most recently used solve
 *           configurations, keyed by the device, precision, workspace
 *           address, operators (with their tiles), preconditioner and
 *           hierarchy: a repeated solve with the same operator, options and
 *           workspace (e.g. every time step) replays them with no capture.
 *           Same kernels, arguments and order as PHASES: the same X bitwise.
 *           Capturing allocates host and driver resources, so
 *           fvx_poisson_solve_noalloc always launches phase by phase.
 *           Dropping a cached configuration synchronises the device.
 *           On MI355X the replay saves 0-3 % per solve (the GPU's own time
 *           per dependent kernel, not the host's launch cost, bounds these
 *           iterations); the first solve of a configuration pays the capture
 *           (about 15 % of a plain-CG solve of 1.57 M unknowns). */
#define FVX_LAUNCH_PHASES 0
#define FVX_LAUNCH_GRAPH 1

/* Preconditioners of the CG (A = -L, D = diag(A); every step an SpMM or a
 * row-local update, no extra reductions):
 *   JACOBI:    z = D^-1 r, formed on the fly where z is read (no extra
 *              vector traffic per iteration).
 *   CHEBYSHEV: z = p(D^-1 A) D^-1 r, cheb_degree steps of the Chebyshev
 *              semi-iteration for D^-1 A z = D^-1 r from z = 0 (Saad,
 *              Iterative Methods for Sparse Linear Systems, Algorithm 12.1)
 *              on [2 / cheb_ratio, 2]; 2 bounds the spectrum of D^-1 A
 *              (Gershgorin).  Each step after the first is one fused SpMM
 *              kernel (4 vector passes); the workspace grows by 2 vectors
 *              per precision.
 *   AMG:       z = one V-cycle of the aggregation multigrid opts.amg (see
 *              fvx_amg_create), in the solve's precision (FP32 inside the
 *              MIXED inner CG); single solves only (FVX_E_ARG in a batch).
 * The paper's own solver preconditions CG with an adaptive AMG (Section 4);
 * every level of these preconditioners is applied as an SpMM. */
#define FVX_PRECOND_NONE 0
#define FVX_PRECOND_JACOBI 1
#define FVX_PRECOND_CHEBYSHEV 2
#define FVX_PRECOND_AMG 3

typedef struct fvx_solve_stats {
    int32_t status;       /* same as the return value */
    int32_t iters;        /* CG iterations (max over columns when planes are independent) */
    int32_t outer;        /* MIXED: outer corrections */
    int32_t rhs_projected;/* 1 if b had a nonzero plain mean that was removed */
    double relres_rec;    /* recursive residual / ||b|| at exit (max over columns) */
    double relres_true;   /* ||b - L x|| / ||b|| recomputed in FP64 (max over columns) */
    double r0_over_b;     /* ||b - L x0|| / ||b|| (max over columns) */
    double bnorm;         /* ||b|| after projection (max over columns) */
    double seconds;       /* wall time of the call */
} fvx_solve_stats;

/* Fills opts with defaults: rtol 1e-8, max_iter 100000, FP64, inner_rtol 1e-4,
 * max_outer 50, zero guess, poll_every 64, no preconditioner (cheb_degree 8,
 * cheb_ratio 300: the fastest FP64 setting measured on the 192 x 128 x 64
 * channel). */
int fvx_solve_opts_default(fvx_solve_opts *opts);

/* Device workspace bytes for fvx_poisson_solve. */
int fvx_solve_bytes(const fvx_op *op, const fvx_solve_opts *opts, size_t *bytes);

/* Solves L x = b.  B, X: device double [n_b][ld].  With coupled planes the
 * system is one CG with global scalars; with independent planes
 * (FVX_COUPLING_NONE) each column runs its own CG (its own alpha, beta and
 * stopping test) inside the shared SpMM, as k independent systems.  When L is
 * singular, b is projected to zero plain mean (per column for independent
 * planes) and x is returned with zero mean.  ws: device workspace of at least
 * fvx_solve_bytes bytes.  Synchronises `stream` before returning.  Returns
 * FVX_NOT_CONVERGED when the cap is hit, FVX_E_BREAKDOWN, FVX_E_NONFINITE. */
int fvx_poisson_solve(const fvx_op *op, const double *B, double *X, const fvx_solve_opts *opts,
                      void *ws, size_t ws_bytes, fvx_solve_stats *stats, void *stream);

/* The same solve with no device allocation and no workspace argument, for
 * callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The workspace is
 * the library's built-in scratch, a device array of
 * FVX_NOALLOC_SCRATCH_BYTES (128 MiB) that each device the library runs on
 * holds until the process ends; enough for an FP64 or MIXED plain-CG solve of
 * about 2.4 M unknowns (FP64) or 1.5 M (MIXED), e.g. 192 x 128 cells x 64
 * planes in either precision.  A solve whose workspace (fvx_solve_bytes)
 * exceeds the scratch fails with FVX_E_NOMEM before any device work.  B, X,
 * opts, stats and the other results are those of fvx_poisson_solve with the
 * same tiles (bitwise the same X); opts.launch is ignored (phase by phase).  The solve initialises every scratch byte
 * it reads, so nothing carries over from the previous call; but all calls on
 * one device share that device's scratch, so calls that overlap in time on
 * one device (several host threads or streams) race and must be serialised
 * by the caller.  Calls no hipMalloc/hipFree.  Synchronises `stream`. */
#define FVX_NOALLOC_SCRATCH_BYTES (128u * 1024u * 1024u)
int fvx_poisson_solve_noalloc(const fvx_op *op, const double *B, double *X, const fvx_solve_opts *opts,
                              fvx_solve_stats *stats, void *stream);

/* Many independent solves (uneven meshes and k) advanced together: every
 * CG phase of all problems still iterating is one launch (per group of
 * problems sharing a kernel instance: block size, vector width, coupling and
 * ELL width), each workgroup running one block of one problem's grid.  Each
 * problem takes exactly the steps and decisions of fvx_poisson_solve on its
 * own, so its result is bitwise identical to that solve with the same tiles.
 * ops, B, X: host arrays of n pointers (B[i], X[i] as in fvx_poisson_solve).
 * stats: host array of n records (or NULL).  Returns FVX_OK when all
 * converged, else the most severe status (errors before warnings). */
int fvx_solve_batch_bytes(int n, const fvx_op *const *ops, const fvx_solve_opts *opts, size_t *bytes);
int fvx_poisson_solve_batch(int n, const fvx_op *const *ops, const double *const *B, double *const *X,
                            const fvx_solve_opts *opts, void *ws, size_t ws_bytes, fvx_solve_stats *stats,
                            void *stream);

/* ------------------------------------------------------------------ */
/* Aggregation multigrid preconditioner (Section 4, Appendix A)          */
/* ------------------------------------------------------------------ */
/* The paper preconditions its CG with an algebraic multigrid whose every
 * level, and every restriction and prolongation between levels, is applied
 * to all stacked fields as one SpMM (Appendix A lists those products).  This
 * hierarchy keeps the repeated-block form on every level: a Galerkin product
 * P^T A P with piecewise-constant aggregates P of an operator
 * I_k (x) A_b + C is again such an operator, so each level is an fvx_op and
 * runs the same SpMM kernels as the fine one.
 *   Coarsening (host, once): each level is coarsened EITHER in the base
 *   plane, by two passes of pairwise aggregation of the base cells (cells in
 *   index order; a free cell i joins its free neighbour j of largest coupling
 *   t_ij among those with t_ij >= beta * max_j' t_ij', ties within a relative
 *   1e-9 to the smallest j; else it stays alone, and after the pass joins the
 *   aggregate of its neighbour of largest coupling), OR along the repeated
 *   direction, merging planes 2l and 2l + 1 (coupled planes, k even), which
 *   it does when the lower median over base cells of w_i / max_j t_ij
 *   exceeds z_rule (w_i: coupling to a neighbouring plane).  A level with at
 *   most coarse_max unknowns (n_b k, all planes) is the coarsest; it is
 *   solved with its dense pseudo-inverse (inverse with Dirichlet walls) per
 *   independent system, formed on the host in FP64.
 *   Plane modes (mode_cells > 0): a level with at most mode_cells base
 *   cells whose solve per plane (below) multiplies at most 2^23
 *   pseudo-inverse terms per cycle, u n_b^2 <= 2^23 with u = floor(k/2) + 1
 *   for coupled planes and u = ceil(k/2) for independent ones, is also the
 *   coarsest, and a coarsest level within both limits and above coarse_max
 *   unknowns is solved per plane: independent planes by the one n_b x n_b
 *   pseudo-inverse, two planes per row read; coupled planes per mode.  Their
 *   planes are coupled periodically, so the real discrete Fourier basis
 *   along the planes splits the level exactly into floor(k/2) + 1 systems
 *   A_b + (2 - 2 cos(2 pi m / k)) W of n_b unknowns (mode m; one right-hand
 *   side for m = 0 and m = k/2, a cosine and a sine one otherwise).  It is
 *   solved by the transform to the modes,
 *   the dense pseudo-inverse of every mode system (formed on the host in
 *   FP64) and the transform back: the same pseudo-inverse of the whole level,
 *   in three launches and (floor(k/2) + 1) n_b^2 stored terms instead of
 *   (n_b k)^2.
 *   Cycle: V-cycle; on each level `degree` Chebyshev steps for A z = r on
 *   [2 / ratio, 2] of the spectrum of D^-1 A from z = 0, restriction of the
 *   residual (fused with its SpMM), the coarse cycle, prolongation of the
 *   correction (fused with the first post-smoothing SpMM) and `degree`
 *   post-smoothing steps from the corrected iterate.  Pre- and post-smoother
 *   are the same symmetric polynomial, so the cycle is a symmetric
 *   preconditioner for CG.  Kernels per level: 2 degree + 1 (one fewer for
 *   degree 2 on the way down); every one returns at once once the solve
 *   using the cycle has converged.
 * Ownership: dev_mem (fvx_amg_bytes) holds every coarse operator, the
 * aggregate maps and the coarsest pseudo-inverse (or the plane modes'
 * pseudo-inverses and the Fourier basis); the caller keeps it and the fine
 * op alive until fvx_amg_destroy.  The hierarchy is immutable. */
typedef struct fvx_amg_opts {
    int32_t degree;      /* Chebyshev smoothing steps before and after the coarse correction (2..8) */
    double ratio;        /* smoother interval [2 / ratio, 2] (> 1) */
    double beta;         /* aggregation strength threshold (0 < beta <= 1) */
    double z_rule;       /* plane-merging threshold (>= 0) */
    int32_t coarse_max;  /* coarsest level size n_b k (1..2048) */
    int32_t max_levels;  /* 1..16 */
    int32_t mode_cells;  /* coarsest at <= mode_cells base cells (and <= 2^23 terms per cycle),
                            solved per plane mode (0: off; 0..2048) */
} fvx_amg_opts;

/* degree 2, ratio 8, beta 0.75, z_rule 1, coarse_max 2048, max_levels 16, mode_cells 2048. */
int fvx_amg_opts_default(fvx_amg_opts *opts);

/* Builds the hierarchy of op (which must have been built from mesh m with
 * the finite-volume stencil, 7) on the host and returns the device bytes it
 * needs (the coarsest pseudo-inverses are sized here and formed by
 * fvx_amg_create).  FVX_E_UNSUPPORTED for the 13/27-point operators. */
int fvx_amg_bytes(const fvx_mesh *m, const fvx_op *op, const fvx_amg_opts *opts, size_t *bytes);
/* Builds the hierarchy into dev_mem (256-byte aligned, >= fvx_amg_bytes);
 * the coarse operators carry FP32 copies when op does.  Copies on `stream`
 * and returns after the copies. */
int fvx_amg_create(const fvx_mesh *m, const fvx_op *op, const fvx_amg_opts *opts, void *dev_mem, size_t bytes,
                   void *stream, fvx_amg **out);
int fvx_amg_destroy(fvx_amg *amg);

/* Number of levels (the fine operator is level 0). */
int fvx_amg_n_levels(const fvx_amg *amg, int32_t *n_levels);
/* Level `level`: base cells, planes, nonzeros of its base block, how the
 * next level is made (0: this is the coarsest, 1: base-plane aggregation,
 * 2: plane merging) and its operator (owned by the hierarchy; usable with
 * fvx_lap and the other operator calls).  Any pointer may be NULL. */
int fvx_amg_level(const fvx_amg *amg, int32_t level, int64_t *n_b, int32_t *k, int64_t *nnz_b, int32_t *kind,
                  const fvx_op **op);
/* Base cell -> aggregate of a level of kind 1 (host int32 [n_b]). */
int fvx_amg_aggregates(const fvx_amg *amg, int32_t level, int32_t *agg);
/* Systems of the coarsest level's solve per plane: floor(k/2) + 1 plane
 * modes (coupled planes) or 1 shared by the planes (independent planes); 0
 * when it is solved by one dense pseudo-inverse over its unknowns (host
 * int32). */
int fvx_amg_coarsest_modes(const fvx_amg *amg, int32_t *modes);

/* One V-cycle Z = M^-1 R (device [n_b][ld] of the fine op, precision dtype
 * FVX_F64 or FVX_F32; R and Z must not overlap).  ws: device workspace of at
 * least fvx_amg_apply_bytes bytes (per-level vectors).  Asynchronous. */
int fvx_amg_apply_bytes(const fvx_amg *amg, int dtype, size_t *bytes);
int fvx_amg_apply(const fvx_amg *amg, int dtype, const void *R, void *Z, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* Learned initial guess                                                */
/* ------------------------------------------------------------------ */
/* Not part of the paper's method: a small convolutional network that
 * predicts the initial guess of the pressure Poisson solve of the projection
 * step (Section 3, Eq. 9: L = M G with the Kronecker-repeated blocks of
 * Section 2) from the right-hand side and the previous pressure, with the
 * residual deciding whether the prediction is used.
 *
 * Network: four 3x3x3 convolutions 2 -> 32 -> 32 -> 32 -> 1 with ReLU after
 * the first three and the input's channel 1 added to the output (the network
 * refines the previous pressure), FP32 weights and FP32 accumulation, on the grid of a
 * Cartesian base (fvx_mesh_cartesian, nx x ny cells) extruded into nz = k
 * planes.  Padding: periodic in x and z, edge-replicated in y.
 * Tensors (device, float): samples [ns][2][nz][ny][nx] (channel 0 = f / s,
 * channel 1 = p_prev / s), outputs and targets [ns][nz][ny][nx], where
 * f = (b - mean b) / (cell volume) is the source density (mean removed only
 * for singular operators), s its rms over the cells (1 if zero).  The guess
 * is x0 = s * (out - mean out) (mean removed only for singular operators).
 * Parameters (host float, fvx_net_n_params() values): per layer its weights
 * [co][ci][tap], tap = (dz*3 + dy)*3 + dx reading the input at offsets
 * (dz-1, dy-1, dx-1), followed by its biases [co].
 * Training: loss = mean over ns*cells of (out - target)^2; Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8) with bias correction.  Deterministic.
 * Calls are asynchronous on `stream` unless stated.  Errors: FVX_E_ARG for
 * NULL pointers, sample counts outside [1, batch] or an operator that is not
 * this grid; FVX_E_NOMEM for a short buffer. */
int fvx_net_n_params(void);

/* Device bytes of a network for an nx x ny x nz grid that trains on up to
 * `batch` samples per step (parameters, Adam moments, activations, gradient
 * scratch). */
int fvx_net_bytes(int nx, int ny, int nz, int batch, size_t *bytes);

/* Creates the network in caller-owned device memory dev_mem (256-byte
 * aligned, >= fvx_net_bytes; must outlive the handle).  init: host
 * parameters, or NULL for zeros.  Synchronises `stream`. */
int fvx_net_create(int nx, int ny, int nz, int batch, const float *init, void *dev_mem, size_t bytes,
                   void *stream, fvx_net **out);
int fvx_net_destroy(fvx_net *net);

/* Copies the parameters and/or the last gradients to host arrays (either may
 * be NULL).  Synchronous. */
int fvx_net_get_params(const fvx_net *net, float *params, float *grads);

/* Replaces the parameters and clears the Adam state.  Synchronises `stream`. */
int fvx_net_set_params(fvx_net *net, const float *params, void *stream);

/* Checkpoint of a network in a file: the parameters, the Adam moments and
 * the number of Adam steps taken, so that training resumes exactly where it
 * stopped.  Format (the host's byte order, little-endian on x86-64 hosts):
 * the 8 bytes "FVXNET01", int32 n_params (= fvx_net_n_params()), int32
 * steps, then float32 params[n_params], m[n_params], v[n_params].  The
 * parameters do not depend on the grid: a checkpoint loads into a network of
 * any grid and batch.  Both calls synchronise `stream`.  Errors: FVX_E_ARG
 * for a NULL net or path; FVX_E_IO when the file cannot be opened, read or
 * written, or its magic or parameter count differ (the network is then left
 * unchanged). */
int fvx_net_save(const fvx_net *net, const char *path, void *stream);
int fvx_net_load(fvx_net *net, const char *path, void *stream);

/* out = net(in) for ns samples (device arrays as above). */
int fvx_net_forward(fvx_net *net, int ns, const float *in, float *out, void *stream);

/* Gradients of the loss of ns samples with respect to every parameter (kept
 * in the network; read with fvx_net_get_params), no update.  *loss (may be
 * NULL) = the loss before the step.  Synchronises `stream`. */
int fvx_net_gradients(fvx_net *net, int ns, const float *in, const float *target, double *loss, void *stream);

/* One Adam step with learning rate lr on ns samples (fvx_net_gradients then
 * fvx_net_apply_adam).  Synchronises `stream`. */
int fvx_net_train_step(fvx_net *net, int ns, const float *in, const float *target, float lr, double *loss,
                       void *stream);

/* The network's gradient buffer: device float [fvx_net_n_params()], written
 * by fvx_net_gradients and read by fvx_net_apply_adam.  A caller may combine
 * gradients in place between the two (sum over micro-batches, or an
 * all-reduce across data-parallel replicas).  NULL for a NULL net. */
float *fvx_net_grads(fvx_net *net);

/* One Adam step with learning rate lr from the gradient buffer as it is. */
int fvx_net_apply_adam(fvx_net *net, float lr, void *stream);

/* One training sample from solver vectors (device double [n_b][ld]): B the
 * right-hand side, Pprev the previous pressure (NULL = none), Xstar the
 * solution (NULL with target = NULL: input only).  in: device float
 * [2][nz][ny][nx]; target: device float [nz][ny][nx] = Xstar / s. */
int fvx_net_prepare(fvx_net *net, const fvx_op *op, const double *B, const double *Pprev, const double *Xstar,
                    float *in, float *target, void *stream);

/* X0 (device double [n_b][ld], columns < k written) = the network's guess
 * for right-hand side B and previous pressure Pprev (NULL = none). */
int fvx_net_guess(fvx_net *net, const fvx_op *op, const double *B, const double *Pprev, double *X0, void *stream);

/* fvx_poisson_solve started from the best of three initial guesses, judged
 * by the FP64 residual ||b - L x0|| / ||b|| (b after projection, max over CG
 * groups): the network's guess (if finite), the previous pressure Pprev (if
 * not NULL) and zero (ratio 1).  Ties keep the earlier candidate in that
 * order.  With zero chosen the solve is exactly fvx_poisson_solve with
 * FVX_GUESS_ZERO; opts->guess is ignored.  *source (may be NULL) =
 * FVX_GUESS_NET, FVX_GUESS_GIVEN (the previous pressure) or FVX_GUESS_ZERO.
 * Pprev must not overlap X.  ws as fvx_poisson_solve; stats->seconds
 * includes the inference and the residual checks. */
int fvx_poisson_solve_net(const fvx_op *op, fvx_net *net, const double *B, const double *Pprev, double *X,
                          const fvx_solve_opts *opts, void *ws, size_t ws_bytes, fvx_solve_stats *stats,
                          int *source, void *stream);

/* ------------------------------------------------------------------ */
/* Comparators for measurement                                         */
/* ------------------------------------------------------------------ */

/* The assembled 3D Laplacian with no block reuse: I_k (x) A_b + C expanded
 * into one CSR matrix over plane-major rows l*n_b + c (columns ascending,
 * duplicate entries merged).  Host arrays: ptr [k*n_b + 1], col and val
 * [*nnz].  Call with ptr = col = val = NULL to query *nnz.  FVX_E_ARG when the
 * expansion does not fit int32 indices. */
int fvx_expand_csr(const fvx_mesh *m, const fvx_op_desc *d, int64_t *nnz, int32_t *ptr, int32_t *col,
                   double *val);

/* y = A x for an assembled CSR matrix (device arrays, int32 row pointers and
 * column indices, FP64 values): the plain SpMV that the repeated-block SpMM
 * replaces.  nnz = ptr[n_rows], passed from the host, only sizes the lane
 * groups: a group of lanes per row (the mean row length rounded up to a power
 * of two, 1 when it is at most 2) strides over the row and reduces by
 * shuffles. */
int fvx_csr_spmv(int64_t n_rows, int64_t nnz, const int32_t *ptr, const int32_t *col, const double *val,
                 const double *x, double *y, void *stream);

/* Textbook FP64 CG on an assembled CSR matrix (SPD -A form as fvx_poisson_solve)
 * with separate kernels for the SpMV (as fvx_csr_spmv), each dot product,
 * each axpy and the search-direction update.  B, X: device double [n].  singular != 0
 * projects b (and x on exit) to zero plain mean.  Options and statistics as
 * fvx_poisson_solve (precision must be FVX_F64). */
int fvx_csr_solve_bytes(int64_t n_rows, size_t *bytes);
int fvx_csr_poisson_solve(int64_t n_rows, int64_t nnz, const int32_t *ptr, const int32_t *col, const double *val,
                          const double *B, double *X, int singular, const fvx_solve_opts *opts,
                          void *ws, size_t ws_bytes, fvx_solve_stats *stats, void *stream);

/* ------------------------------------------------------------------ */
/* General sparse matrix times multivector (Section 2, Algorithm 1)     */
/* ------------------------------------------------------------------ */
/* Any n_rows x n_cols matrix A (rectangular allowed) given in CSR on the host
 * (int32 ptr [n_rows+1] with ptr[0] = 0, int32 col [nnz] in 0..n_cols-1,
 * finite double val [nnz]; duplicates allowed and summed), copied once into
 * caller-owned device memory of fvx_sparse_bytes bytes (256-byte aligned;
 * FP32 values too when with_f32).  The handle owns no device memory; the
 * buffer must outlive it.  Errors: FVX_E_ARG for a malformed CSR, FVX_E_NOMEM
 * for a short buffer. */
int fvx_sparse_bytes(int64_t n_rows, int64_t nnz, int with_f32, size_t *bytes);
int fvx_sparse_create(int64_t n_rows, int64_t n_cols, const int32_t *ptr, const int32_t *col, const double *val,
                      int with_f32, void *dev_mem, size_t bytes, void *stream, fvx_sparse **out);
int fvx_sparse_destroy(fvx_sparse *A);
int fvx_sparse_shape(const fvx_sparse *A, int64_t *n_rows, int64_t *n_cols, int64_t *nnz);
/* Launch tile (fvx_tile; stage_lds must be 0).  block 0 or NULL restores the
 * default: the widest vector dividing ldx and ldy, lanes per row covering k,
 * 256 threads, XCD remap.  lanes_per_row beyond what k needs (c = the power of
 * two covering ceil(k / vec)) splits each row's nonzeros among
 * lanes_per_row / c sub-groups whose sums are added by shuffles.  Tiles with
 * the same split factor give bitwise the same product. */
int fvx_sparse_set_tile(fvx_sparse *A, int dtype, const fvx_tile *tile);
/* Y = diag(colscale) (A X): X device [n_cols][ldx], Y device [n_rows][ldy],
 * row-major multivectors of k columns (16-byte aligned; ldx a multiple of the
 * tile's vector width holding k rounded up to it, ldy >= k; only the first k
 * columns of Y are written).  colscale: device double [k] (one factor per
 * column, e.g. one viscosity per parameter) or NULL.  Each stored entry of A
 * is read once per row group and applied to all k columns in entry order with
 * fused multiply-adds.  X and Y must not overlap. */
int fvx_sparse_spmm(const fvx_sparse *A, int dtype, int k, const void *X, int ldx, void *Y, int ldy,
                    const double *colscale, void *stream);
/* Autotuner of the tile for products with k columns and these strides: times
 * every row mapping (vector width, lanes per row, workgroup), then the launch
 * options (XCD remap, grid cap, non-temporal stores) around the best, `reps`
 * launches each on the caller's X (finite values) and Y, and keeps the
 * fastest as A's tile for dtype.  results: optional [max_results] timings. */
int fvx_sparse_tune(fvx_sparse *A, int dtype, int k, const void *X, int ldx, void *Y, int ldy, int reps,
                    void *stream, fvx_tune_result *results, int max_results, int *n_results);

/* Inline mesh refinement (Section 3.3) on a Cartesian base: fvx_mesh_refine
 * splits every cell into rf x rf equal children (rf 1..16; the same periodic
 * axes and walls); fvx_refine_prolongation gives the coarse-to-fine state
 * mapping as a CSR matrix of (nx rf)(ny rf) rows and nx ny columns (rows and
 * columns in the meshes' j*nx+i order): each fine value is the bilinear
 * interpolation of the coarse cell-centre values at the fine centre, periodic
 * axes wrapping across the period and wall-bounded axes taking the end
 * centre's value beyond it (zero gradient at walls); rows sum to 1.  Call with
 * ptr, col and val NULL for nnz, then with arrays of n_fine+1, nnz, nnz.
 * Applied with fvx_sparse_spmm to all k states at once.  FVX_E_UNSUPPORTED
 * for non-Cartesian meshes. */
int fvx_mesh_refine(const fvx_mesh *coarse, int rf, fvx_mesh **fine);
int fvx_refine_prolongation(const fvx_mesh *coarse, int rf, int64_t *nnz, int32_t *ptr, int32_t *col,
                            double *val);

/* ------------------------------------------------------------------ */
/* Incompressible time step (Sections 3 and 4)                          */
/* ------------------------------------------------------------------ */
/* One step of Heun's third-order Runge-Kutta scheme for the incompressible
 * Navier-Stokes equations on the extruded mesh, with a projection at every
 * stage (collocated velocities, symmetry-preserving operators):
 *   Omega du/dt = -C(u_s) u + nu L_v u - Omega Gamma_sc G p,   M u_s = 0,
 * C(u_s) = M U_s Pi (fvx_convect), L_v the viscous Laplacian of `visc` (NULL:
 * op's own L; e.g. an operator with FVX_WALL_DIRICHLET for no-slip walls),
 * Gamma_cs the cell-to-face interpolation u_s = n_f . (u_c1 + u_c2)/2 (and
 * (w_l + w_{l+1})/2 between planes), Gamma_sc = Omega^-1 Gamma_cs^T Omega_s its
 * volume-weighted adjoint.  A stage u* is projected by solving
 * L phi = M Gamma_cs u* / (c dt) with fvx_poisson_solve(opts) and setting
 * u_s = Gamma_cs u* - c dt G phi, u = u* - c dt Gamma_sc G phi; Heun's nodes
 * are 0, 1/3, 2/3 and weights 1/4, 0, 3/4.
 * U[3]: device double [n_b][ld] cell velocity components (in/out); Uf, Wz:
 * face velocities as in fvx_div (in: those of U; out: divergence-free); P:
 * device double [n_b][ld], out: phi of the last projection (its initial
 * guess when opts->guess is FVX_GUESS_GIVEN).  dt > 0, nu >= 0.  ws: device
 * workspace of fvx_ns_step_bytes bytes (256-byte aligned).  stats: the last
 * solve's, with iters summed over the three projections.  FP64 only; needs
 * face normals (Cartesian or triangle bases), else FVX_E_UNSUPPORTED. */
int fvx_ns_step_bytes(const fvx_op *op, const fvx_solve_opts *opts, size_t *bytes);
int fvx_ns_step(const fvx_op *op, const fvx_op *visc, double *const U[3], double *Uf, double *Wz, double *P,
                double dt, double nu, const fvx_solve_opts *opts, void *ws, size_t ws_bytes, fvx_solve_stats *stats,
                void *stream);

/* Streaming device copy of `bytes` (multiple of 16, 16-byte aligned buffers):
 * the achievable-bandwidth reference of the roofline. */
int fvx_copy(void *dst, const void *src, size_t bytes, void *stream);

/* n copies dst[i] <- src[i] of `bytes` each (same rules as fvx_copy),
 * launched back to back from the library: a bandwidth sweep whose launch
 * rate is not limited by the caller's language. */
int fvx_copy_many(int n, void *const *dst, const void *const *src, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FVX_H */
