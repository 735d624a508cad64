"""Aggregation multigrid for the Poisson solve (TEST INFRASTRUCTURE ONLY: the
test suite, the smoke check and the benchmark's CPU-baseline leg may use it;
the library never does).

The paper preconditions CG with an adaptive algebraic multigrid whose levels
are all applied as SpMMs, square operators on every level and rectangular
restriction and prolongation between levels (Section 4, Appendix A).  This
oracle is the multigrid the library builds, written on the ASSEMBLED matrices
with no block reuse:

* Levels.  A_0 = -L (SPD on the complement of its null space).  A level is
  coarsened either in the base plane or along the repeated direction:
    - base plane: two passes of pairwise aggregation of the base cells
      (Notay, ETNA 37, 2010): cells are visited in index order; an
      unaggregated cell i joins the unaggregated neighbour j with the largest
      coupling t_ij among those with t_ij >= beta * max_j' t_ij' (ties within
      a relative 1e-9 go to the smallest j), else it stays alone; then each
      cell left alone joins the aggregate of its neighbour of largest
      coupling (the second phase of plain aggregation).  The second pass
      pairs the aggregates of the first on the coarse couplings;
    - repeated direction: planes 2l and 2l+1 are merged (k even, planes
      coupled periodically);
  the direction is the repeated one when the plane coupling dominates: the
  lower median over base cells of w_i / max_j t_ij exceeds z_rule.
  P is the piecewise-constant prolongation of the aggregates, and the coarse
  operator is the Galerkin product A_c = P^T A P, formed here by sparse
  products on the assembled matrices.  t and w of a level are read back from
  its assembled operator: t_ij = -a_ij within plane 0, w_i = -a_i,(plane 1, i)
  (halved for two planes, whose two plane neighbours coincide).
* Coarsest level (at most coarse_max unknowns, counted over all planes;
  independent planes share one hierarchy; with mode_cells > 0 also a level
  of at most mode_cells base cells whose solve per plane multiplies at most
  MODE_TERMS pseudo-inverse terms, u n_b^2 with u = k // 2 + 1 plane modes
  of coupled planes or u = ceil(columns / 2) plane pairs of independent
  ones, which the library solves per plane (mode) -- here it is solved like
  any other coarsest level, as one matrix): the pseudo-inverse, from the
  eigen-decomposition with the eigenvalues below 1e-10 of the Galerkin scale
  dropped (the largest row sum of |P|^T |A| |P| carried down the levels: a
  one-cell Neumann level is zero up to the rounding of its sums).
* Cycle: a V-cycle with the Chebyshev-polynomial smoother of the
  preconditioned CG on [2 / ratio, 2] (Saad, Iterative Methods for Sparse
  Linear Systems, 2nd ed., Algorithm 12.1, with the Jacobi scaling D^-1):
  `degree` steps from zero before the coarse correction and `degree` steps
  from the corrected iterate after it.  Pre- and post-smoother are the same
  symmetric polynomial, so the cycle is a symmetric preconditioner.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

TIE = 1e-9
MODE_TERMS = 2 ** 23   # plane-mode pseudo-inverse terms a coarsest level may hold


@dataclass
class AmgOpts:
    degree: int = 2
    ratio: float = 8.0
    beta: float = 0.75
    z_rule: float = 1.0
    coarse_max: int = 2048
    max_levels: int = 16
    mode_cells: int = 0     # off here; comparisons with the library pass the value they use


@dataclass
class Level:
    A: sp.csr_matrix            # assembled level operator (plane-major: plane l, cell c at l * n_b + c)
    n_b: int
    k: int
    kind: str = ""              # how the next level was made: "xy" or "z"; "" on the coarsest
    agg: np.ndarray | None = None   # base cell -> aggregate (kind "xy")
    P: sp.csr_matrix | None = None  # prolongation to this level from the next


@dataclass
class Hierarchy:
    levels: list = field(default_factory=list)
    pinv: np.ndarray | None = None
    opts: AmgOpts = field(default_factory=AmgOpts)


def couplings(A: sp.csr_matrix, n_b: int, k: int):
    """In-plane couplings t (positive, zero diagonal) and plane coupling w of
    an assembled level operator."""
    B = A[:n_b, :n_b].tocoo()
    off = B.row != B.col
    T = sp.csr_matrix((-B.data[off], (B.row[off], B.col[off])), shape=(n_b, n_b))
    T.sum_duplicates()
    T.eliminate_zeros()
    if k >= 2:
        w = -A[:n_b, n_b:2 * n_b].diagonal()
        if k == 2:
            w = w / 2.0
    else:
        w = np.zeros(n_b)
    return T, w


def _row(T: sp.csr_matrix, i: int):
    cols = T.indices[T.indptr[i]:T.indptr[i + 1]]
    vals = T.data[T.indptr[i]:T.indptr[i + 1]]
    keep = cols != i
    return cols[keep], vals[keep]


def pairwise(T: sp.csr_matrix, beta: float):
    """One pass of pairwise aggregation; returns (aggregate of each node, count).

    Pairing: nodes in index order; a free node pairs with its free neighbour
    of largest coupling among those at least beta times its largest coupling.
    Then every node left alone (with a neighbour) joins, in index order, the
    aggregate of its neighbour of largest coupling: without this, a node whose
    strong neighbours are always taken first stays alone on every level and
    coarsening stalls.  Aggregates are numbered in order of their smallest
    node."""
    n = T.shape[0]
    agg = -np.ones(n, np.int64)
    nc = 0
    for i in range(n):
        if agg[i] >= 0:
            continue
        cols, vals = _row(T, i)
        pick = -1
        if len(vals):
            mx = vals.max()
            cand = (agg[cols] < 0) & (vals >= beta * mx * (1.0 - TIE))
            if cand.any():
                best = vals[cand].max()
                good = cols[cand & (vals >= best * (1.0 - TIE))]
                pick = int(good.min())
        agg[i] = nc
        if pick >= 0:
            agg[pick] = nc
        nc += 1
    size = np.bincount(agg, minlength=nc)
    for i in range(n):
        if size[agg[i]] != 1:
            continue
        cols, vals = _row(T, i)
        if not len(vals):
            continue
        j = int(cols[vals >= vals.max() * (1.0 - TIE)].min())
        size[agg[i]] -= 1
        agg[i] = agg[j]
        size[agg[j]] += 1
    used = np.flatnonzero(size > 0)
    renum = -np.ones(nc, np.int64)
    renum[used] = np.arange(len(used))
    return renum[agg], len(used)


def aggregate(T: sp.csr_matrix, beta: float, passes: int = 2):
    """Composite of `passes` pairwise passes: base cell -> aggregate."""
    n = T.shape[0]
    total = np.arange(n)
    for _ in range(passes):
        agg, nc = pairwise(T, beta)
        Pb = sp.csr_matrix((np.ones(len(agg)), (np.arange(len(agg)), agg)), shape=(len(agg), nc))
        Tc = (Pb.T @ T @ Pb).tocoo()
        off = Tc.row != Tc.col
        T = sp.csr_matrix((Tc.data[off], (Tc.row[off], Tc.col[off])), shape=(nc, nc))
        total = agg[total]
    return total, int(total.max()) + 1 if n else 0


def lower_median(v: np.ndarray) -> float:
    s = np.sort(v)
    return float(s[(len(s) - 1) // 2])


def build(A0: sp.csr_matrix, n_b: int, k: int, coupled: bool, opts: AmgOpts | None = None,
          columns: int = 1, solve_coarsest: bool = True) -> Hierarchy:
    """The hierarchy of A0 (SPD form -L of one independent system: k planes
    coupled periodically when `coupled`, else k = 1), shared by `columns`
    independent systems (the planes of uncoupled operators): a level with at
    most coarse_max unknowns over all of them is the coarsest.  Without
    solve_coarsest the levels only (no pseudo-inverse)."""
    opts = opts or AmgOpts()
    h = Hierarchy(opts=opts)
    lev = Level(A0.tocsr(), n_b, k)
    absA = abs(lev.A)  # |P|^T |A| |P| down the levels: the scale of the Galerkin sums' rounding
    while True:
        h.levels.append(lev)
        if lev.n_b * lev.k * columns <= opts.coarse_max or len(h.levels) >= opts.max_levels:
            break
        units = lev.k // 2 + 1 if coupled else (columns + 1) // 2
        if opts.mode_cells > 0 and lev.n_b <= opts.mode_cells and units * lev.n_b ** 2 <= MODE_TERMS:
            break
        T, w = couplings(lev.A, lev.n_b, lev.k)
        tmax = np.zeros(lev.n_b)
        nz = np.diff(T.indptr) > 0
        tmax[nz] = np.maximum.reduceat(T.data, T.indptr[:-1][nz])
        ratio = w / np.where(tmax > 0, tmax, np.inf)
        if coupled and lev.k >= 2 and lev.k % 2 == 0 and lower_median(ratio) > opts.z_rule:
            Pz = sp.csr_matrix((np.ones(lev.k), (np.arange(lev.k), np.arange(lev.k) // 2)), shape=(lev.k, lev.k // 2))
            P = sp.kron(Pz, sp.identity(lev.n_b)).tocsr()
            lev.kind, lev.P = "z", P
            nxt = Level((P.T @ lev.A @ P).tocsr(), lev.n_b, lev.k // 2)
        else:
            agg, nc = aggregate(T, opts.beta)
            if nc == lev.n_b:
                break
            Pb = sp.csr_matrix((np.ones(lev.n_b), (np.arange(lev.n_b), agg)), shape=(lev.n_b, nc))
            P = sp.kron(sp.identity(lev.k), Pb).tocsr()
            lev.kind, lev.agg, lev.P = "xy", agg, P
            nxt = Level((P.T @ lev.A @ P).tocsr(), nc, lev.k)
        absA = (lev.P.T @ absA @ lev.P).tocsr()
        lev = nxt
    last = h.levels[-1]
    last.kind, last.agg, last.P = "", None, None
    if not solve_coarsest:
        return h
    lam, Q = np.linalg.eigh(last.A.toarray())
    keep = lam > 1e-10 * abs(absA).sum(axis=1).max()
    h.pinv = (Q[:, keep] / lam[keep]) @ Q[:, keep].T
    return h


def chebyshev_smooth(A: sp.csr_matrix, dinv: np.ndarray, r: np.ndarray, degree: int, ratio: float,
                     z0: np.ndarray | None = None) -> np.ndarray:
    """`degree` Chebyshev steps for A z = r from z0 (zero if None) with the
    Jacobi scaling, on [2 / ratio, 2] (Saad, Algorithm 12.1)."""
    b = 2.0
    a = b / ratio
    theta, delta = (b + a) / 2.0, (b - a) / 2.0
    sigma = theta / delta
    rho = 1.0 / sigma
    z = np.zeros_like(r) if z0 is None else np.array(z0, dtype=np.float64, copy=True)
    res = r - A @ z if z0 is not None else r.copy()
    d = dinv * res / theta
    for _ in range(degree - 1):
        z = z + d
        res = res - A @ d
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * res)
        rho = rho_new
    return z + d


def vcycle(h: Hierarchy, r: np.ndarray, level: int = 0) -> np.ndarray:
    """One V-cycle z = M^-1 r on `level`."""
    lev = h.levels[level]
    if level == len(h.levels) - 1:
        return h.pinv @ r
    o = h.opts
    dinv = 1.0 / lev.A.diagonal()
    z = chebyshev_smooth(lev.A, dinv, r, o.degree, o.ratio)
    rc = lev.P.T @ (r - lev.A @ z)
    z = z + lev.P @ vcycle(h, rc, level + 1)
    return chebyshev_smooth(lev.A, dinv, r, o.degree, o.ratio, z0=z)


def two_level_error(h: Hierarchy, level: int = 0) -> np.ndarray:
    """Error propagation I - M^-1 A of the cycle on `level` when the next
    level is solved exactly, as the product of its three stages:
    (I - S A)(I - P A_c^+ P^T A)(I - S A), S the smoother's matrix (dense;
    tiny levels only)."""
    lev = h.levels[level]
    A = lev.A.toarray()
    n = A.shape[0]
    dinv = 1.0 / np.diag(A)
    o = h.opts
    S = np.column_stack([chebyshev_smooth(lev.A, dinv, e, o.degree, o.ratio) for e in np.eye(n)])
    P = lev.P.toarray()
    Ac = P.T @ A @ P
    lam, Q = np.linalg.eigh(Ac)
    keep = lam > 1e-10 * lam.max()
    Acp = (Q[:, keep] / lam[keep]) @ Q[:, keep].T
    I = np.eye(n)
    return (I - S @ A) @ (I - P @ Acp @ P.T @ A) @ (I - S @ A)


def level_table(h: Hierarchy) -> list:
    """(n_b, k, nnz of the assembled level operator, kind) per level."""
    return [(lv.n_b, lv.k, lv.A.nnz, lv.kind) for lv in h.levels]
