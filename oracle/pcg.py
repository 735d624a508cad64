"""Preconditioned CG for the Poisson solve (TEST INFRASTRUCTURE ONLY: the
test suite, the smoke check and the benchmark's CPU-baseline leg may use
it; the library never does).

The paper solves its Poisson equation with CG preconditioned by an adaptive
AMG (Section 4); the cheapest preconditioners that keep every operator an
SpMM are written here in their textbook form, on the assembled matrix:

* Jacobi: z = D^-1 r, D the diagonal of A = -L.
* Chebyshev polynomial: z = p(D^-1 A) D^-1 r, the result of m steps of the
  Chebyshev semi-iteration for D^-1 A z = D^-1 r from z = 0 on the interval
  [b/ratio, b] (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed.,
  Sec. 12.3, Algorithm 12.1).  b = 2 bounds the spectrum of D^-1 A for every
  operator here (Gershgorin: each row of A has off-diagonal magnitudes
  summing to at most its diagonal).  m = 1 is Jacobi scaled by 1/theta.

CG runs on A = -L with right-hand side -b (as the library does), so the
preconditioner sees an SPD matrix.  Singular operators project b (and x at
the end) to zero plain mean per group.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

CHEB_BMAX = 2.0


@dataclass
class PCGResult:
    x: np.ndarray
    iters: list
    status: list
    relres_rec: list
    relres_true: list


def chebyshev_apply(A: sp.csr_matrix, dinv: np.ndarray, r: np.ndarray, degree: int, ratio: float) -> np.ndarray:
    """m = degree steps of the Chebyshev semi-iteration for D^-1 A z = D^-1 r
    from z = 0 on [b/ratio, b], b = CHEB_BMAX (Saad, Algorithm 12.1)."""
    b = CHEB_BMAX
    a = b / ratio
    theta, delta = (b + a) / 2.0, (b - a) / 2.0
    sigma = theta / delta
    rho = 1.0 / sigma
    d = dinv * r / theta
    z = d.copy()
    for _ in range(degree - 1):
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * (r - A @ z))
        z = z + d
        rho = rho_new
    return z


def chebyshev_polynomial(lam: np.ndarray, degree: int, ratio: float) -> np.ndarray:
    """p(lambda) of chebyshev_apply in closed form: the residual polynomial of
    m Chebyshev steps is 1 - lambda p(lambda) = T_m((theta - lambda)/delta) /
    T_m(theta/delta) (Saad, Sec. 12.3), with T_m the Chebyshev polynomial of
    the first kind."""
    b = CHEB_BMAX
    a = b / ratio
    theta, delta = (b + a) / 2.0, (b - a) / 2.0
    T = np.polynomial.chebyshev.Chebyshev.basis(degree)
    res = T((theta - lam) / delta) / T(theta / delta)
    return (1.0 - res) / lam


def pcg(mesh, L: sp.csr_matrix, b: np.ndarray, tol: float, precond: str = "jacobi", degree: int = 1,
        ratio: float = 30.0, max_iter: int = 100000, x0: np.ndarray | None = None, amg_opts=None) -> PCGResult:
    """Textbook preconditioned CG for L x = b; stops when ||r|| <= tol ||b||
    (b after projection), r the recursive residual.  Independent planes
    (coupling NONE, or k == 1) are solved plane by plane.  precond "amg": one
    V-cycle of the aggregation multigrid (oracle/amg.py) of each system."""
    from . import NONE
    ind = mesh.coupling == NONE or mesh.k == 1
    groups = [(l * mesh.n_b, mesh.n_b) for l in range(mesh.k)] if ind else [(0, mesh.N)]
    x = np.zeros(mesh.N) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    out = PCGResult(x, [], [], [], [])
    for r0, n in groups:
        A = (-L[r0:r0 + n, r0:r0 + n]).tocsr()
        diag = A.diagonal()
        dinv = np.where(diag != 0.0, 1.0 / np.where(diag != 0.0, diag, 1.0), 1.0)
        bb = np.array(b[r0:r0 + n], dtype=np.float64)
        if mesh.singular:
            bb -= bb.mean()
        bnorm = np.linalg.norm(bb)
        xs = x[r0:r0 + n].copy()
        if bnorm == 0.0:
            x[r0:r0 + n] = 0.0
            out.iters.append(0), out.status.append(0), out.relres_rec.append(0.0), out.relres_true.append(0.0)
            continue

        if precond == "amg":
            from . import amg as _amg
            hier = _amg.build(A, mesh.n_b, 1 if ind else mesh.k, not ind, amg_opts, columns=mesh.k if ind else 1)

        def prec(v):
            if precond == "amg":
                return _amg.vcycle(hier, v)
            if precond == "none":
                return v.copy()
            if precond == "jacobi":
                return dinv * v
            return chebyshev_apply(A, dinv, v, degree, ratio)

        r = -bb - A @ xs
        z = prec(r)
        p = z.copy()
        rz = float(r @ z)
        rr = float(r @ r)
        it, status = 0, 1
        if np.sqrt(rr) <= tol * bnorm:
            status = 0
        while status == 1 and it < max_iter:
            q = A @ p
            pq = float(p @ q)
            if not (pq > 0.0) or not np.isfinite(pq):
                status = -5
                break
            alpha = rz / pq
            xs += alpha * p
            r -= alpha * q
            rr = float(r @ r)
            it += 1
            if np.sqrt(rr) <= tol * bnorm:
                status = 0
                break
            z = prec(r)
            rz_new = float(r @ z)
            p = z + (rz_new / rz) * p
            rz = rz_new
        if mesh.singular:
            xs -= xs.mean()
        x[r0:r0 + n] = xs
        out.iters.append(it)
        out.status.append(status)
        out.relres_rec.append(np.sqrt(rr) / bnorm)
        out.relres_true.append(np.linalg.norm(bb + (A @ xs)) / bnorm)
    return out
