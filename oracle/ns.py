"""Pieces of the incompressible time step on the extruded mesh (TEST
INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU leg may
use it).

Section 3.1 writes the convective term of the symmetry-preserving
discretisation as C(u_s) = M U_s Pi: the divergence M of the face velocities
U_s = diag(u_s) times the cell values interpolated to the faces.  Pi is the
midpoint interpolation: each face takes the mean of the two cells it joins.
Here Pi is read off the sparsity of M itself (every face column of M holds
its two cells), so the oracle's convective operator depends only on its
already pinned divergence.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def midpoint_interpolation(M: sp.csr_matrix) -> sp.csr_matrix:
    """Pi [faces x cells]: 1/2 at the two cells of every face (faces from a
    cell to itself have no entry in M and get none)."""
    P = abs(M.T).tocsr()
    P.data[:] = 0.5
    P.eliminate_zeros()
    return P


def convective(M: sp.csr_matrix, us: np.ndarray) -> sp.csr_matrix:
    """C(u_s) = M diag(u_s) Pi."""
    return (M @ sp.diags(np.asarray(us, dtype=np.float64)) @ midpoint_interpolation(M)).tocsr()


# --------------------------------------------------------------------------
# The time step: cell velocities (u, v, w), face velocities u_s, Heun RK3
# with a projection per stage (Sections 3 and 4), on assembled matrices.
# --------------------------------------------------------------------------

def face_normals(spec, geom) -> tuple[np.ndarray, np.ndarray]:
    """Unit normals of the in-plane faces, oriented from c1 to c2.  Cartesian
    bases list their x-faces first (normal +x) and then their y-faces (+y);
    triangle faces are perpendicular to the edge the two triangles share."""
    nf = geom.n_faces
    if not hasattr(spec, "triangles"):
        n_x = spec.ny * (spec.nx if spec.periodic_x else spec.nx - 1)
        nx = np.zeros(nf)
        ny = np.zeros(nf)
        nx[:n_x] = 1.0
        ny[n_x:] = 1.0
        return nx, ny
    tri = np.asarray(spec.triangles)
    pts = np.asarray(spec.points, dtype=np.float64)
    nx, ny = np.zeros(nf), np.zeros(nf)
    for f in range(nf):
        a, b = int(geom.c1[f]), int(geom.c2[f])
        shared = sorted(set(tri[a].tolist()) & set(tri[b].tolist()))
        p, q = pts[shared[0]], pts[shared[1]]
        t = q - p
        n = np.array([t[1], -t[0]]) / np.hypot(t[0], t[1])
        d = np.array([geom.cx[b] - geom.cx[a], geom.cy[b] - geom.cy[a]])
        if n @ d < 0:
            n = -n
        nx[f], ny[f] = n
    return nx, ny


def interp_cell_to_face(m3, nx: np.ndarray, ny: np.ndarray) -> sp.csr_matrix:
    """Gamma_cs [F3 x 3N]: in-plane face f of plane l takes n_f . (u_c1 +
    u_c2) / 2; the face above cell c of plane l takes (w_l + w_{l+1 mod k}) / 2."""
    g, k, nb, N = m3.g, m3.k, m3.n_b, m3.N
    rows, cols, vals = [], [], []
    F = g.n_faces
    for l in range(k):
        for f in range(F):
            r = l * F + f
            for c in (int(g.c1[f]), int(g.c2[f])):
                rows += [r, r]
                cols += [l * nb + c, N + l * nb + c]
                vals += [0.5 * nx[f], 0.5 * ny[f]]
    nz = m3.F3 - k * F
    if nz:
        for l in range(k):
            for c in range(nb):
                r = k * F + l * nb + c
                rows += [r, r]
                cols += [2 * N + l * nb + c, 2 * N + ((l + 1) % k) * nb + c]
                vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(m3.F3, 3 * N))


class NSOracle:
    """Assembled operators of the time step on one extruded mesh."""

    def __init__(self, spec, m3, visc_m3=None):
        self.m3 = m3
        self.M, self.G, self.L = m3.div(), m3.grad(), m3.lap()
        self.Lv = (visc_m3 or m3).lap()
        nx, ny = face_normals(spec, m3.g)
        self.Gcs = interp_cell_to_face(m3, nx, ny)
        om_c = np.tile(m3.cell_volumes(), 3)
        self.Gsc = (sp.diags(1.0 / om_c) @ self.Gcs.T @ sp.diags(m3.face_volumes())).tocsr()
        self.vol = m3.cell_volumes()

    def rhs(self, U, us, nu):
        C = convective(self.M, us)
        return [(-(C @ u) + nu * (self.Lv @ u)) / self.vol for u in U]

    def project(self, U, cdt, tol):
        ustar = self.Gcs @ np.concatenate(U)
        b = (self.M @ ustar) / cdt
        from . import cg
        phi = cg(self.m3, self.L, b, tol).x
        gp = self.G @ phi
        us = ustar - cdt * gp
        corr = self.Gsc @ gp
        N = self.m3.N
        return [U[d] - cdt * corr[d * N:(d + 1) * N] for d in range(3)], us, phi

    def step(self, U, us, dt, nu, tol=1e-13):
        """Heun RK3 with a projection after every stage."""
        R1 = self.rhs(U, us, nu)
        U2, us2, _ = self.project([U[d] + dt / 3 * R1[d] for d in range(3)], dt / 3, tol)
        R2 = self.rhs(U2, us2, nu)
        U3, us3, _ = self.project([U[d] + 2 * dt / 3 * R2[d] for d in range(3)], 2 * dt / 3, tol)
        R3 = self.rhs(U3, us3, nu)
        return self.project([U[d] + dt * (R1[d] / 4 + 3 * R3[d] / 4) for d in range(3)], dt, tol)
