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
