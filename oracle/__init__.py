"""CPU oracle for the repeated-block finite-volume operators.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the library and its binding never
do.  It shares no code with the HIP library (see ``oracle.c`` for what it
follows).  The heavy loops live in plain C (``oracle.c``, built by
``oracle.build``); this module marshals numpy arrays to and from it and holds
the paper's closed-form performance model (Section 2, Eqs. 2, 3a, 3b, 7).
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


class _Mesh3D(C.Structure):
    _fields_ = [("n_cells", C.c_int), ("n_faces", C.c_int), ("n_walls", C.c_int),
                ("area", C.c_void_p), ("c1", C.c_void_p), ("c2", C.c_void_p),
                ("len", C.c_void_p), ("dist", C.c_void_p),
                ("wcell", C.c_void_p), ("wlen", C.c_void_p), ("wdist", C.c_void_p),
                ("k", C.c_int), ("dz", C.c_double), ("coupling", C.c_int),
                ("dirichlet", C.c_int)]


class _CGStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("status", C.c_int), ("bnorm", C.c_double),
                ("relres_rec", C.c_double), ("relres_true", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        i, d, l64 = C.c_int, C.c_double, C.c_int64
        P = C.POINTER
        L.orc_cart_sizes.argtypes = [i, i, i, i, P(i), P(i), P(i)]
        L.orc_cart_geometry.argtypes = [i, i, d, d, d, d, d, i, i, _dp, _dp, _dp,
                                        _ip, _ip, _dp, _dp, _ip, _dp, _dp]
        L.orc_tri_sizes.argtypes = [i, _dp, i, _ip, P(i), P(i)]
        L.orc_tri_geometry.argtypes = [i, _dp, i, _ip, _dp, _dp, _dp,
                                       _ip, _ip, _dp, _dp, _ip, _dp, _dp]
        m3 = P(_Mesh3D)
        for name in ("orc_n_faces3d", "orc_lap_max_nnz", "orc_div_max_nnz"):
            getattr(L, name).argtypes = [m3]
            getattr(L, name).restype = l64
        for name in ("orc_assemble_lap", "orc_assemble_div", "orc_assemble_grad"):
            getattr(L, name).argtypes = [m3, _lp, _ip, _dp, P(l64)]
        L.orc_face_volumes.argtypes = [m3, _dp]
        L.orc_cell_volumes.argtypes = [m3, _dp]
        for name in ("orc_dense_lap", "orc_dense_div", "orc_dense_grad"):
            getattr(L, name).argtypes = [m3, _dp]
        L.orc_dense_solve.argtypes = [i, _dp, _dp, _dp, i]
        L.orc_spmv.argtypes = [l64, _lp, _ip, _dp, _dp, _dp]
        L.orc_spmv.restype = None
        L.orc_cg.argtypes = [l64, l64, _lp, _ip, _dp, _dp, _dp, i, d, i, i, P(_CGStats)]
        L.orc_threads.argtypes = []
        L.orc_set_threads.argtypes = [i]
        L.orc_set_threads.restype = None
        L.orc_stencil_max_nnz.argtypes = [i, i, i, i]
        L.orc_stencil_max_nnz.restype = l64
        L.orc_assemble_stencil.argtypes = [i, i, d, d, d, d, d, i, i, i, d, i, _lp, _ip, _dp, P(l64)]
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


# --------------------------------------------------------------------------
# Geometry
# --------------------------------------------------------------------------

@dataclass
class Geometry:
    """2D base face graph: cells with areas and centroids, interior faces with
    their two cells, length and centre-to-centre distance, and wall faces."""
    area: np.ndarray
    cx: np.ndarray
    cy: np.ndarray
    c1: np.ndarray
    c2: np.ndarray
    len: np.ndarray
    dist: np.ndarray
    wcell: np.ndarray
    wlen: np.ndarray
    wdist: np.ndarray

    @property
    def n_cells(self):
        return len(self.area)

    @property
    def n_faces(self):
        return len(self.c1)

    @property
    def n_walls(self):
        return len(self.wcell)


def _alloc_geom(nc, nf, nw):
    return Geometry(np.zeros(nc), np.zeros(nc), np.zeros(nc),
                    np.zeros(nf, np.int32), np.zeros(nf, np.int32), np.zeros(nf), np.zeros(nf),
                    np.zeros(nw, np.int32), np.zeros(nw), np.zeros(nw))


def cart_geometry(spec) -> Geometry:
    """Geometry of an ``inputs.CartSpec`` base mesh."""
    L = lib()
    nc, nf, nw = C.c_int(), C.c_int(), C.c_int()
    _check(L.orc_cart_sizes(spec.nx, spec.ny, int(spec.periodic_x), int(spec.periodic_y),
                            C.byref(nc), C.byref(nf), C.byref(nw)), "cart_sizes")
    g = _alloc_geom(nc.value, nf.value, nw.value)
    _check(L.orc_cart_geometry(spec.nx, spec.ny, spec.x0, spec.Lx, spec.y0, spec.y1,
                               spec.stretch, int(spec.periodic_x), int(spec.periodic_y),
                               g.area, g.cx, g.cy, g.c1, g.c2, g.len, g.dist,
                               g.wcell, g.wlen, g.wdist), "cart_geometry")
    return g


def tri_geometry(spec) -> Geometry:
    """Geometry of an ``inputs.TriSpec`` triangle mesh (cells = triangles)."""
    L = lib()
    xy = np.ascontiguousarray(spec.points, dtype=np.float64).ravel()
    tri = np.ascontiguousarray(spec.triangles, dtype=np.int32).ravel()
    npts, ntri = len(spec.points), len(spec.triangles)
    nf, nw = C.c_int(), C.c_int()
    _check(L.orc_tri_sizes(npts, xy, ntri, tri, C.byref(nf), C.byref(nw)), "tri_sizes")
    g = _alloc_geom(ntri, nf.value, nw.value)
    _check(L.orc_tri_geometry(npts, xy, ntri, tri, g.area, g.cx, g.cy, g.c1, g.c2,
                              g.len, g.dist, g.wcell, g.wlen, g.wdist), "tri_geometry")
    return g


def geometry(spec) -> Geometry:
    return tri_geometry(spec) if hasattr(spec, "triangles") else cart_geometry(spec)


# --------------------------------------------------------------------------
# Extruded 3D mesh and its assembled operators
# --------------------------------------------------------------------------

NONE, PERIODIC_Z = 0, 1


class Mesh3D:
    """The base mesh extruded into ``k`` planes of spacing ``dz``.

    ``coupling`` is ``NONE`` (k independent planes) or ``PERIODIC_Z`` (faces
    between neighbouring planes, periodic).  Vectors are plane-major: cell c of
    plane l sits at ``l * n_b + c``.
    """

    def __init__(self, geom: Geometry, k: int, dz: float, coupling: int = PERIODIC_Z,
                 dirichlet: bool = False):
        self.g = geom
        self.k, self.dz, self.coupling, self.dirichlet = int(k), float(dz), int(coupling), bool(dirichlet)
        self._s = _Mesh3D(geom.n_cells, geom.n_faces, geom.n_walls,
                          geom.area.ctypes.data, geom.c1.ctypes.data, geom.c2.ctypes.data,
                          geom.len.ctypes.data, geom.dist.ctypes.data,
                          geom.wcell.ctypes.data, geom.wlen.ctypes.data, geom.wdist.ctypes.data,
                          self.k, self.dz, self.coupling, int(self.dirichlet))
        self.n_b = geom.n_cells
        self.N = self.n_b * self.k
        self.F3 = int(lib().orc_n_faces3d(C.byref(self._s)))

    @property
    def singular(self) -> bool:
        """True when L has the constant null space (no Dirichlet wall acts)."""
        return not (self.dirichlet and self.g.n_walls > 0)

    def _asm(self, fn, n_rows, n_cols, max_nnz):
        ptr = np.zeros(n_rows + 1, np.int64)
        col = np.zeros(max(max_nnz, 1), np.int32)
        val = np.zeros(max(max_nnz, 1))
        nnz = C.c_int64()
        _check(fn(C.byref(self._s), ptr, col, val, C.byref(nnz)), fn.__name__)
        n = nnz.value
        return sp.csr_matrix((val[:n], col[:n], ptr), shape=(n_rows, n_cols))

    def lap(self) -> sp.csr_matrix:
        L = lib()
        return self._asm(L.orc_assemble_lap, self.N, self.N, int(L.orc_lap_max_nnz(C.byref(self._s))))

    def div(self) -> sp.csr_matrix:
        L = lib()
        return self._asm(L.orc_assemble_div, self.N, self.F3, int(L.orc_div_max_nnz(C.byref(self._s))))

    def grad(self) -> sp.csr_matrix:
        L = lib()
        return self._asm(L.orc_assemble_grad, self.F3, self.N, int(L.orc_div_max_nnz(C.byref(self._s))))

    def face_volumes(self) -> np.ndarray:
        out = np.zeros(self.F3)
        lib().orc_face_volumes(C.byref(self._s), out)
        return out

    def cell_volumes(self) -> np.ndarray:
        out = np.zeros(self.N)
        lib().orc_cell_volumes(C.byref(self._s), out)
        return out

    def dense_lap(self) -> np.ndarray:
        out = np.zeros(self.N * self.N)
        _check(lib().orc_dense_lap(C.byref(self._s), out), "dense_lap")
        return out.reshape(self.N, self.N)

    def dense_div(self) -> np.ndarray:
        out = np.zeros(self.N * self.F3)
        _check(lib().orc_dense_div(C.byref(self._s), out), "dense_div")
        return out.reshape(self.N, self.F3)

    def dense_grad(self) -> np.ndarray:
        out = np.zeros(self.N * self.F3)
        _check(lib().orc_dense_grad(C.byref(self._s), out), "dense_grad")
        return out.reshape(self.F3, self.N)

    def n_groups(self) -> int:
        """Number of independent null-space groups of L (0 when nonsingular)."""
        if not self.singular:
            return 0
        return 1 if (self.coupling == PERIODIC_Z and self.k >= 2) else self.k

    def z_centres(self) -> np.ndarray:
        return (np.arange(self.k) + 0.5) * self.dz


def stencil_lap(spec, k: int, dz: float, stencil: int) -> sp.csr_matrix:
    """The 13- or 27-point operator of a Cartesian base ``spec`` repeated in k
    periodic planes (see ``orc_assemble_stencil`` in oracle.c), plane-major."""
    L = lib()
    n = spec.nx * spec.ny * k
    cap = int(L.orc_stencil_max_nnz(spec.nx, spec.ny, k, stencil))
    ptr = np.zeros(n + 1, np.int64)
    col = np.zeros(cap, np.int32)
    val = np.zeros(cap)
    nnz = C.c_int64()
    _check(L.orc_assemble_stencil(spec.nx, spec.ny, spec.x0, spec.Lx, spec.y0, spec.y1, spec.stretch,
                                  int(spec.periodic_x), int(spec.periodic_y), k, float(dz), int(stencil),
                                  ptr, col, val, C.byref(nnz)), "assemble_stencil")
    m = nnz.value
    return sp.csr_matrix((val[:m], col[:m], ptr), shape=(n, n))


def threads() -> int:
    """Number of host threads the oracle's OpenMP loops use."""
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Sets the number of host threads of the oracle's OpenMP loops."""
    lib().orc_set_threads(int(n))


def spmv(A: sp.csr_matrix, x: np.ndarray, out: np.ndarray | None = None) -> np.ndarray:
    """y = A x by the oracle's row-sequential CSR loop."""
    A = A.tocsr()
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.shape[0]) if out is None else out
    lib().orc_spmv(A.shape[0], A.indptr.astype(np.int64, copy=False), A.indices.astype(np.int32, copy=False),
                   np.ascontiguousarray(A.data), x, y)
    return y


@dataclass
class CGResult:
    x: np.ndarray
    iters: list
    status: list
    bnorm: list
    relres_rec: list
    relres_true: list


def cg(mesh: Mesh3D, L: sp.csr_matrix, b: np.ndarray, tol: float, max_iter: int = 100000,
       x0: np.ndarray | None = None) -> CGResult:
    """Textbook CG for L x = b on the assembled matrix.

    Coupled planes form one system; independent planes (coupling NONE, or
    k == 1) are solved plane by plane, each to its own tolerance.
    """
    ind = mesh.coupling == NONE or mesh.k == 1
    groups = [(l * mesh.n_b, mesh.n_b) for l in range(mesh.k)] if ind else [(0, mesh.N)]
    x = np.zeros(mesh.N) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    ptr, col, val = L.indptr.astype(np.int64), L.indices.astype(np.int32), np.ascontiguousarray(L.data)
    res = CGResult(x, [], [], [], [], [])
    for r0, n in groups:
        st = _CGStats()
        xs = np.ascontiguousarray(x[r0:r0 + n])
        bs = np.ascontiguousarray(b[r0:r0 + n], dtype=np.float64)
        rc = lib().orc_cg(r0, n, ptr, col, val, bs, xs, int(x0 is not None), tol, max_iter,
                          int(mesh.singular), C.byref(st))
        if rc not in (0, -5):
            raise ValueError(f"oracle cg failed with code {rc}")
        x[r0:r0 + n] = xs
        res.iters.append(st.iters)
        res.status.append(st.status)
        res.bnorm.append(st.bnorm)
        res.relres_rec.append(st.relres_rec)
        res.relres_true.append(st.relres_true)
    return res


def dense_solve(L: np.ndarray, b: np.ndarray, n_groups: int) -> np.ndarray:
    """Direct solve of L x = b (Cholesky of -L, plus the group indicators'
    outer products when L is singular, which pins 1^T x = 0 per group)."""
    n = L.shape[0]
    x = np.zeros(n)
    _check(lib().orc_dense_solve(n, np.ascontiguousarray(L, dtype=np.float64).ravel(),
                                 np.ascontiguousarray(b, dtype=np.float64), x, n_groups),
           "dense_solve")
    return x


def project_mean(v: np.ndarray, n_groups: int) -> np.ndarray:
    """Subtract the plain mean per group (n_groups equal consecutive ranges)."""
    v = np.array(v, dtype=np.float64, copy=True)
    if n_groups <= 0:
        return v
    w = v.reshape(n_groups, -1)
    w -= w.mean(axis=1, keepdims=True)
    return w.ravel()


# --------------------------------------------------------------------------
# Closed-form performance model of Section 2
# --------------------------------------------------------------------------

def ai_spmm(nnz: float, n_r: float, n_c: float, m: float) -> float:
    """Arithmetic intensity of an m-column CSR SpMM, Eq. 2 (8-byte values,
    4-byte indices): flops (2 nnz + 1) m over bytes 12 nnz + 4 (n_r + 1)
    + m (8 n_r + 8 n_c + 8)."""
    return (2 * nnz + 1) * m / (8 * nnz + 4 * nnz + 4 * (n_r + 1) + m * (8 * n_r + 8 * n_c + 8))


def p_spmm_ub(nnz: float, n_r: float, n_c: float, m: float) -> float:
    """Upper speed-up bound, Eq. 3a, read with its bracket closed after the
    3 (nnz + n_r + 1) term (the reading that equals I(m)/I(1) of Eq. 2)."""
    return m * (3 * (nnz + n_r + 1) + 2 * n_c) / (3 * nnz + (1 + 2 * m) * (n_r + 1) + 2 * m * n_c)


def p_spmm_lb(nnz: float, n_r: float, m: float) -> float:
    """Lower speed-up bound, Eq. 3b: zero temporal locality in the input
    vector (every one of the nnz gathers is a fresh 8-byte load per column)."""
    return m * (5 * nnz + 3 * (n_r + 1)) / ((3 + 2 * m) * nnz + (1 + 2 * m) * (n_r + 1))


def p_poisson(p_spmm: float, chi: float) -> float:
    """Poisson speed-up from the SpMM speed-up and the SpMM time weight, Eq. 7."""
    return p_spmm / (chi + (1.0 - chi) * p_spmm)
