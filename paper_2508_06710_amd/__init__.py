"""Python binding of libfvx: repeated-block finite-volume operators on MI355X.

Argument marshalling only.  Every operator application and solve runs in the
HIP kernels of libfvx.so; torch supplies device memory and the current
stream.  See include/fvx.h for the operations, layouts and error behaviour.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import _lib
from ._lib import (DIRICHLET, F32, F64, GUESS_GIVEN, GUESS_NET, GUESS_ZERO, MIXED, NEUMANN, NONE,  # noqa: F401
                   PERIODIC_Z, PRECOND_AMG, PRECOND_CHEBYSHEV, PRECOND_JACOBI, PRECOND_NONE, LAUNCH_PHASES,
                   LAUNCH_GRAPH, FvxError, SolveOpts, SolveStats,
                   Tile, check, lib)

__all__ = ["Mesh", "hilbert_order", "Operator", "GuessNet", "SparseMatrix", "FvxError", "F64", "F32", "MIXED", "NONE", "PERIODIC_Z",
           "NEUMANN", "DIRICHLET", "PRECOND_NONE", "PRECOND_JACOBI", "PRECOND_CHEBYSHEV", "PRECOND_AMG", "LAUNCH_PHASES",
           "LAUNCH_GRAPH", "Amg", "lib"]


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def hilbert_order(x, y):
    """Host permutation that visits the points (x[i], y[i]) along a Hilbert
    curve over their bounding box (fvx_hilbert_order)."""
    xs = np.ascontiguousarray(x, dtype=np.float64)
    ys = np.ascontiguousarray(y, dtype=np.float64)
    if xs.shape != ys.shape or xs.ndim != 1:
        raise ValueError("x and y must be 1-D arrays of one length")
    perm = np.empty(len(xs), dtype=np.int32)
    check(lib().fvx_hilbert_order(len(xs), _np_ptr(xs), _np_ptr(ys), _np_ptr(perm)), "fvx_hilbert_order")
    return perm


class Mesh:
    """A 2D finite-volume base mesh (host object).  cell_perm: for a mesh
    whose cells were renumbered at build time (order="hilbert"), new cell i is
    cell cell_perm[i] of the input; None otherwise."""

    def __init__(self, handle: C.c_void_p, keep=(), cell_perm=None):
        self._h = handle
        self._keep = keep
        self.cell_perm = cell_perm

    @classmethod
    def cartesian(cls, nx, ny, x0=0.0, Lx=1.0, y0=0.0, y1=1.0, stretch=0.0, periodic_x=True,
                  periodic_y=False):
        h = C.c_void_p()
        check(lib().fvx_mesh_cartesian(nx, ny, x0, Lx, y0, y1, stretch, int(periodic_x),
                                       int(periodic_y), C.byref(h)), "fvx_mesh_cartesian")
        return cls(h)

    @classmethod
    def from_spec(cls, spec, order=None):
        """From an ``inputs.CartSpec`` or ``inputs.TriSpec`` (order: see
        ``triangles``; a Cartesian base is already in line order)."""
        if hasattr(spec, "triangles"):
            return cls.triangles(spec.points, spec.triangles, order=order)
        return cls.cartesian(spec.nx, spec.ny, spec.x0, spec.Lx, spec.y0, spec.y1, spec.stretch,
                             spec.periodic_x, spec.periodic_y)

    @classmethod
    def triangles(cls, points, tris, order=None):
        """Triangle base; order="hilbert" numbers the cells along a Hilbert
        curve of their vertex centroids (fvx_hilbert_order) and keeps the
        permutation in cell_perm."""
        xy = np.ascontiguousarray(points, dtype=np.float64)
        tri = np.ascontiguousarray(tris, dtype=np.int32)
        perm = None
        if order == "hilbert":
            cen = xy[tri].mean(axis=1)
            perm = hilbert_order(cen[:, 0], cen[:, 1])
            tri = np.ascontiguousarray(tri[perm])
        elif order is not None:
            raise ValueError(f"unknown cell order {order!r}")
        h = C.c_void_p()
        check(lib().fvx_mesh_triangles(len(xy), _np_ptr(xy), len(tri), _np_ptr(tri), C.byref(h)),
              "fvx_mesh_triangles")
        return cls(h, cell_perm=perm)

    @classmethod
    def from_faces(cls, area, c1, c2, length, dist, wcell=None, wlen=None, wdist=None,
                   cx=None, cy=None):
        a = np.ascontiguousarray(area, np.float64)
        f1, f2 = np.ascontiguousarray(c1, np.int32), np.ascontiguousarray(c2, np.int32)
        ln, ds = np.ascontiguousarray(length, np.float64), np.ascontiguousarray(dist, np.float64)
        nw = 0 if wcell is None else len(wcell)
        wc = None if wcell is None else np.ascontiguousarray(wcell, np.int32)
        wl = None if wlen is None else np.ascontiguousarray(wlen, np.float64)
        wd = None if wdist is None else np.ascontiguousarray(wdist, np.float64)
        cxa = None if cx is None else np.ascontiguousarray(cx, np.float64)
        cya = None if cy is None else np.ascontiguousarray(cy, np.float64)
        h = C.c_void_p()
        check(lib().fvx_mesh_from_faces(len(a), _np_ptr(a), _np_ptr(cxa), _np_ptr(cya), len(f1),
                                        _np_ptr(f1), _np_ptr(f2), _np_ptr(ln), _np_ptr(ds), nw,
                                        _np_ptr(wc), _np_ptr(wl), _np_ptr(wd), C.byref(h)),
              "fvx_mesh_from_faces")
        return cls(h)

    def info(self):
        n = [C.c_int64() for _ in range(3)]
        check(lib().fvx_mesh_info(self._h, *[C.byref(v) for v in n]), "fvx_mesh_info")
        return tuple(v.value for v in n)

    @property
    def n_cells(self):
        return self.info()[0]

    @property
    def n_faces(self):
        return self.info()[1]

    def centroids(self):
        n = self.n_cells
        cx, cy = np.zeros(n), np.zeros(n)
        check(lib().fvx_mesh_centroids(self._h, _np_ptr(cx), _np_ptr(cy)), "fvx_mesh_centroids")
        return cx, cy

    def refine(self, rf=2):
        """The Cartesian mesh with every cell split into rf x rf children."""
        h = C.c_void_p()
        check(lib().fvx_mesh_refine(self._h, int(rf), C.byref(h)), "fvx_mesh_refine")
        return Mesh(h)

    def prolongation(self, rf=2):
        """Host CSR (ptr, col, val) of the coarse-to-fine state mapping onto refine(rf)."""
        nnz = C.c_int64()
        check(lib().fvx_refine_prolongation(self._h, int(rf), C.byref(nnz), None, None, None),
              "fvx_refine_prolongation")
        n_fine = self.n_cells * rf * rf
        ptr = np.zeros(n_fine + 1, np.int32)
        col = np.zeros(max(nnz.value, 1), np.int32)
        val = np.zeros(max(nnz.value, 1))
        check(lib().fvx_refine_prolongation(self._h, int(rf), C.byref(nnz), _np_ptr(ptr), _np_ptr(col),
                                            _np_ptr(val)), "fvx_refine_prolongation")
        return ptr, col[:nnz.value], val[:nnz.value]

    def faces(self):
        nc, nf, _ = self.info()
        area = np.zeros(nc)
        c1, c2 = np.zeros(nf, np.int32), np.zeros(nf, np.int32)
        ln, ds = np.zeros(nf), np.zeros(nf)
        check(lib().fvx_mesh_faces(self._h, _np_ptr(area), _np_ptr(c1), _np_ptr(c2), _np_ptr(ln),
                                   _np_ptr(ds)), "fvx_mesh_faces")
        return area, c1, c2, ln, ds

    def __del__(self):
        if getattr(self, "_h", None) and lib is not None:
            try:
                lib().fvx_mesh_destroy(self._h)
            except Exception:
                pass
            self._h = None


_DT = {F64: "float64", F32: "float32"}


def expand_csr(mesh: Mesh, k: int, dz: float, coupling: int = PERIODIC_Z, wall_bc: int = NEUMANN, stencil: int = 7):
    """Host: the assembled 3D Laplacian I_k (x) A_b + C as CSR arrays (ptr, col, val)."""
    d = _lib.OpDesc()
    d.k, d.coupling, d.dz, d.wall_bc, d.with_f32 = int(k), int(coupling), float(dz), int(wall_bc), 0
    d.stencil = int(stencil)
    nnz = C.c_int64()
    check(lib().fvx_expand_csr(mesh._h, C.byref(d), C.byref(nnz), None, None, None), "fvx_expand_csr")
    ptr = np.zeros(k * mesh.n_cells + 1, np.int32)
    col = np.zeros(max(nnz.value, 1), np.int32)
    val = np.zeros(max(nnz.value, 1))
    check(lib().fvx_expand_csr(mesh._h, C.byref(d), C.byref(nnz), _np_ptr(ptr), _np_ptr(col), _np_ptr(val)),
          "fvx_expand_csr")
    return ptr, col[:nnz.value], val[:nnz.value]


class Operator:
    """Repeated-block operator L = I_k (x) A_b + C (plus M_b, G_b) on the device."""

    def __init__(self, mesh: Mesh, k: int, dz: float, coupling: int = PERIODIC_Z,
                 wall_bc: int = NEUMANN, with_f32: bool = True, device=None, stream=None, stencil: int = 7):
        torch = _torch()
        self.mesh = mesh
        self.device = torch.device(device if device is not None else "cuda")
        d = _lib.OpDesc()
        d.k, d.coupling, d.dz, d.wall_bc, d.with_f32 = int(k), int(coupling), float(dz), int(wall_bc), int(with_f32)
        d.stencil = int(stencil)
        self.stencil = int(stencil) if stencil in (13, 27) else 7
        self._desc = d
        nbytes = C.c_size_t()
        check(lib().fvx_op_bytes(mesh._h, C.byref(d), C.byref(nbytes)), "fvx_op_bytes")
        self._mem = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        check(lib().fvx_op_create(mesh._h, C.byref(d), _ptr(self._mem), nbytes.value, _stream(stream),
                                  C.byref(h)), "fvx_op_create")
        self._h = h
        nb, fb, kk, ld, nnz = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int32(), C.c_int64()
        check(lib().fvx_op_shape(h, C.byref(nb), C.byref(fb), C.byref(kk), C.byref(ld), C.byref(nnz)),
              "fvx_op_shape")
        self.n_b, self.F_b, self.k, self.ld, self.nnz_b = nb.value, fb.value, kk.value, ld.value, nnz.value
        self.coupling, self.dz, self.wall_bc = int(coupling), float(dz), int(wall_bc)
        self.zfaces = coupling == PERIODIC_Z and k >= 2
        self.singular = bool(lib().fvx_op_singular(h))
        self.op_bytes = int(nbytes.value)
        self._ws = {}

    # ---- buffers -------------------------------------------------------
    def empty(self, rows: int | None = None, dtype=F64):
        torch = _torch()
        n = self.n_b if rows is None else rows
        return torch.empty((max(n, 1), self.ld), dtype=getattr(torch, _DT[dtype]), device=self.device)

    def zeros(self, rows: int | None = None, dtype=F64):
        t = self.empty(rows, dtype)
        t.zero_()
        return t

    def to_rows(self, plane_major, rows: int | None = None, dtype=F64):
        """Plane-major host or device vector [k * n] -> device [n][ld] (via fvx_pack)."""
        torch = _torch()
        n = self.n_b if rows is None else rows
        src = torch.as_tensor(plane_major, dtype=getattr(torch, _DT[dtype])).to(self.device).contiguous()
        dst = self.zeros(n, dtype)
        check(lib().fvx_pack(self._h, dtype, n, _ptr(src), _ptr(dst), _stream()), "fvx_pack")
        return dst

    def to_planes(self, rows_t, rows: int | None = None, dtype=F64):
        """Device [n][ld] -> plane-major numpy vector [k * n] (via fvx_unpack)."""
        torch = _torch()
        n = self.n_b if rows is None else rows
        dst = torch.empty(self.k * n, dtype=getattr(torch, _DT[dtype]), device=self.device)
        check(lib().fvx_unpack(self._h, dtype, n, _ptr(rows_t), _ptr(dst), _stream()), "fvx_unpack")
        torch.cuda.synchronize(self.device)
        return dst.cpu().numpy()

    # ---- tiles ----------------------------------------------------------
    def get_tile(self, dtype=F64):
        t = Tile()
        check(lib().fvx_op_get_tile(self._h, dtype, C.byref(t)), "fvx_op_get_tile")
        return t.as_tuple()

    def set_tile(self, vec, lanes_per_row, block=256, xcd_remap=1, max_blocks=0, stage_lds=0, nt_store=0,
                 dtype=F64):
        t = Tile(int(vec), int(lanes_per_row), int(block), int(xcd_remap), int(max_blocks), int(stage_lds),
                 int(nt_store))
        check(lib().fvx_op_set_tile(self._h, dtype, C.byref(t)), "fvx_op_set_tile")

    def tune(self, dtype=F64, scratch_bytes=None, reps=3, max_results=512, stream=None):
        """Times candidate SpMM tiles on the device and keeps the fastest.
        Returns [(tile tuple, us per launch), ...] in the order tried."""
        torch = _torch()
        esize = 8 if dtype == F64 else 4
        pair = 2 * self.n_b * self.ld * esize
        nbytes = max(pair, int(scratch_bytes) if scratch_bytes else pair)
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        res = (_lib.TuneResult * max_results)()
        n = C.c_int()
        check(lib().fvx_tune(self._h, dtype, _ptr(scratch), nbytes, int(reps), _stream(stream), res, max_results,
                             C.byref(n)), "fvx_tune")
        return [(res[i].tile.as_tuple(), res[i].us) for i in range(min(n.value, max_results))]

    def get_cg_tile(self, dtype=F64):
        t = Tile()
        check(lib().fvx_op_get_cg_tile(self._h, dtype, C.byref(t)), "fvx_op_get_cg_tile")
        return t.as_tuple()

    def set_cg_tile(self, vec=0, lanes_per_row=1, block=0, xcd_remap=1, max_blocks=0, lines=0, dtype=F64):
        """CG launch tile (block 0 restores the default); lines = 1 selects the
        line tiles of the iteration kernels on Cartesian bases."""
        t = Tile(int(vec), int(lanes_per_row), int(block), int(xcd_remap), int(max_blocks), int(lines), 0)
        check(lib().fvx_op_set_cg_tile(self._h, dtype, C.byref(t)), "fvx_op_set_cg_tile")

    def tune_cg(self, dtype=F64, iters=40, max_results=64, stream=None):
        """Times CG iterations for candidate CG tiles and keeps the fastest.
        Returns [(tile tuple, us per iteration), ...] in the order tried."""
        torch = _torch()
        nbytes = C.c_size_t()
        check(lib().fvx_tune_cg_bytes(self._h, dtype, C.byref(nbytes)), "fvx_tune_cg_bytes")
        ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        res = (_lib.TuneResult * max_results)()
        n = C.c_int()
        check(lib().fvx_tune_cg(self._h, dtype, _ptr(ws), nbytes.value, int(iters), _stream(stream), res,
                                max_results, C.byref(n)), "fvx_tune_cg")
        return [(res[i].tile.as_tuple(), res[i].us) for i in range(min(n.value, max_results))]

    def tune_cg_cached(self, dtype=F64, cache_path=None, iters=40, stream=None):
        """CG tile through a tile cache file (fvx_tune_cg_cached: the keys of
        tune_cached prefixed 'cg|', with the coupling in place of the stencil).
        Returns (tile, "cache" or "tuned")."""
        torch = _torch()
        nbytes = C.c_size_t()
        check(lib().fvx_tune_cg_bytes(self._h, dtype, C.byref(nbytes)), "fvx_tune_cg_bytes")
        ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        t = Tile()
        hit = C.c_int()
        check(lib().fvx_tune_cg_cached(self._h, dtype, os.fsencode(cache_path) if cache_path else None, _ptr(ws),
                                       nbytes.value, int(iters), _stream(stream), C.byref(t), C.byref(hit)),
              "fvx_tune_cg_cached")
        return t.as_tuple(), "cache" if hit.value else "tuned"

    # ---- operators --------------------------------------------------------
    def lap(self, X, Y=None, colscale=None, dtype=None, stream=None):
        dt = dtype if dtype is not None else (F32 if str(X.dtype).endswith("float32") else F64)
        Y = self.empty(dtype=dt) if Y is None else Y
        check(lib().fvx_lap(self._h, dt, _ptr(X), _ptr(Y), _ptr(colscale), _stream(stream)), "fvx_lap")
        return Y

    def lap_many(self, Xs, Ys, dtype=None, stream=None):
        """Y[i] = L X[i] for every pair, launched back to back from C."""
        dt = dtype if dtype is not None else (F32 if str(Xs[0].dtype).endswith("float32") else F64)
        n = len(Xs)
        xa = (C.c_void_p * n)(*[x.data_ptr() for x in Xs])
        ya = (C.c_void_p * n)(*[y.data_ptr() for y in Ys])
        check(lib().fvx_lap_many(self._h, dt, n, xa, ya, _stream(stream)), "fvx_lap_many")
        return Ys

    def _tile_key(self, dtype):
        torch = _torch()
        arch = getattr(torch.cuda.get_device_properties(self.device), "gcnArchName", "unknown").split(":")[0]
        return (f"{arch}|{'f64' if dtype == F64 else 'f32'}|k={self.k}|ld={self.ld}|n_b={self.n_b}|nnz_b={self.nnz_b}"
                f"|stencil={self.stencil}")

    def remember_tile(self, tile, cache_path, dtype=F64, note="refined"):
        """Stores a tile chosen outside the autotuner in the tile cache."""
        import json
        import os
        if not cache_path:
            return
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as fh:
                cache = json.load(fh)
        entry = cache.get(self._tile_key(dtype), {})
        entry.update({"tile": list(tile), "source": note})
        cache[self._tile_key(dtype)] = entry
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)

    def tune_cached(self, dtype=F64, cache_path=None, scratch_bytes=int(1.1 * 2 ** 30), reps=2, stream=None):
        """Autotuned SpMM tile through a tile cache file (fvx_tune_cached: keyed
        by device architecture, precision, k, ld, base rows, base nonzeros,
        stencil).  Returns (tile, "cache" or "tuned")."""
        torch = _torch()
        es = 8 if dtype == F64 else 4
        pair = 2 * self.n_b * self.ld * es
        nbytes = max(pair, min(int(scratch_bytes), 512 * pair))
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        t = Tile()
        hit = C.c_int()
        check(lib().fvx_tune_cached(self._h, dtype, os.fsencode(cache_path) if cache_path else None, _ptr(scratch),
                                    nbytes, int(reps), _stream(stream), C.byref(t), C.byref(hit)), "fvx_tune_cached")
        return t.as_tuple(), "cache" if hit.value else "tuned"

    def div(self, Uf, Wz=None, D=None, dtype=None, stream=None):
        dt = dtype if dtype is not None else (F32 if str(Uf.dtype).endswith("float32") else F64)
        D = self.empty(dtype=dt) if D is None else D
        check(lib().fvx_div(self._h, dt, _ptr(Uf), _ptr(Wz), _ptr(D), _stream(stream)), "fvx_div")
        return D

    def convect(self, Uf, Wz, Phi, Out=None, dtype=None, stream=None):
        """Out = C(u_s) Phi = M U_s Pi Phi (fvx_convect)."""
        dt = dtype if dtype is not None else (F32 if str(Phi.dtype).endswith("float32") else F64)
        Out = self.empty(dtype=dt) if Out is None else Out
        check(lib().fvx_convect(self._h, dt, _ptr(Uf), _ptr(Wz), _ptr(Phi), _ptr(Out), _stream(stream)),
              "fvx_convect")
        return Out

    def grad_axpy(self, alpha, P, Gf, Gz=None, dtype=None, stream=None):
        """Gf += alpha * G P (and Gz on the faces between planes)."""
        dt = dtype if dtype is not None else (F32 if str(P.dtype).endswith("float32") else F64)
        check(lib().fvx_grad_axpy(self._h, dt, float(alpha), _ptr(P), _ptr(Gf), _ptr(Gz), _stream(stream)),
              "fvx_grad_axpy")
        return Gf, Gz

    def grad(self, P, Gf=None, Gz=None, dtype=None, stream=None):
        dt = dtype if dtype is not None else (F32 if str(P.dtype).endswith("float32") else F64)
        Gf = self.empty(self.F_b, dt) if Gf is None else Gf
        if Gz is None and self.zfaces:
            Gz = self.empty(dtype=dt)
        check(lib().fvx_grad(self._h, dt, _ptr(P), _ptr(Gf), _ptr(Gz), _stream(stream)), "fvx_grad")
        return Gf, Gz

    # ---- solves -----------------------------------------------------------
    def solve_opts(self, rtol=1e-8, max_iter=100000, precision=F64, inner_rtol=1e-4, max_outer=50,
                   guess=GUESS_ZERO, poll_every=64, precond=PRECOND_NONE, cheb_degree=8, cheb_ratio=300.0, amg=None,
                   launch=None):
        """Solve options; amg: an Amg hierarchy of this operator (sets the
        AMG preconditioner unless precond is given otherwise); launch:
        LAUNCH_PHASES or LAUNCH_GRAPH (None: the library's default)."""
        o = SolveOpts()
        check(lib().fvx_solve_opts_default(C.byref(o)), "fvx_solve_opts_default")
        o.rtol, o.max_iter, o.precision = float(rtol), int(max_iter), int(precision)
        o.inner_rtol, o.max_outer, o.guess, o.poll_every = float(inner_rtol), int(max_outer), int(guess), int(poll_every)
        o.precond, o.cheb_degree, o.cheb_ratio = int(precond), int(cheb_degree), float(cheb_ratio)
        if launch is not None:
            o.launch = int(launch)
        if amg is not None:
            o.amg = amg._h.value
            if precond == PRECOND_NONE:
                o.precond = PRECOND_AMG
        return o

    def workspace(self, opts):
        torch = _torch()
        nbytes = C.c_size_t()
        check(lib().fvx_solve_bytes(self._h, C.byref(opts), C.byref(nbytes)), "fvx_solve_bytes")
        key = (int(opts.precision), int(opts.precond == PRECOND_CHEBYSHEV and opts.cheb_degree > 1),
               int(opts.amg or 0) if opts.precond == PRECOND_AMG else 0)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes.value:
            ws = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def solve(self, B, X=None, stream=None, allow_not_converged=False, **kw):
        """Solves L x = b (B, X: device [n_b][ld] float64).  Returns (X, stats dict)."""
        opts = self.solve_opts(**kw)
        if X is None:
            X = self.zeros()
        ws = self.workspace(opts)
        st = SolveStats()
        rc = lib().fvx_poisson_solve(self._h, _ptr(B), _ptr(X), C.byref(opts), _ptr(ws), ws.numel(),
                                     C.byref(st), _stream(stream))
        allow = (0, 1) if allow_not_converged else (0,)
        check(rc, "fvx_poisson_solve", allow)
        return X, st.as_dict()

    def solve_noalloc(self, B, X=None, stream=None, allow_not_converged=False, **kw):
        """The same solve on the library's built-in device scratch
        (fvx_poisson_solve_noalloc): no workspace is allocated."""
        opts = self.solve_opts(**kw)
        if X is None:
            X = self.zeros()
        st = SolveStats()
        rc = lib().fvx_poisson_solve_noalloc(self._h, _ptr(B), _ptr(X), C.byref(opts), C.byref(st), _stream(stream))
        check(rc, "fvx_poisson_solve_noalloc", (0, 1) if allow_not_converged else (0,))
        return X, st.as_dict()

    def ns_step(self, U, Uf, Wz, P, dt, nu, visc=None, stream=None, allow_not_converged=False, **kw):
        """One Heun-RK3 projection step (fvx_ns_step): U = [u, v, w] device
        [n_b][ld] tensors, Uf/Wz face velocities, P pressure; all updated in
        place.  Returns the stats dict (iters summed over the 3 projections)."""
        torch = _torch()
        opts = self.solve_opts(**kw)
        nbytes = C.c_size_t()
        check(lib().fvx_ns_step_bytes(self._h, C.byref(opts), C.byref(nbytes)), "fvx_ns_step_bytes")
        key = ("ns", int(nbytes.value))
        ws = self._ws.get(key)
        if ws is None:
            ws = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        ua = (C.c_void_p * 3)(*[u.data_ptr() for u in U])
        st = SolveStats()
        rc = lib().fvx_ns_step(self._h, None if visc is None else visc._h, ua, _ptr(Uf), _ptr(Wz), _ptr(P),
                               float(dt), float(nu), C.byref(opts), _ptr(ws), ws.numel(), C.byref(st),
                               _stream(stream))
        check(rc, "fvx_ns_step", (0, 1) if allow_not_converged else (0,))
        return st.as_dict()

    @classmethod
    def _borrow(cls, handle, owner, mesh=None):
        """An Operator view of a handle owned by `owner` (a multigrid level)."""
        self = cls.__new__(cls)
        self.mesh, self._owner, self._borrowed = mesh, owner, True
        self.device = owner.device
        self._h = C.c_void_p(handle)
        nb, fb, kk, ld, nnz = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int32(), C.c_int64()
        check(lib().fvx_op_shape(self._h, C.byref(nb), C.byref(fb), C.byref(kk), C.byref(ld), C.byref(nnz)),
              "fvx_op_shape")
        self.n_b, self.F_b, self.k, self.ld, self.nnz_b = nb.value, fb.value, kk.value, ld.value, nnz.value
        self.stencil, self.coupling, self.dz, self.wall_bc = 7, owner.op.coupling, 1.0, owner.op.wall_bc
        self.zfaces = self.coupling == PERIODIC_Z and self.k >= 2
        self.singular = bool(lib().fvx_op_singular(self._h))
        self.op_bytes = 0
        self._ws = {}
        return self

    def __del__(self):
        if getattr(self, "_h", None) and not getattr(self, "_borrowed", False):
            try:
                lib().fvx_op_destroy(self._h)
            except Exception:
                pass
            self._h = None


class Amg:
    """Aggregation multigrid hierarchy of an operator (fvx_amg_*): every
    level an operator of the same repeated-block form.  Pass it to
    Operator.solve(amg=...) to precondition CG with one V-cycle.
    mode_cells (None: the library's default, 2048; 0: off) lets coarsening
    stop at the first level of at most that many base cells whose solve per
    plane mode fits the library's term budget; coarsest_modes reports how
    that level is solved (0: one dense pseudo-inverse)."""

    def __init__(self, op: Operator, degree=2, ratio=8.0, beta=0.75, z_rule=1.0, coarse_max=2048, max_levels=16,
                 mode_cells=None, stream=None):
        torch = _torch()
        if op.mesh is None:
            raise ValueError("the operator's mesh is needed to build its multigrid")
        o = _lib.AmgOpts()
        check(lib().fvx_amg_opts_default(C.byref(o)), "fvx_amg_opts_default")
        o.degree, o.ratio, o.beta, o.z_rule = int(degree), float(ratio), float(beta), float(z_rule)
        o.coarse_max, o.max_levels = int(coarse_max), int(max_levels)
        if mode_cells is not None:        # None: the library's default
            o.mode_cells = int(mode_cells)
        nbytes = C.c_size_t()
        check(lib().fvx_amg_bytes(op.mesh._h, op._h, C.byref(o), C.byref(nbytes)), "fvx_amg_bytes")
        self.op, self.device = op, op.device
        self._mem = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        check(lib().fvx_amg_create(op.mesh._h, op._h, C.byref(o), _ptr(self._mem), nbytes.value, _stream(stream),
                                   C.byref(h)), "fvx_amg_create")
        self._h = h
        n = C.c_int32()
        check(lib().fvx_amg_n_levels(h, C.byref(n)), "fvx_amg_n_levels")
        self.n_levels = n.value
        check(lib().fvx_amg_coarsest_modes(h, C.byref(n)), "fvx_amg_coarsest_modes")
        self.coarsest_modes = n.value      # plane modes of the coarsest solve (0: one dense pseudo-inverse)
        self._ws = {}

    def level(self, i):
        """(n_b, k, nnz_b, kind) of level i (kind 0 coarsest, 1 base aggregation, 2 plane merging)."""
        nb, kk, nnz, kind = C.c_int64(), C.c_int32(), C.c_int64(), C.c_int32()
        check(lib().fvx_amg_level(self._h, int(i), C.byref(nb), C.byref(kk), C.byref(nnz), C.byref(kind), None),
              "fvx_amg_level")
        return nb.value, kk.value, nnz.value, kind.value

    def levels(self):
        return [self.level(i) for i in range(self.n_levels)]

    def level_op(self, i):
        """Level i's operator (level 0 is the fine operator itself)."""
        if i == 0:
            return self.op
        h = C.c_void_p()
        check(lib().fvx_amg_level(self._h, int(i), None, None, None, None, C.byref(h)), "fvx_amg_level")
        return Operator._borrow(h.value, self)

    def aggregates(self, i):
        nb = self.level(i)[0]
        out = np.zeros(nb, np.int32)
        check(lib().fvx_amg_aggregates(self._h, int(i), _np_ptr(out)), "fvx_amg_aggregates")
        return out

    def apply(self, R, Z=None, dtype=None, stream=None):
        """One V-cycle Z = M^-1 R (device [n_b][ld] tensors of the fine operator)."""
        torch = _torch()
        dt = dtype if dtype is not None else (F32 if str(R.dtype).endswith("float32") else F64)
        Z = torch.zeros_like(R) if Z is None else Z
        nbytes = C.c_size_t()
        check(lib().fvx_amg_apply_bytes(self._h, dt, C.byref(nbytes)), "fvx_amg_apply_bytes")
        ws = self._ws.get(dt)
        if ws is None or ws.numel() < nbytes.value:
            ws = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
            self._ws[dt] = ws
        check(lib().fvx_amg_apply(self._h, dt, _ptr(R), _ptr(Z), _ptr(ws), ws.numel(), _stream(stream)),
              "fvx_amg_apply")
        return Z

    def __del__(self):
        if getattr(self, "_h", None):
            try:
                lib().fvx_amg_destroy(self._h)
            except Exception:
                pass
            self._h = None


def solve_batch(ops, Bs, Xs=None, stream=None, allow_not_converged=False, **kw):
    """Solves L_i x_i = b_i for several operators at once (fvx_poisson_solve_batch).
    Returns (list of X, list of stats dicts)."""
    torch = _torch()
    n = len(ops)
    opts = ops[0].solve_opts(**kw)
    Xs = [op.zeros() for op in ops] if Xs is None else Xs
    oa = (C.c_void_p * n)(*[op._h.value for op in ops])
    ba = (C.c_void_p * n)(*[b.data_ptr() for b in Bs])
    xa = (C.c_void_p * n)(*[x.data_ptr() for x in Xs])
    nbytes = C.c_size_t()
    check(lib().fvx_solve_batch_bytes(n, oa, C.byref(opts), C.byref(nbytes)), "fvx_solve_batch_bytes")
    ws = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=ops[0].device)
    st = (SolveStats * n)()
    rc = lib().fvx_poisson_solve_batch(n, oa, ba, xa, C.byref(opts), _ptr(ws), ws.numel(), st, _stream(stream))
    check(rc, "fvx_poisson_solve_batch", (0, 1) if allow_not_converged else (0,))
    return Xs, [st[i].as_dict() for i in range(n)]


class SparseMatrix:
    """A general CSR matrix on the device applied to row-major multivectors
    (fvx_sparse_*): Y = diag(colscale) (A X) for k columns at once."""

    def __init__(self, ptr, col, val, n_cols, with_f32=True, device=None, stream=None):
        torch = _torch()
        self.device = torch.device(device if device is not None else "cuda")
        self.ptr = np.ascontiguousarray(ptr, np.int32)
        self.col = np.ascontiguousarray(col, np.int32)
        self.val = np.ascontiguousarray(val, np.float64)
        self.n_rows, self.n_cols = len(self.ptr) - 1, int(n_cols)
        nbytes = C.c_size_t()
        check(lib().fvx_sparse_bytes(self.n_rows, int(self.ptr[-1]), int(with_f32), C.byref(nbytes)),
              "fvx_sparse_bytes")
        self._mem = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        check(lib().fvx_sparse_create(self.n_rows, self.n_cols, _np_ptr(self.ptr), _np_ptr(self.col),
                                      _np_ptr(self.val), int(with_f32), _ptr(self._mem), nbytes.value,
                                      _stream(stream), C.byref(h)), "fvx_sparse_create")
        self._h = h
        self.nnz = int(self.ptr[-1])

    def set_tile(self, vec=0, lanes_per_row=1, block=0, xcd_remap=1, max_blocks=0, nt_store=0, dtype=F64):
        t = Tile(int(vec), int(lanes_per_row), int(block), int(xcd_remap), int(max_blocks), 0, int(nt_store))
        check(lib().fvx_sparse_set_tile(self._h, dtype, C.byref(t)), "fvx_sparse_set_tile")

    def tune(self, X, Y, k=None, reps=5, dtype=None, stream=None):
        """Autotunes the tile for products with X's and Y's strides
        (fvx_sparse_tune); returns the number of candidates timed."""
        dt = dtype if dtype is not None else (F32 if str(X.dtype).endswith("float32") else F64)
        k = X.shape[1] if k is None else int(k)
        n = C.c_int()
        check(lib().fvx_sparse_tune(self._h, dt, k, _ptr(X), X.shape[1], _ptr(Y), Y.shape[1], int(reps),
                                    _stream(stream), None, 0, C.byref(n)), "fvx_sparse_tune")
        return n.value

    def spmm(self, X, Y=None, k=None, colscale=None, dtype=None, stream=None):
        """X: device [n_cols][ldx] tensor; Y: device [n_rows][ldy] (allocated with ldy = ldx if None)."""
        torch = _torch()
        dt = dtype if dtype is not None else (F32 if str(X.dtype).endswith("float32") else F64)
        ldx = X.shape[1]
        k = ldx if k is None else int(k)
        if Y is None:
            Y = torch.zeros((self.n_rows, ldx), dtype=X.dtype, device=X.device)
        check(lib().fvx_sparse_spmm(self._h, dt, k, _ptr(X), ldx, _ptr(Y), Y.shape[1], _ptr(colscale),
                                    _stream(stream)), "fvx_sparse_spmm")
        return Y

    def __del__(self):
        if getattr(self, "_h", None):
            try:
                lib().fvx_sparse_destroy(self._h)
            except Exception:
                pass


class CsrMatrix:
    """An assembled CSR matrix on the device (the no-block-reuse comparator)."""

    def __init__(self, ptr, col, val, device=None):
        torch = _torch()
        dev = torch.device(device if device is not None else "cuda")
        self.n = len(ptr) - 1
        self.nnz = len(col)
        self.ptr = torch.as_tensor(np.ascontiguousarray(ptr, np.int32)).to(dev)
        self.col = torch.as_tensor(np.ascontiguousarray(col, np.int32)).to(dev)
        self.val = torch.as_tensor(np.ascontiguousarray(val, np.float64)).to(dev)
        self.device = dev
        self._ws = None

    def spmv(self, x, y=None, stream=None):
        torch = _torch()
        y = torch.empty(self.n, dtype=torch.float64, device=self.device) if y is None else y
        check(lib().fvx_csr_spmv(self.n, self.nnz, _ptr(self.ptr), _ptr(self.col), _ptr(self.val), _ptr(x), _ptr(y),
                                 _stream(stream)), "fvx_csr_spmv")
        return y

    def solve(self, b, x=None, singular=True, stream=None, allow_not_converged=False, rtol=1e-8,
              max_iter=100000, guess=GUESS_ZERO, poll_every=64):
        torch = _torch()
        o = SolveOpts()
        check(lib().fvx_solve_opts_default(C.byref(o)), "fvx_solve_opts_default")
        o.rtol, o.max_iter, o.guess, o.poll_every = float(rtol), int(max_iter), int(guess), int(poll_every)
        nbytes = C.c_size_t()
        check(lib().fvx_csr_solve_bytes(self.n, C.byref(nbytes)), "fvx_csr_solve_bytes")
        if self._ws is None or self._ws.numel() < nbytes.value:
            self._ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        x = torch.zeros(self.n, dtype=torch.float64, device=self.device) if x is None else x
        st = SolveStats()
        rc = lib().fvx_csr_poisson_solve(self.n, self.nnz, _ptr(self.ptr), _ptr(self.col), _ptr(self.val), _ptr(b),
                                         _ptr(x),
                                         int(singular), C.byref(o), _ptr(self._ws), self._ws.numel(), C.byref(st),
                                         _stream(stream))
        check(rc, "fvx_csr_poisson_solve", (0, 1) if allow_not_converged else (0,))
        return x, st.as_dict()


class GuessNet:
    """Learned initial guess (fvx_net_*): a 4-layer 3x3x3 conv net on the grid
    of a Cartesian base nx x ny extruded into nz planes, with device buffers
    for training batches of up to ``batch`` samples."""

    def __init__(self, nx, ny, nz, batch=16, params=None, device=None, stream=None):
        torch = _torch()
        self.nx, self.ny, self.nz, self.batch = int(nx), int(ny), int(nz), int(batch)
        self.device = torch.device(device if device is not None else "cuda")
        self.cells = self.nx * self.ny * self.nz
        nbytes = C.c_size_t()
        check(lib().fvx_net_bytes(self.nx, self.ny, self.nz, self.batch, C.byref(nbytes)), "fvx_net_bytes")
        self._mem = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        if p is not None and p.size != self.n_params():
            raise ValueError(f"expected {self.n_params()} parameters, got {p.size}")
        h = C.c_void_p()
        check(lib().fvx_net_create(self.nx, self.ny, self.nz, self.batch, _np_ptr(p), _ptr(self._mem),
                                   nbytes.value, _stream(stream), C.byref(h)), "fvx_net_create")
        self._h = h

    @staticmethod
    def n_params():
        return int(lib().fvx_net_n_params())

    def samples(self, ns, channels=2):
        """Uninitialised device float32 buffer [ns][channels][nz][ny][nx]."""
        torch = _torch()
        return torch.empty((ns, channels, self.nz, self.ny, self.nx), dtype=torch.float32, device=self.device)

    def params(self):
        p = np.zeros(self.n_params(), np.float32)
        check(lib().fvx_net_get_params(self._h, _np_ptr(p), None), "fvx_net_get_params")
        return p

    def grads(self):
        g = np.zeros(self.n_params(), np.float32)
        check(lib().fvx_net_get_params(self._h, None, _np_ptr(g)), "fvx_net_get_params")
        return g

    def save(self, path, stream=None):
        """Checkpoint (parameters, Adam moments and step count) to a file (fvx_net_save)."""
        check(lib().fvx_net_save(self._h, os.fsencode(path), _stream(stream)), "fvx_net_save")

    def load(self, path, stream=None):
        """Restores a checkpoint written by save (fvx_net_load); the network is
        unchanged if the file is not a checkpoint of this parameter count."""
        check(lib().fvx_net_load(self._h, os.fsencode(path), _stream(stream)), "fvx_net_load")

    def set_params(self, params, stream=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.n_params():
            raise ValueError(f"expected {self.n_params()} parameters, got {p.size}")
        check(lib().fvx_net_set_params(self._h, _np_ptr(p), _stream(stream)), "fvx_net_set_params")

    def forward(self, inp, out=None, stream=None):
        ns = int(inp.shape[0])
        out = self.samples(ns, 1) if out is None else out
        check(lib().fvx_net_forward(self._h, ns, _ptr(inp), _ptr(out), _stream(stream)), "fvx_net_forward")
        return out

    def gradients(self, inp, target, stream=None):
        loss = C.c_double()
        check(lib().fvx_net_gradients(self._h, int(inp.shape[0]), _ptr(inp), _ptr(target), C.byref(loss),
                                      _stream(stream)), "fvx_net_gradients")
        return loss.value

    def train_step(self, inp, target, lr=1e-3, stream=None):
        loss = C.c_double()
        check(lib().fvx_net_train_step(self._h, int(inp.shape[0]), _ptr(inp), _ptr(target), float(lr),
                                       C.byref(loss), _stream(stream)), "fvx_net_train_step")
        return loss.value

    def grads_tensor(self):
        """The device gradient buffer (fvx_net_grads) as a float32 tensor view."""
        torch = _torch()
        ptr = lib().fvx_net_grads(self._h)
        off = ptr - self._mem.data_ptr()
        n = self.n_params()
        return self._mem[off:off + 4 * n].view(torch.float32)

    def apply_adam(self, lr=1e-3, stream=None):
        check(lib().fvx_net_apply_adam(self._h, float(lr), _stream(stream)), "fvx_net_apply_adam")

    def prepare(self, op, B, Pprev=None, Xstar=None, inp=None, target=None, stream=None):
        """One sample's input (and target when Xstar is given) from solver vectors."""
        inp = self.samples(1, 2)[0] if inp is None else inp
        if Xstar is not None and target is None:
            target = self.samples(1, 1)[0]
        check(lib().fvx_net_prepare(self._h, op._h, _ptr(B), _ptr(Pprev), _ptr(Xstar), _ptr(inp),
                                    _ptr(target if Xstar is not None else None), _stream(stream)),
              "fvx_net_prepare")
        return inp, target

    def guess(self, op, B, Pprev=None, X0=None, stream=None):
        X0 = op.zeros() if X0 is None else X0
        check(lib().fvx_net_guess(self._h, op._h, _ptr(B), _ptr(Pprev), _ptr(X0), _stream(stream)),
              "fvx_net_guess")
        return X0

    def solve(self, op, B, Pprev=None, X=None, stream=None, allow_not_converged=False, **kw):
        """fvx_poisson_solve_net: returns (X, stats dict with 'source', the guess
        used: GUESS_NET, GUESS_GIVEN (previous pressure) or GUESS_ZERO)."""
        opts = op.solve_opts(**kw)
        X = op.zeros() if X is None else X
        ws = op.workspace(opts)
        st = SolveStats()
        fb = C.c_int(0)
        rc = lib().fvx_poisson_solve_net(op._h, self._h, _ptr(B), _ptr(Pprev), _ptr(X), C.byref(opts), _ptr(ws),
                                         ws.numel(), C.byref(st), C.byref(fb), _stream(stream))
        check(rc, "fvx_poisson_solve_net", (0, 1) if allow_not_converged else (0,))
        d = st.as_dict()
        d["source"] = int(fb.value)
        return X, d

    def __del__(self):
        if getattr(self, "_h", None):
            try:
                lib().fvx_net_destroy(self._h)
            except Exception:
                pass
            self._h = None


def copy(dst, src, nbytes=None, stream=None):
    """Device streaming copy (the bandwidth reference kernel)."""
    n = dst.numel() * dst.element_size() if nbytes is None else nbytes
    check(lib().fvx_copy(_ptr(dst), _ptr(src), n, _stream(stream)), "fvx_copy")


def copy_many(dsts, srcs, nbytes=None, stream=None):
    """dsts[i] <- srcs[i] for every pair, launched back to back from C."""
    n = len(dsts)
    nb = dsts[0].numel() * dsts[0].element_size() if nbytes is None else nbytes
    da = (C.c_void_p * n)(*[d.data_ptr() for d in dsts])
    sa = (C.c_void_p * n)(*[t.data_ptr() for t in srcs])
    check(lib().fvx_copy_many(n, da, sa, nb, _stream(stream)), "fvx_copy_many")
