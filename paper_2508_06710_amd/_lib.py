"""ctypes declarations of the C ABI in include/fvx.h.

Loading fails loudly when libfvx.so has not been built: there is no other
implementation behind these names.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfvx.so")

F64, F32, MIXED = 0, 1, 2
NONE, PERIODIC_Z = 0, 1
NEUMANN, DIRICHLET = 0, 1
GUESS_ZERO, GUESS_GIVEN, GUESS_NET = 0, 1, 2

OK, NOT_CONVERGED = 0, 1
E_ARG, E_MESH, E_NOMEM, E_HIP, E_BREAKDOWN, E_NONFINITE, E_UNSUPPORTED, E_IO = -1, -2, -3, -4, -5, -6, -7, -8
PRECOND_NONE, PRECOND_JACOBI, PRECOND_CHEBYSHEV, PRECOND_AMG = 0, 1, 2, 3
LAUNCH_PHASES, LAUNCH_GRAPH = 0, 1
NOALLOC_SCRATCH_BYTES = 128 * 1024 * 1024


class OpDesc(C.Structure):
    _fields_ = [("k", C.c_int32), ("coupling", C.c_int32), ("dz", C.c_double),
                ("wall_bc", C.c_int32), ("with_f32", C.c_int32), ("stencil", C.c_int32),
                ("reserved", C.c_int32 * 3)]


class Tile(C.Structure):
    _fields_ = [("vec", C.c_int32), ("lanes_per_row", C.c_int32), ("block", C.c_int32),
                ("xcd_remap", C.c_int32), ("max_blocks", C.c_int32), ("stage_lds", C.c_int32),
                ("nt_store", C.c_int32)]

    def as_tuple(self):
        return (self.vec, self.lanes_per_row, self.block, self.xcd_remap, self.max_blocks, self.stage_lds,
                self.nt_store)


class TuneResult(C.Structure):
    _fields_ = [("tile", Tile), ("us", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32), ("precision", C.c_int32),
                ("inner_rtol", C.c_double), ("max_outer", C.c_int32), ("guess", C.c_int32),
                ("poll_every", C.c_int32), ("precond", C.c_int32), ("cheb_degree", C.c_int32),
                ("cheb_ratio", C.c_double), ("amg", C.c_void_p), ("launch", C.c_int32)]


class AmgOpts(C.Structure):
    _fields_ = [("degree", C.c_int32), ("ratio", C.c_double), ("beta", C.c_double), ("z_rule", C.c_double),
                ("coarse_max", C.c_int32), ("max_levels", C.c_int32), ("mode_cells", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("outer", C.c_int32),
                ("rhs_projected", C.c_int32), ("relres_rec", C.c_double),
                ("relres_true", C.c_double), ("r0_over_b", C.c_double), ("bnorm", C.c_double),
                ("seconds", C.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_vp = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_P = C.POINTER

# name -> (restype, argtypes); every entry point declared in include/fvx.h.
SIGNATURES = {
    "fvx_status_str": (C.c_char_p, [C.c_int]),
    "fvx_last_error": (C.c_char_p, []),
    "fvx_version": (C.c_int, []),
    "fvx_mesh_cartesian": (C.c_int, [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                     C.c_double, C.c_double, C.c_int, C.c_int, _P(_vp)]),
    "fvx_mesh_triangles": (C.c_int, [C.c_int, _vp, C.c_int, _vp, _P(_vp)]),
    "fvx_mesh_from_faces": (C.c_int, [C.c_int, _vp, _vp, _vp, C.c_int, _vp, _vp, _vp, _vp,
                                      C.c_int, _vp, _vp, _vp, _P(_vp)]),
    "fvx_mesh_info": (C.c_int, [_vp, _P(_i64), _P(_i64), _P(_i64)]),
    "fvx_mesh_centroids": (C.c_int, [_vp, _vp, _vp]),
    "fvx_hilbert_order": (C.c_int, [_i64, _vp, _vp, _vp]),
    "fvx_mesh_faces": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "fvx_mesh_destroy": (C.c_int, [_vp]),
    "fvx_op_bytes": (C.c_int, [_vp, _P(OpDesc), _P(C.c_size_t)]),
    "fvx_op_create": (C.c_int, [_vp, _P(OpDesc), _vp, C.c_size_t, _vp, _P(_vp)]),
    "fvx_op_destroy": (C.c_int, [_vp]),
    "fvx_op_shape": (C.c_int, [_vp, _P(_i64), _P(_i64), _P(_i32), _P(_i32), _P(_i64)]),
    "fvx_op_singular": (C.c_int, [_vp]),
    "fvx_op_get_tile": (C.c_int, [_vp, C.c_int, _P(Tile)]),
    "fvx_op_set_tile": (C.c_int, [_vp, C.c_int, _P(Tile)]),
    "fvx_tune": (C.c_int, [_vp, C.c_int, _vp, C.c_size_t, C.c_int, _vp, _vp, C.c_int, _P(C.c_int)]),
    "fvx_op_get_cg_tile": (C.c_int, [_vp, C.c_int, _P(Tile)]),
    "fvx_op_set_cg_tile": (C.c_int, [_vp, C.c_int, _P(Tile)]),
    "fvx_tune_cg_bytes": (C.c_int, [_vp, C.c_int, _P(C.c_size_t)]),
    "fvx_tune_cg": (C.c_int, [_vp, C.c_int, _vp, C.c_size_t, C.c_int, _vp, _vp, C.c_int, _P(C.c_int)]),
    "fvx_tune_cached": (C.c_int, [_vp, C.c_int, C.c_char_p, _vp, C.c_size_t, C.c_int, _vp, _vp, _vp]),
    "fvx_tune_cg_cached": (C.c_int, [_vp, C.c_int, C.c_char_p, _vp, C.c_size_t, C.c_int, _vp, _vp, _vp]),
    "fvx_lap": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp, _vp]),
    "fvx_lap_many": (C.c_int, [_vp, C.c_int, C.c_int, _P(_vp), _P(_vp), _vp]),
    "fvx_div": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp, _vp]),
    "fvx_convect": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp, _vp, _vp]),
    "fvx_grad": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp, _vp]),
    "fvx_grad_axpy": (C.c_int, [_vp, C.c_int, C.c_double, _vp, _vp, _vp, _vp]),
    "fvx_pack": (C.c_int, [_vp, C.c_int, _i64, _vp, _vp, _vp]),
    "fvx_unpack": (C.c_int, [_vp, C.c_int, _i64, _vp, _vp, _vp]),
    "fvx_solve_opts_default": (C.c_int, [_P(SolveOpts)]),
    "fvx_solve_bytes": (C.c_int, [_vp, _P(SolveOpts), _P(C.c_size_t)]),
    "fvx_poisson_solve": (C.c_int, [_vp, _vp, _vp, _P(SolveOpts), _vp, C.c_size_t,
                                    _P(SolveStats), _vp]),
    "fvx_poisson_solve_noalloc": (C.c_int, [_vp, _vp, _vp, _P(SolveOpts), _P(SolveStats), _vp]),
    "fvx_solve_batch_bytes": (C.c_int, [C.c_int, _P(_vp), _P(SolveOpts), _P(C.c_size_t)]),
    "fvx_poisson_solve_batch": (C.c_int, [C.c_int, _P(_vp), _P(_vp), _P(_vp), _P(SolveOpts), _vp, C.c_size_t,
                                          _vp, _vp]),
    "fvx_expand_csr": (C.c_int, [_vp, _P(OpDesc), _P(_i64), _vp, _vp, _vp]),
    "fvx_csr_spmv": (C.c_int, [_i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fvx_csr_solve_bytes": (C.c_int, [_i64, _P(C.c_size_t)]),
    "fvx_csr_poisson_solve": (C.c_int, [_i64, _i64, _vp, _vp, _vp, _vp, _vp, C.c_int, _P(SolveOpts), _vp,
                                        C.c_size_t, _P(SolveStats), _vp]),
    "fvx_copy": (C.c_int, [_vp, _vp, C.c_size_t, _vp]),
    "fvx_copy_many": (C.c_int, [C.c_int, _P(_vp), _P(_vp), C.c_size_t, _vp]),
    "fvx_sparse_bytes": (C.c_int, [_i64, _i64, C.c_int, _P(C.c_size_t)]),
    "fvx_sparse_create": (C.c_int, [_i64, _i64, _vp, _vp, _vp, C.c_int, _vp, C.c_size_t, _vp, _P(C.c_void_p)]),
    "fvx_sparse_destroy": (C.c_int, [_vp]),
    "fvx_sparse_shape": (C.c_int, [_vp, _P(_i64), _P(_i64), _P(_i64)]),
    "fvx_sparse_set_tile": (C.c_int, [_vp, C.c_int, _vp]),
    "fvx_sparse_spmm": (C.c_int, [_vp, C.c_int, C.c_int, _vp, C.c_int, _vp, C.c_int, _vp, _vp]),
    "fvx_amg_opts_default": (C.c_int, [_P(AmgOpts)]),
    "fvx_amg_bytes": (C.c_int, [_vp, _vp, _P(AmgOpts), _P(C.c_size_t)]),
    "fvx_amg_create": (C.c_int, [_vp, _vp, _P(AmgOpts), _vp, C.c_size_t, _vp, _P(C.c_void_p)]),
    "fvx_amg_destroy": (C.c_int, [_vp]),
    "fvx_amg_n_levels": (C.c_int, [_vp, _P(_i32)]),
    "fvx_amg_coarsest_modes": (C.c_int, [_vp, _P(_i32)]),
    "fvx_amg_level": (C.c_int, [_vp, _i32, _P(_i64), _P(_i32), _P(_i64), _P(_i32), _P(C.c_void_p)]),
    "fvx_amg_aggregates": (C.c_int, [_vp, _i32, _vp]),
    "fvx_amg_apply_bytes": (C.c_int, [_vp, C.c_int, _P(C.c_size_t)]),
    "fvx_amg_apply": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp, C.c_size_t, _vp]),
    "fvx_sparse_tune": (C.c_int, [_vp, C.c_int, C.c_int, _vp, C.c_int, _vp, C.c_int, C.c_int, _vp, _vp, C.c_int,
                                  _P(C.c_int)]),
    "fvx_mesh_refine": (C.c_int, [_vp, C.c_int, _P(C.c_void_p)]),
    "fvx_ns_step_bytes": (C.c_int, [_vp, _P(SolveOpts), _P(C.c_size_t)]),
    "fvx_ns_step": (C.c_int, [_vp, _vp, _P(C.c_void_p), _vp, _vp, _vp, C.c_double, C.c_double, _P(SolveOpts), _vp,
                              C.c_size_t, _P(SolveStats), _vp]),
    "fvx_refine_prolongation": (C.c_int, [_vp, C.c_int, _P(_i64), _vp, _vp, _vp]),
    "fvx_net_n_params": (C.c_int, []),
    "fvx_net_bytes": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, _P(C.c_size_t)]),
    "fvx_net_create": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, _vp, _vp, C.c_size_t, _vp, _P(_vp)]),
    "fvx_net_destroy": (C.c_int, [_vp]),
    "fvx_net_get_params": (C.c_int, [_vp, _vp, _vp]),
    "fvx_net_set_params": (C.c_int, [_vp, _vp, _vp]),
    "fvx_net_save": (C.c_int, [_vp, C.c_char_p, _vp]),
    "fvx_net_load": (C.c_int, [_vp, C.c_char_p, _vp]),
    "fvx_net_forward": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "fvx_net_gradients": (C.c_int, [_vp, C.c_int, _vp, _vp, _P(C.c_double), _vp]),
    "fvx_net_train_step": (C.c_int, [_vp, C.c_int, _vp, _vp, C.c_float, _P(C.c_double), _vp]),
    "fvx_net_grads": (_vp, [_vp]),
    "fvx_net_apply_adam": (C.c_int, [_vp, C.c_float, _vp]),
    "fvx_net_prepare": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fvx_net_guess": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "fvx_poisson_solve_net": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _P(SolveOpts), _vp, C.c_size_t, _P(SolveStats),
                                        _P(C.c_int), _vp]),
}

_lib = None


class FvxError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: status {code} ({detail})")
        self.code = code


def lib() -> C.CDLL:
    """The loaded libfvx.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2508_06710_amd.build` "
                              "(or __graft_entry__.build()); there is no fallback implementation")
        # torch first: its wheel carries its own HIP runtime (same soname as
        # /opt/rocm's).  Loaded after the library, it would bring a second
        # runtime into the process, and device memory from one is unknown to
        # the other; loaded before, the library binds to torch's runtime.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int, where: str, allow=(OK,)) -> int:
    if rc in allow:
        return rc
    L = lib()
    detail = L.fvx_last_error().decode() or L.fvx_status_str(rc).decode()
    raise FvxError(rc, where, detail)
