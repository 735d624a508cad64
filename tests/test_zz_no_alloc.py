"""fvx_poisson_solve_noalloc: the Poisson solve on the library's built-in
device scratch, called through the C ABI, against fvx_poisson_solve with a
caller workspace (same kernels and tiles, so the same X bit for bit), on
consecutive calls whose second input is smaller than the first, plus the
size limit of the scratch."""
import ctypes as C

import numpy as np
import pytest
import torch

import inputs
import oracle
from helpers import Case

pytestmark = pytest.mark.gpu


def _noalloc(op, B, **kw):
    from paper_2508_06710_amd import _lib
    opts = op.solve_opts(**kw)
    X = op.zeros()
    st = _lib.SolveStats()
    rc = _lib.lib().fvx_poisson_solve_noalloc(op._h, C.c_void_p(B.data_ptr()), C.c_void_p(X.data_ptr()),
                                              C.byref(opts), C.byref(st), None)
    return rc, X, st.as_dict()


def _check(c, b, **kw):
    op = c.op
    B = op.to_rows(b)
    rc, Xn, stn = _noalloc(op, B, **kw)
    assert rc == 0, rc
    Xw, stw = op.solve(B, **kw)
    torch.cuda.synchronize()
    assert torch.equal(Xn, Xw), "no-alloc solve differs from the workspace solve"
    assert stn["iters"] == stw["iters"] and stn["outer"] == stw["outer"]
    assert stn["relres_true"] == stw["relres_true"]
    # and the result solves the oracle's system
    x = op.to_planes(Xn)
    bp = oracle.project_mean(b, 1)
    rel = np.linalg.norm(bp - oracle.spmv(c.L, x)) / np.linalg.norm(bp)
    assert rel <= kw["rtol"] * 1.05, rel
    return stn


def test_noalloc_matches_workspace_solve_on_consecutive_calls():
    big = Case(inputs.channel_base(64, 64), 8)
    st1 = _check(big, inputs.rhs_uniform(31, big.m3.N), rtol=1e-10)
    small = Case(inputs.channel_base(16, 12), 4)
    st2 = _check(small, inputs.rhs_uniform(32, small.m3.N), rtol=1e-10)
    assert st1["iters"] > 0 and st2["iters"] > 0
    # mixed precision after the smaller FP64 call, on the larger operator again
    import paper_2508_06710_amd as fvx
    _check(big, inputs.rhs_uniform(33, big.m3.N), rtol=1e-10, precision=fvx.MIXED)


def test_noalloc_rejects_a_solve_beyond_the_scratch():
    import paper_2508_06710_amd as fvx
    from paper_2508_06710_amd import _lib
    op = fvx.Operator(fvx.Mesh.from_spec(inputs.channel_base(256, 192)), 128, np.pi / 128, fvx.PERIODIC_Z,
                      with_f32=False)
    need = C.c_size_t()
    opts = op.solve_opts(rtol=1e-8)
    assert _lib.lib().fvx_solve_bytes(op._h, C.byref(opts), C.byref(need)) == 0
    assert need.value > _lib.NOALLOC_SCRATCH_BYTES
    B = op.zeros()
    rc, _, _ = _noalloc(op, B, rtol=1e-8)
    assert rc == _lib.E_NOMEM
    assert b"scratch" in _lib.lib().fvx_last_error()
