"""GPU Poisson solves against the oracle.

Solution vectors of two correct solves may differ by about cond(L) * rtol,
so parity is defined through residuals recomputed with the ORACLE's matrix,
brute-force dense solves on tiny meshes, the oracle CG's iteration count,
and bitwise repeatability of the deterministic reductions."""
import math

import numpy as np
import pytest
import torch

import inputs
import oracle
from helpers import Case

pytestmark = pytest.mark.gpu


def _true_relres(c, x, b):
    """Per group ||bp - L x|| / ||bp|| with the oracle's assembled matrix."""
    ng = c.m3.n_groups()
    bp = oracle.project_mean(b, ng)
    r = bp - oracle.spmv(c.L, x)
    if c.coupling == 0 and c.k > 1:
        return [np.linalg.norm(rr) / np.linalg.norm(bb) for rr, bb in
                zip(r.reshape(c.k, -1), bp.reshape(c.k, -1))]
    return [np.linalg.norm(r) / np.linalg.norm(bp)]


def _solve(c, b, **kw):
    X, st = c.op.solve(c.op.to_rows(b), **kw)
    return c.op.to_planes(X), st


@pytest.mark.parametrize("spec,k,coupling", [
    (inputs.channel_base(64, 64), 8, 1),        # the 64x64 stretched channel, 8 planes
    (inputs.channel_base(13, 9), 1, 1),
    (inputs.channel_base(13, 9), 2, 1),
    (inputs.channel_base(13, 9), 5, 0),
    (inputs.convection_base(12, 20), 16, 1),
    (inputs.unit_square_triangles(8), 4, 1),
])
def test_true_residual_and_iterations_match_oracle(spec, k, coupling):
    c = Case(spec, k, coupling=coupling)
    b = inputs.rhs_uniform(0, c.m3.N)
    for rtol in (1e-8, 1e-10):
        x, st = _solve(c, b, rtol=rtol)
        assert st["status"] == 0
        rel = _true_relres(c, x, b)
        assert max(rel) <= rtol * 1.05, rel
        assert abs(st["relres_true"] - max(rel)) <= 1e-3 * rtol + 1e-14
        ref = oracle.cg(c.m3, c.L, b, rtol)
        it_ref = max(ref.iters)
        assert abs(st["iters"] - it_ref) <= max(2, math.ceil(0.01 * it_ref)), (st["iters"], it_ref)
        # zero plain mean on exit (singular operator)
        for g in x.reshape(c.m3.n_groups(), -1):
            assert abs(g.mean()) <= 1e-13 * np.abs(g).max()


@pytest.mark.parametrize("k,coupling,dirichlet", [(1, 1, False), (2, 1, False), (3, 1, False),
                                                  (4, 0, False), (3, 1, True)])
def test_tiny_mesh_matches_dense_direct_solve(k, coupling, dirichlet):
    c = Case(inputs.channel_base(6, 5, 0.5), k, 0.6, coupling, dirichlet)
    b = inputs.rhs_uniform(3, c.m3.N)
    x, st = _solve(c, b, rtol=1e-15, max_iter=500, allow_not_converged=True)
    ng = c.m3.n_groups()
    xd = oracle.dense_solve(c.m3.dense_lap(), oracle.project_mean(b, ng), ng)
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)


def test_finite_termination_special_case():
    """A uniform 4-cell periodic ring x 4 periodic planes has four distinct
    nonzero eigenvalues: CG ends within 4 iterations."""
    c = Case(inputs.CartSpec(4, 1, 4.0, 0.0, 1.0, 0.0, True, False), 4, 1.0)
    b = inputs.rhs_uniform(11, c.m3.N)
    x, st = _solve(c, b, rtol=1e-13, max_iter=50)
    assert st["iters"] <= 4 and st["relres_true"] < 1e-13


def test_bitwise_repeatable():
    c = Case(inputs.channel_base(48, 40), 16)
    b = c.op.to_rows(inputs.rhs_uniform(2, c.m3.N))
    X1, s1 = c.op.solve(b, rtol=1e-9)
    X2, s2 = c.op.solve(b, rtol=1e-9)
    assert torch.equal(X1, X2) and s1["iters"] == s2["iters"]


def test_initial_guess_and_projection_flags():
    c = Case(inputs.channel_base(20, 16), 4)
    b = inputs.rhs_uniform(4, c.m3.N) + 3.0  # nonzero mean: projected
    x, st = _solve(c, b, rtol=1e-10)
    assert st["rhs_projected"] == 1
    X0 = c.op.to_rows(x)
    _, st2 = c.op.solve(c.op.to_rows(b), X=X0, guess=1, rtol=1e-10)
    assert st2["iters"] <= 1 and st2["r0_over_b"] <= 1.1e-10
    # a constant right-hand side projects to zero: x = 0 without iterating
    x0, st0 = _solve(c, np.ones(c.m3.N), rtol=1e-10)
    assert st0["iters"] == 0 and np.all(x0 == 0)


def test_failure_paths():
    c = Case(inputs.channel_base(16, 12), 4)
    fvx = c.fvx
    b = inputs.rhs_uniform(5, c.m3.N)
    _, st = c.op.solve(c.op.to_rows(b), rtol=1e-10, max_iter=1, allow_not_converged=True)
    assert st["status"] == fvx._lib.NOT_CONVERGED and st["iters"] == 1
    bad = b.copy()
    bad[7] = np.nan
    with pytest.raises(fvx.FvxError) as e:
        c.op.solve(c.op.to_rows(bad), rtol=1e-8)
    assert e.value.code == fvx._lib.E_NONFINITE
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    from paper_2508_06710_amd import _lib
    import ctypes as C
    opts = c.op.solve_opts()
    st = _lib.SolveStats()
    B = c.op.to_rows(b)
    X = c.op.zeros()
    rc = _lib.lib().fvx_poisson_solve(c.op._h, C.c_void_p(B.data_ptr()), C.c_void_p(X.data_ptr()),
                                      C.byref(opts), C.c_void_p(small.data_ptr()), 16, C.byref(st), None)
    assert rc == _lib.E_NOMEM


@pytest.mark.parametrize("spec,k,coupling", [
    (inputs.channel_base(64, 64), 8, 1),
    (inputs.channel_base(24, 16), 8, 1),
    (inputs.channel_base(13, 9), 6, 0),
    (inputs.unit_square_triangles(10), 8, 1),
])
def test_mixed_precision_reaches_fp64_residual(spec, k, coupling):
    """FP32-SpMM CG inside an FP64 defect correction: the true residual by the
    oracle's matrix reaches 1e-10, and the error against the FP64 solution x*
    (rtol 1e-13) is within the a-posteriori bound kappa (relres + relres*),
    where ||x - x_true|| <= ||r|| / lambda_min and ||x_true|| >= ||b|| /
    lambda_max; kappa = lambda_max / lambda_min of -L on the complement of
    its null space, from the oracle matrix's dense spectrum (meshes of at
    most a few thousand cells)."""
    c = Case(spec, k, coupling=coupling)
    fvx = c.fvx
    b = inputs.rhs_uniform(7, c.m3.N)
    x, st = _solve(c, b, rtol=1e-10, precision=fvx.MIXED, inner_rtol=1e-4)
    assert st["status"] == 0 and st["outer"] >= 2
    rel = max(_true_relres(c, x, b))
    assert rel <= 1e-10 * 1.05, rel
    xr, _ = _solve(c, b, rtol=1e-13)
    rel_star = max(_true_relres(c, xr, b))
    err = np.linalg.norm(x - xr) / np.linalg.norm(xr)
    if c.m3.N <= 4000:
        groups = k if (coupling == 0 or k == 1) else 1
        ev = np.linalg.eigvalsh((-c.L).toarray())
        lam_min, lam_max = ev[groups], ev[-1]  # the null space holds one constant per group
        assert abs(ev[groups - 1]) <= 1e-10 * lam_max < lam_min
        kappa = lam_max / lam_min
        bound = kappa * (rel + rel_star)
        print(f"mixed vs fp64 solution: rel err {err:.2e}, bound {bound:.2e} (kappa {kappa:.3e}), "
              f"inner iters {st['iters']}, outer {st['outer']}")
        assert err <= bound * (1 + 1e-6)
    else:
        print(f"mixed vs fp64 solution: rel err {err:.2e}, inner iters {st['iters']}, outer {st['outer']}")
        assert err <= 1e-6


@pytest.mark.parametrize("spec,k", [(inputs.channel_base(64, 64), 8), (inputs.unit_square_triangles(8), 3)])
def test_assembled_csr_comparator(spec, k):
    """The no-block-reuse comparator: its SpMV reproduces the oracle product and
    its textbook CG reaches the tolerance with the oracle's iteration count."""
    c = Case(spec, k)
    fvx = c.fvx
    ptr, col, val = fvx.expand_csr(c.op.mesh, k, c.dz, fvx.PERIODIC_Z)
    A = fvx.CsrMatrix(ptr, col, val)
    x = inputs.uniform(21, 0, c.m3.N)
    y = A.spmv(torch.as_tensor(x).cuda()).cpu().numpy()
    from helpers import componentwise
    assert componentwise(y, oracle.spmv(c.L, x), c.L, x) <= 1e-12
    b = inputs.rhs_uniform(22, c.m3.N)
    xs, st = A.solve(torch.as_tensor(b).cuda(), rtol=1e-10)
    xs = xs.cpu().numpy()
    assert max(_true_relres(c, xs, b)) <= 1.05e-10
    ref = oracle.cg(c.m3, c.L, b, 1e-10)
    assert abs(st["iters"] - ref.iters[0]) <= max(2, math.ceil(0.01 * ref.iters[0]))
    assert abs(xs.mean()) <= 1e-13 * np.abs(xs).max()


@pytest.mark.parametrize("per_row", [1, 2, 3, 7, 13, 27, 50, 100])
def test_csr_spmv_lane_groups(per_row):
    """The comparator SpMV over every lane-group width (1 to 64 lanes per row,
    chosen from the mean row length), on random rows of varied length with
    repeated columns, against the oracle's CSR loop."""
    import scipy.sparse as sp
    fvx = __import__("paper_2508_06710_amd")
    n = 3001
    lens = (inputs.u64(23, 0, n) % np.uint64(2 * per_row)).astype(np.int64) + 1  # mean about per_row
    ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    nnz = int(ptr[-1])
    col = (inputs.u64(23, 1, nnz) % np.uint64(n)).astype(np.int32)
    val = inputs.uniform(23, 2, nnz)
    A = sp.csr_matrix((val, col, ptr), shape=(n, n))
    x = inputs.uniform(23, 3, n)
    y = fvx.CsrMatrix(ptr, col, val).spmv(torch.as_tensor(x).cuda()).cpu().numpy()
    ref = oracle.spmv(A, x)
    from helpers import componentwise
    assert componentwise(y, ref, A, x) <= 1e-12


@pytest.mark.parametrize("stencil", [13, 27])
def test_csr_comparator_on_structured_operators(stencil):
    fvx = __import__("paper_2508_06710_amd")
    spec, k, dz = inputs.channel_base(12, 10), 6, 0.4
    ptr, col, val = fvx.expand_csr(fvx.Mesh.from_spec(spec), k, dz, fvx.PERIODIC_Z, stencil=stencil)
    L = oracle.stencil_lap(spec, k, dz, stencil)
    x = inputs.uniform(24, 0, L.shape[0])
    y = fvx.CsrMatrix(ptr, col, val).spmv(torch.as_tensor(x).cuda()).cpu().numpy()
    from helpers import componentwise
    assert componentwise(y, oracle.spmv(L, x), L, x) <= 1e-12


def test_copy_kernel():
    fvx = __import__("paper_2508_06710_amd")
    src = torch.arange(1 << 20, dtype=torch.float64, device="cuda")
    dst = torch.zeros_like(src)
    fvx.copy(dst, src)
    assert torch.equal(dst, src)
    with pytest.raises(fvx.FvxError):
        fvx.copy(dst[1:], src[1:], 8 * 100)


def test_mixed_precision_does_not_depend_on_workspace_contents():
    """Regression: the mixed solve must not read stale per-column norms from a
    reused workspace (a zeroed and a garbage-filled workspace give the same x)."""
    c = Case(inputs.channel_base(13, 9), 6, coupling=0)
    fvx = c.fvx
    b = c.op.to_rows(inputs.rhs_uniform(8, c.m3.N))
    opts = dict(rtol=1e-10, precision=fvx.MIXED)
    ws = c.op.workspace(c.op.solve_opts(**opts))
    ws.zero_()
    X1, _ = c.op.solve(b, **opts)
    ws.fill_(0x7F)
    X2, _ = c.op.solve(b, **opts)
    assert torch.equal(X1, X2)
    assert max(_true_relres(c, c.op.to_planes(X1), c.op.to_planes(b))) <= 1.05e-10


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_cg_tiles_and_tuner(precision):
    """Every CG tile solves to the tolerance by the oracle's residual; the CG
    autotuner keeps its fastest candidate; block 0 restores the default."""
    c = Case(inputs.channel_base(40, 24), 16, with_f32=True)
    fvx = c.fvx
    dt = fvx.F64 if precision == "f64" else fvx.F32
    prec = fvx.F64 if precision == "f64" else fvx.MIXED
    b = inputs.rhs_uniform(77, c.op.n_b * c.k)
    B = c.op.to_rows(b)
    vec = c.op.get_cg_tile(dt)[0]
    for block, remap, cap in ((128, 0, 512), (512, 1, 2048), (256, 1, 0)):
        c.op.set_cg_tile(vec, 1, block, remap, cap, dtype=dt)
        got = c.op.get_cg_tile(dt)
        assert got[2] == block and got[1] * got[0] >= c.k  # lanes widened to one pass
        X, st = c.op.solve(B, rtol=1e-10, precision=prec)
        assert max(_true_relres(c, c.op.to_planes(X), b)) <= 1e-10 * 1.0001
    res = c.op.tune_cg(dt, iters=16)
    assert len(res) >= 6
    assert c.op.get_cg_tile(dt) == min(res, key=lambda r: r[1])[0]
    X, st = c.op.solve(B, rtol=1e-10, precision=prec)
    assert max(_true_relres(c, c.op.to_planes(X), b)) <= 1e-10 * 1.0001
    c.op.set_cg_tile(block=0, dtype=dt)
    assert c.op.get_cg_tile(dt)[2] == 256
    with pytest.raises(fvx.FvxError):
        c.op.set_cg_tile(vec, 8, 1024, 1, 0, dtype=dt)


@pytest.mark.parametrize("spec,k,coupling", [
    (inputs.channel_base(40, 24), 16, 1),                                   # ragged tiles along x
    (inputs.convection_base(12, 22), 8, 1),                                 # walls on all sides, ny % 4 = 2
    (inputs.CartSpec(10, 9, 1.0, 0.0, 1.0, 0.3, True, True), 4, 1),        # periodic in x and y
    (inputs.channel_base(13, 9), 5, 0),                                     # independent planes, k = 5
    (inputs.channel_base(24, 16), 1, 1),                                    # one plane: no coupling term
])
@pytest.mark.parametrize("kw", [{}, {"precond": 1}, {"precond": 2, "cheb_degree": 3, "cheb_ratio": 30.0},
                                {"precision": 2}])
def test_cg_line_tiles(spec, k, coupling, kw):
    """The CG iteration kernels on line tiles (stage_lds = 1 of a CG tile: a
    row group takes 4 grid lines of one cell column) against the row tiles:
    the same products in another order of the FP64 partial sums, so the true
    residual by the oracle's matrix meets the tolerance, the iteration count
    is the row tiles' within one, and the solve is bitwise repeatable."""
    c = Case(spec, k, coupling=coupling, with_f32=True)
    fvx = c.fvx
    prec = kw.get("precision", fvx.F64)
    dt = fvx.F32 if prec == fvx.MIXED else fvx.F64
    b = inputs.rhs_uniform(41, c.m3.N)
    B = c.op.to_rows(b)
    vec = c.op.get_cg_tile(dt)[0]
    out = {}
    for lines in (0, 1):
        c.op.set_cg_tile(vec, 1, 128, 1, 0, lines, dtype=dt)
        assert c.op.get_cg_tile(dt)[5] == lines
        X, st = c.op.solve(B, rtol=1e-10, **kw)
        X2, st2 = c.op.solve(B, rtol=1e-10, **kw)
        assert torch.equal(X, X2) and st["iters"] == st2["iters"]
        assert max(_true_relres(c, c.op.to_planes(X), b)) <= 1e-10 * 1.05
        out[lines] = st["iters"]
    assert abs(out[1] - out[0]) <= 1, out
    c.op.set_cg_tile(block=0, dtype=dt)
