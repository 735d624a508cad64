"""The aggregation multigrid on the GPU (fvx_amg_*) against the oracle's
multigrid on assembled matrices (oracle/amg.py): the same levels and
aggregates (integer work: bit-exact), every coarse level's SpMM against the
oracle's Galerkin product P^T A P, one V-cycle element by element, and CG
preconditioned by the cycle against the oracle's PCG (true residual,
iteration count, dense solves), in FP64 and mixed precision."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import inputs
import oracle
from helpers import Case
from oracle import amg as oamg
from oracle import pcg as opcg

pytestmark = pytest.mark.gpu

CASES = [
    # spec, k, dz, coupling, dirichlet, coarse_max
    (inputs.channel_base(32, 24), 8, None, 1, False, 40),
    (inputs.channel_base(24, 20), 16, 0.02, 1, False, 40),      # planes strongly coupled: plane merging
    (inputs.convection_base(12, 20), 16, None, 1, False, 60),
    (inputs.channel_base(16, 12), 6, None, 1, True, 30),        # Dirichlet walls
    (inputs.channel_base(20, 16), 5, None, 0, False, 20),       # independent planes
    (inputs.channel_base(17, 13), 5, 0.05, 1, False, 25),       # odd k: no plane merging possible
    (inputs.unit_square_triangles(8), 4, None, 1, False, 30),
    (inputs.naca_delaunay(seed=3, n_interior=1500, n_surface=60, n_box_side=16), 4, 0.2, 1, False, 40),
]
IDS = ["channel", "channel-z", "convection", "dirichlet", "independent", "odd-k", "triangles", "airfoil"]
# coarsest level solved per plane mode (last entry: mode_cells); the oracle
# solves the same coarsest level with one pseudo-inverse of all its planes
MODE_CASES = [
    (inputs.channel_base(32, 24), 8, None, 1, False, 40, 50),
    (inputs.channel_base(24, 20), 16, 0.02, 1, False, 40, 30),   # planes merged down to one: a single mode
    (inputs.channel_base(24, 20), 2, None, 1, False, 40, 150),   # two planes: modes 0 and 1, no sine
    (inputs.channel_base(16, 12), 6, None, 1, True, 30, 60),
    (inputs.channel_base(17, 13), 5, 0.05, 1, False, 25, 60),    # odd k: every mode > 0 has a sine
    (inputs.unit_square_triangles(8), 4, None, 1, False, 30, 40),
    (inputs.channel_base(20, 16), 5, None, 0, False, 20, 100),   # independent planes: one shared system
    (inputs.channel_base(24, 20), 8, None, 0, False, 20, 100),   # independent planes, an even count
    (inputs.channel_base(17, 13), 1, None, 1, False, 20, 400),   # one plane: a single mode, 221 cells
]
MODE_IDS = ["channel-modes", "channel-z-modes", "k2-modes", "dirichlet-modes", "odd-k-modes", "triangles-modes",
            "independent-modes", "independent-8-modes", "k1-modes"]
ALL, ALL_IDS = CASES + MODE_CASES, IDS + MODE_IDS


def _setup(spec, k, dz, coupling, dirichlet, coarse_max, mode_cells=0, degree=2):
    import paper_2508_06710_amd as fvx
    c = Case(spec, k, dz=dz, coupling=coupling, dirichlet=dirichlet)
    amg = fvx.Amg(c.op, degree=degree, coarse_max=coarse_max, mode_cells=mode_cells)
    coupled = coupling == 1 and k >= 2
    A = (-c.L).tocsr()
    n_b = c.m3.n_b
    opts = oamg.AmgOpts(degree=degree, coarse_max=coarse_max, mode_cells=mode_cells)
    h = oamg.build(A if coupled else A[:n_b, :n_b].tocsr(), n_b, k if coupled else 1, coupled, opts,
                   columns=1 if coupled else k)
    return c, amg, h, coupled


@pytest.mark.parametrize("case", ALL, ids=ALL_IDS)
def test_levels_and_aggregates_equal_the_oracle(case):
    c, amg, h, coupled = _setup(*case)
    got = amg.levels()
    assert len(got) == len(h.levels)
    kinds = {"": 0, "xy": 1, "z": 2}
    for l, (lv, g) in enumerate(zip(h.levels, got)):
        n_b, k, _, kind = g
        assert (n_b, kind) == (lv.n_b, kinds[lv.kind]), l
        assert k == (lv.k if coupled else c.k), l
        if lv.kind == "xy":
            assert np.array_equal(amg.aggregates(l), lv.agg), l
    last, cells = h.levels[-1], (case[6] if len(case) > 6 else 0)
    units = last.k // 2 + 1 if coupled else (c.k + 1) // 2
    above = last.n_b * (last.k if coupled else c.k) > case[5]       # within coarse_max: the dense solve
    by_modes = above and 0 < last.n_b <= cells and units * last.n_b ** 2 <= oamg.MODE_TERMS
    assert amg.coarsest_modes == ((last.k // 2 + 1 if coupled else 1) if by_modes else 0)


@pytest.mark.parametrize("case", ALL, ids=ALL_IDS)
def test_every_level_operator_is_the_galerkin_product(case):
    """Element by element within 1e-12 of (P^T |A| P)|x| carried down the
    levels -- the scale of the rounding of the Galerkin sums (a coarse entry
    can vanish exactly, as a one-cell Neumann level does)."""
    c, amg, h, coupled = _setup(*case)
    absA = abs(h.levels[0].A)
    for l in range(1, len(h.levels)):
        P = h.levels[l - 1].P
        absA = (P.T @ absA @ P).tocsr()
        op = amg.level_op(l)
        lv = h.levels[l]
        A = lv.A if coupled else sp.kron(sp.identity(c.k), lv.A).tocsr()
        S = absA if coupled else sp.kron(sp.identity(c.k), absA).tocsr()
        x = inputs.uniform(100 + l, 0, A.shape[0])
        y = op.to_planes(op.lap(op.to_rows(x)))
        ref = -(A @ x)
        bound = S @ np.abs(x)
        assert np.max(np.abs(y - ref) / bound) <= 1e-12, l


def _oracle_cycle(h, c, coupled, r):
    if coupled:
        return oamg.vcycle(h, r)
    n_b = c.m3.n_b
    return np.concatenate([oamg.vcycle(h, r[l * n_b:(l + 1) * n_b]) for l in range(c.k)])


@pytest.mark.parametrize("degree", [2, 3])
@pytest.mark.parametrize("case", ALL, ids=ALL_IDS)
def test_one_v_cycle_matches_the_oracle(case, degree):
    c, amg, h, coupled = _setup(*case, degree=degree)
    ng = c.m3.n_groups()
    r = inputs.rhs_uniform(110, c.m3.N)
    if c.m3.singular:
        r = oracle.project_mean(r, ng)
    z = c.op.to_planes(amg.apply(c.op.to_rows(r)))
    ref = _oracle_cycle(h, c, coupled, r)
    # the cycle is one linear map computed in two rounding orders; its error
    # grows with the coarse levels' condition numbers (< 1e5 here): 1e-16 x 1e5 x margin
    assert np.linalg.norm(z - ref) <= 1e-9 * np.linalg.norm(ref)


@pytest.mark.parametrize("case", [CASES[0], MODE_CASES[0], MODE_CASES[4]], ids=["dense", "modes", "modes-odd-cells"])
def test_fp32_cycle_is_close_to_the_fp64_cycle(case):
    c, amg, h, coupled = _setup(*case)
    r = oracle.project_mean(inputs.rhs_uniform(111, c.m3.N), 1)
    z32 = c.op.to_planes(amg.apply(c.op.to_rows(r, dtype=c.fvx.F32)), dtype=c.fvx.F32).astype(np.float64)
    ref = oamg.vcycle(h, r)
    assert np.linalg.norm(z32 - ref) <= 1e-3 * np.linalg.norm(ref)


def test_fp32_cycle_with_wide_lanes():
    """An FP32 cycle whose finest levels stream (16384 and 4096 cells x 64
    planes: 4 elements per lane in the smoother, the restriction and the
    prolongation; 2 on the coarser and plane-merged levels) against the
    oracle's FP64 cycle, and the mixed-precision solve with it."""
    c, amg, h, coupled = _setup(inputs.channel_base(128, 128), 64, None, 1, False, 2048)
    assert [lv.n_b for lv in h.levels[:2]] == [16384, 4096] and h.levels[2].kind == "z"
    r = oracle.project_mean(inputs.rhs_uniform(123, c.m3.N), 1)
    z32 = c.op.to_planes(amg.apply(c.op.to_rows(r, dtype=c.fvx.F32)), dtype=c.fvx.F32).astype(np.float64)
    ref = oamg.vcycle(h, r)
    assert np.linalg.norm(z32 - ref) <= 1e-3 * np.linalg.norm(ref)
    b = inputs.rhs_uniform(124, c.m3.N)
    X, st = c.op.solve(c.op.to_rows(b), rtol=1e-10, precision=c.fvx.MIXED, amg=amg)
    assert st["status"] == 0
    assert _true_relres(c, c.op.to_planes(X), b) <= 1e-10 * 1.05


def test_one_level_is_the_exact_pseudo_inverse():
    import paper_2508_06710_amd as fvx
    c = Case(inputs.channel_base(10, 8), 4)
    amg = fvx.Amg(c.op, coarse_max=2048, mode_cells=0)
    assert amg.n_levels == 1 and amg.coarsest_modes == 0
    r = oracle.project_mean(inputs.rhs_uniform(112, c.m3.N), 1)
    z = c.op.to_planes(amg.apply(c.op.to_rows(r)))
    A = (-c.L).tocsr()
    assert np.linalg.norm(A @ z - r) <= 1e-12 * np.linalg.norm(r)
    b = inputs.rhs_uniform(113, c.m3.N)
    X, st = c.op.solve(c.op.to_rows(b), rtol=1e-10, amg=amg)
    assert st["status"] == 0 and st["iters"] == 1


@pytest.mark.parametrize("k", [4, 5])
def test_one_level_by_plane_modes_is_the_exact_pseudo_inverse(k):
    import paper_2508_06710_amd as fvx
    c = Case(inputs.channel_base(10, 8), k)
    amg = fvx.Amg(c.op, coarse_max=20, mode_cells=80)
    assert amg.n_levels == 1 and amg.coarsest_modes == k // 2 + 1
    r = oracle.project_mean(inputs.rhs_uniform(120, c.m3.N), 1)
    z = c.op.to_planes(amg.apply(c.op.to_rows(r)))
    A = (-c.L).tocsr()
    assert np.linalg.norm(A @ z - r) <= 1e-12 * np.linalg.norm(r)
    assert abs(z.sum()) <= 1e-12 * np.abs(z).sum()         # the pseudo-inverse: no constant component
    b = inputs.rhs_uniform(121, c.m3.N)
    X, st = c.op.solve(c.op.to_rows(b), rtol=1e-10, amg=amg)
    assert st["status"] == 0 and st["iters"] == 1


def test_default_options_use_plane_modes_within_the_term_budget():
    """Default options (mode_cells 2048): 17 plane modes of the 768-cell base
    exceed the 2^23-term budget, so the base is aggregated once more and the
    next level is solved per mode; the levels equal the oracle's and the
    preconditioned solve reaches its tolerance by the oracle's matrix."""
    import paper_2508_06710_amd as fvx
    c = Case(inputs.channel_base(32, 24), 32)
    amg = fvx.Amg(c.op)
    h = oamg.build((-c.L).tocsr(), c.m3.n_b, 32, True, oamg.AmgOpts(mode_cells=2048), solve_coarsest=False)
    got = amg.levels()
    assert [(g[0], g[1]) for g in got] == [(lv.n_b, lv.k) for lv in h.levels] and len(got) >= 2
    assert amg.coarsest_modes == h.levels[-1].k // 2 + 1
    b = inputs.rhs_uniform(122, c.m3.N)
    X, st = c.op.solve(c.op.to_rows(b), rtol=1e-10, amg=amg)
    assert st["status"] == 0
    assert _true_relres(c, c.op.to_planes(X), b) <= 1e-10 * 1.05
    _, s0 = c.op.solve(c.op.to_rows(b), rtol=1e-10)
    assert st["iters"] < s0["iters"] // 5


def _true_relres(c, x, b):
    ng = c.m3.n_groups()
    bp = oracle.project_mean(b, ng) if c.m3.singular else b
    r = bp - oracle.spmv(c.L, x)
    if c.coupling == 0 and c.k > 1:
        return max(np.linalg.norm(rr) / np.linalg.norm(bb) for rr, bb in zip(r.reshape(c.k, -1), bp.reshape(c.k, -1)))
    return np.linalg.norm(r) / np.linalg.norm(bp)


@pytest.mark.parametrize("case", ALL, ids=ALL_IDS)
def test_amg_pcg_residual_and_iterations_match_the_oracle(case):
    c, amg, h, coupled = _setup(*case)
    b = inputs.rhs_uniform(114, c.m3.N)
    rtol = 1e-9
    X, st = c.op.solve(c.op.to_rows(b), rtol=rtol, amg=amg)
    assert st["status"] == 0
    assert _true_relres(c, c.op.to_planes(X), b) <= rtol * 1.05
    ref = opcg.pcg(c.m3, c.L, b, rtol, precond="amg", amg_opts=h.opts)
    it_ref = max(ref.iters)
    assert abs(st["iters"] - it_ref) <= max(2, math.ceil(0.02 * it_ref)), (st["iters"], it_ref)
    _, s0 = c.op.solve(c.op.to_rows(b), rtol=rtol)
    assert st["iters"] < s0["iters"]


def test_amg_pcg_matches_dense_solve_and_repeats_bitwise():
    c, amg, h, coupled = _setup(inputs.channel_base(8, 6), 4, None, 1, False, 12)
    assert amg.n_levels >= 3
    b = inputs.rhs_uniform(115, c.m3.N)
    B = c.op.to_rows(b)
    X1, s1 = c.op.solve(B, rtol=1e-13, amg=amg)
    X2, s2 = c.op.solve(B, rtol=1e-13, amg=amg)
    x = c.op.to_planes(X1)
    assert s1["iters"] == s2["iters"] and np.array_equal(x, c.op.to_planes(X2))
    xd = oracle.dense_solve(c.L.toarray(), oracle.project_mean(b, 1), 1)
    assert np.max(np.abs(x - xd)) <= 1e-9 * np.max(np.abs(xd))


@pytest.mark.parametrize("case", [CASES[0], CASES[4], MODE_CASES[0], MODE_CASES[4], MODE_CASES[6]],
                         ids=["coupled", "independent", "modes", "modes-odd-cells", "modes-independent"])
def test_mixed_precision_with_amg(case):
    c, amg, h, coupled = _setup(*case)
    b = inputs.rhs_uniform(116, c.m3.N)
    X, st = c.op.solve(c.op.to_rows(b), rtol=1e-10, precision=c.fvx.MIXED, amg=amg)
    assert st["status"] == 0
    assert _true_relres(c, c.op.to_planes(X), b) <= 1e-10 * 1.05


def test_given_guess_with_amg():
    c, amg, h, coupled = _setup(*CASES[0])
    b = inputs.rhs_uniform(117, c.m3.N)
    x0 = inputs.uniform(117, 1, c.m3.N)
    X, st = c.op.solve(c.op.to_rows(b), X=c.op.to_rows(x0), rtol=1e-10, guess=c.fvx.GUESS_GIVEN, amg=amg)
    assert st["status"] == 0
    assert _true_relres(c, c.op.to_planes(X), b) <= 1e-10 * 1.05
    ref = opcg.pcg(c.m3, c.L, b, 1e-10, precond="amg", amg_opts=h.opts, x0=x0)
    assert abs(st["iters"] - ref.iters[0]) <= max(2, math.ceil(0.02 * ref.iters[0]))


def test_arguments_are_checked():
    import paper_2508_06710_amd as fvx
    c = Case(inputs.channel_base(12, 10), 4)
    amg = fvx.Amg(c.op, coarse_max=20)
    other = Case(inputs.channel_base(12, 10), 4)
    B = c.op.to_rows(inputs.rhs_uniform(118, c.m3.N))
    with pytest.raises(fvx.FvxError):
        other.op.solve(B, amg=amg)                      # hierarchy of another operator
    with pytest.raises(fvx.FvxError):
        c.op.solve(B, precond=fvx.PRECOND_AMG)          # no hierarchy
    with pytest.raises(fvx.FvxError):
        fvx.solve_batch([c.op, c.op], [B, B], amg=amg)  # batches: single solves only
    for kw in (dict(degree=1), dict(degree=9), dict(ratio=1.0), dict(beta=0.0), dict(coarse_max=0),
               dict(coarse_max=4096), dict(max_levels=0), dict(max_levels=17), dict(mode_cells=-1),
               dict(mode_cells=2049)):
        with pytest.raises(fvx.FvxError):
            fvx.Amg(c.op, **kw)
    big = Case(inputs.channel_base(40, 30), 4)          # 4800 unknowns
    with pytest.raises(fvx.FvxError):
        fvx.Amg(big.op, max_levels=1, mode_cells=0)     # coarsest level above 2048 unknowns
    m = fvx.Mesh.from_spec(inputs.channel_base(12, 10))
    s13 = fvx.Operator(m, 4, 0.5, fvx.PERIODIC_Z, stencil=13)
    with pytest.raises(fvx.FvxError):
        fvx.Amg(s13)
    R = c.op.to_rows(inputs.rhs_uniform(119, c.m3.N))
    with pytest.raises(fvx.FvxError):
        amg.apply(R, Z=R)                                # aliasing
