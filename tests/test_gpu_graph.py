"""CG iterations replayed from HIP graphs (launch = LAUNCH_GRAPH) against the
same solves launched phase by phase (LAUNCH_PHASES).

The graphs hold the same kernels with the same arguments in the same order,
so X, the iteration counts and the statistics must be bitwise equal.  Each
configuration is solved twice in graph mode: the second solve replays the
cached graphs, with eager work (the set-up kernels, the polls) between the
replays.  Changing the operator's CG tile or the tolerance between solves
must not replay a graph captured for the old tile or tolerance.  Parity with
the oracle: the true residual by the oracle's assembled matrix."""
import numpy as np
import pytest
import torch

import inputs
import oracle
from helpers import Case

pytestmark = pytest.mark.gpu


def _relres(c, x, b):
    ng = c.m3.n_groups()
    bp = oracle.project_mean(b, ng)
    r = bp - oracle.spmv(c.L, x)
    if c.coupling == 0 and c.k > 1:
        return max(np.linalg.norm(rr) / np.linalg.norm(bb) for rr, bb in zip(r.reshape(c.k, -1), bp.reshape(c.k, -1)))
    return np.linalg.norm(r) / np.linalg.norm(bp)


def _same(a, b):
    Xa, sa = a
    Xb, sb = b
    assert torch.equal(Xa, Xb)
    for key in ("status", "iters", "outer", "relres_rec", "relres_true", "r0_over_b"):
        assert sa[key] == sb[key], (key, sa[key], sb[key])


SOLVES = [
    ({}, "plain"),
    ({"precond": 1}, "jacobi"),
    ({"precond": 2, "cheb_degree": 3, "cheb_ratio": 30.0}, "chebyshev"),
    ({"precision": 2, "inner_rtol": 1e-4}, "mixed"),
]


@pytest.mark.parametrize("spec,k,coupling", [
    (inputs.channel_base(24, 20), 8, 1),
    (inputs.channel_base(13, 9), 5, 0),          # independent planes: the folds of per-column partials
    (inputs.unit_square_triangles(7), 3, 1),
])
@pytest.mark.parametrize("kw,name", SOLVES, ids=[n for _, n in SOLVES])
@pytest.mark.parametrize("poll", [64, 5])        # 5: intervals of odd lengths (graphs of 1, 2 and 4 iterations)
def test_graph_equals_phases(spec, k, coupling, kw, name, poll):
    c = Case(spec, k, coupling=coupling, with_f32=True)
    fvx = c.fvx
    b = inputs.rhs_uniform(17, c.m3.N)
    B = c.op.to_rows(b)
    phases = c.op.solve(B, rtol=1e-10, poll_every=poll, launch=fvx.LAUNCH_PHASES, **kw)
    first = c.op.solve(B, rtol=1e-10, poll_every=poll, launch=fvx.LAUNCH_GRAPH, **kw)
    again = c.op.solve(B, rtol=1e-10, poll_every=poll, launch=fvx.LAUNCH_GRAPH, **kw)
    _same(phases, first)
    _same(phases, again)
    if name in ("plain", "jacobi") and poll == 5:
        assert phases[1]["iters"] > 5          # iterations after the first poll ran from graphs
    assert _relres(c, c.op.to_planes(first[0]), b) <= 1.05e-10


def test_graph_multigrid():
    c = Case(inputs.channel_base(32, 24), 8, with_f32=True)
    fvx = c.fvx
    amg = fvx.Amg(c.op, coarse_max=64, mode_cells=0)
    b = inputs.rhs_uniform(23, c.m3.N)
    B = c.op.to_rows(b)
    for kw in ({}, {"precision": fvx.MIXED, "inner_rtol": 1e-4}):
        phases = c.op.solve(B, rtol=1e-10, amg=amg, poll_every=4, launch=fvx.LAUNCH_PHASES, **kw)
        for _ in range(2):
            _same(phases, c.op.solve(B, rtol=1e-10, amg=amg, poll_every=4, launch=fvx.LAUNCH_GRAPH, **kw))
        assert _relres(c, c.op.to_planes(phases[0]), b) <= 1.05e-10
    # a new hierarchy of the same operator (a new serial) is not served from
    # the old one's graphs; its coarsest level is solved per plane mode
    amg2 = fvx.Amg(c.op, coarse_max=20, degree=3, mode_cells=50)
    assert amg2.n_levels >= 3
    phases = c.op.solve(B, rtol=1e-10, amg=amg2, poll_every=4, launch=fvx.LAUNCH_PHASES)
    _same(phases, c.op.solve(B, rtol=1e-10, amg=amg2, poll_every=4, launch=fvx.LAUNCH_GRAPH))


def test_graph_batch():
    cases = [
        Case(inputs.channel_base(16, 12), 4),
        Case(inputs.channel_base(24, 20), 8),
        Case(inputs.channel_base(13, 9), 6, coupling=0),
        Case(inputs.convection_base(10, 14), 16, dirichlet=True),
        Case(inputs.unit_square_triangles(7), 3),
    ]
    fvx = cases[0].fvx
    Bs = [c.op.to_rows(inputs.rhs_uniform(300 + i, c.m3.N)) for i, c in enumerate(cases)]
    ops = [c.op for c in cases]
    for kw in ({}, {"precision": fvx.MIXED, "inner_rtol": 1e-4}):
        Xp, sp = fvx.solve_batch(ops, Bs, rtol=1e-10, poll_every=7, launch=fvx.LAUNCH_PHASES, **kw)
        for _ in range(2):
            Xg, sg = fvx.solve_batch(ops, Bs, rtol=1e-10, poll_every=7, launch=fvx.LAUNCH_GRAPH, **kw)
            for i in range(len(cases)):
                _same((Xp[i], sp[i]), (Xg[i], sg[i]))


def test_graph_follows_tile_and_tolerance_changes():
    """Between graph-mode solves the CG tile changes (another launch shape)
    and the tolerance changes (read from the descriptors, not captured):
    every solve equals its phase-by-phase twin."""
    c = Case(inputs.channel_base(40, 24), 16, with_f32=True)
    fvx = c.fvx
    B = c.op.to_rows(inputs.rhs_uniform(29, c.m3.N))
    vec = c.op.get_cg_tile(fvx.F64)[0]
    try:
        for tile in ((vec, 1, 128, 1, 0, 0), (vec, 1, 256, 0, 64, 0), (vec, 1, 128, 1, 0, 1), (vec, 1, 128, 1, 0, 0)):
            c.op.set_cg_tile(*tile, dtype=fvx.F64)
            for rtol in (1e-6, 1e-11):
                p = c.op.solve(B, rtol=rtol, poll_every=16, launch=fvx.LAUNCH_PHASES)
                g = c.op.solve(B, rtol=rtol, poll_every=16, launch=fvx.LAUNCH_GRAPH)
                _same(p, g)
    finally:
        c.op.set_cg_tile(block=0, dtype=fvx.F64)


def test_graph_launch_mode_checked():
    c = Case(inputs.channel_base(8, 6), 2)
    fvx = c.fvx
    B = c.op.to_rows(inputs.rhs_uniform(3, c.m3.N))
    with pytest.raises(fvx.FvxError):
        c.op.solve(B, launch=2)


def test_graph_cache_eviction():
    """More solve configurations than the cache keeps (16): the least
    recently used are dropped (after a device synchronisation) and captured
    again when they come back; every solve equals its phase-by-phase twin."""
    import paper_2508_06710_amd as fvx
    cases = [Case(inputs.channel_base(6 + i % 6, 5 + i // 6), 2 + i % 3, with_f32=False) for i in range(18)]
    Bs = [c.op.to_rows(inputs.rhs_uniform(500 + i, c.m3.N)) for i, c in enumerate(cases)]
    ref = [c.op.solve(B, rtol=1e-10, poll_every=4, launch=fvx.LAUNCH_PHASES) for c, B in zip(cases, Bs)]
    for _ in range(2):
        for c, B, r in zip(cases, Bs, ref):
            _same(r, c.op.solve(B, rtol=1e-10, poll_every=4, launch=fvx.LAUNCH_GRAPH))
