"""Batched solves: uneven problems advanced together must give, per problem,
exactly (bitwise) the result of the single-problem solve, and each must meet
its tolerance by the oracle's residual."""
import math

import numpy as np
import pytest
import torch

import inputs
import oracle
from helpers import Case

pytestmark = pytest.mark.gpu


def _cases():
    return [
        Case(inputs.channel_base(16, 12), 4),
        Case(inputs.channel_base(24, 20), 8),
        Case(inputs.channel_base(13, 9), 6, coupling=0),
        Case(inputs.convection_base(10, 14), 16, dirichlet=True),
        Case(inputs.unit_square_triangles(7), 3),
        Case(inputs.channel_base(32, 32), 32),
    ]


def _rel(c, x, b):
    ng = c.m3.n_groups()
    bp = oracle.project_mean(b, ng)
    r = bp - oracle.spmv(c.L, x)
    if c.coupling == 0 and c.k > 1:
        return max(np.linalg.norm(rr) / np.linalg.norm(bb) for rr, bb in zip(r.reshape(c.k, -1), bp.reshape(c.k, -1)))
    return np.linalg.norm(r) / np.linalg.norm(bp)


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_batch_is_bitwise_equal_to_single_solves(precision):
    cases = _cases()
    fvx = cases[0].fvx
    kw = dict(rtol=1e-10)
    if precision == "mixed":
        kw.update(precision=fvx.MIXED, inner_rtol=1e-4)
    bs = [inputs.rhs_uniform(100 + i, c.m3.N) for i, c in enumerate(cases)]
    Bs = [c.op.to_rows(b) for c, b in zip(cases, bs)]
    singles = [c.op.solve(B, **kw) for c, B in zip(cases, Bs)]
    Xs, stats = fvx.solve_batch([c.op for c in cases], Bs, **kw)
    for i, c in enumerate(cases):
        X1, s1 = singles[i]
        assert torch.equal(X1, Xs[i]), f"problem {i} differs"
        assert s1["iters"] == stats[i]["iters"] and s1["outer"] == stats[i]["outer"]
        assert _rel(c, c.op.to_planes(Xs[i]), bs[i]) <= 1.05e-10


def test_batch_reports_per_problem_status():
    cases = _cases()[:3]
    fvx = cases[0].fvx
    Bs = [c.op.to_rows(inputs.rhs_uniform(7 + i, c.m3.N)) for i, c in enumerate(cases)]
    _, stats = fvx.solve_batch([c.op for c in cases], Bs, rtol=1e-12, max_iter=3, allow_not_converged=True)
    assert all(s["status"] == 1 and s["iters"] == 3 for s in stats)


def test_many_small_problems_in_one_batch():
    """300 problems (more than one block of done flags per poll, and a binary
    search over many block ranges): each converges with the oracle's residual
    and equals its single solve bitwise."""
    spec = inputs.channel_base(6, 5)
    cases = [Case(spec, 2 + (i % 5), math.pi / (2 + (i % 5)), with_f32=False) for i in range(5)]
    import paper_2508_06710_amd as fvx
    ops, Bs, bs, cs = [], [], [], []
    for i in range(300):
        c = cases[i % 5]
        b = inputs.rhs_uniform(400 + i, c.op.n_b * c.k)
        ops.append(c.op)
        Bs.append(c.op.to_rows(b))
        bs.append(b)
        cs.append(c)
    Xs, sts = fvx.solve_batch(ops, Bs, rtol=1e-10)
    for i in (0, 1, 2, 3, 4, 150, 299):
        c, b = cs[i], bs[i]
        X1, st1 = c.op.solve(Bs[i], rtol=1e-10)
        assert torch.equal(Xs[i], X1) and sts[i]["iters"] == st1["iters"]
        bp = oracle.project_mean(b, 1)
        x = c.op.to_planes(Xs[i])
        assert np.linalg.norm(bp - oracle.spmv(c.L, x)) <= 1.0001e-10 * np.linalg.norm(bp)
    assert all(s["status"] == 0 for s in sts)
