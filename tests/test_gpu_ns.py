"""The Heun-RK3 projection step on the GPU (fvx_ns_step) against the
oracle's step on assembled matrices: cell and face velocities after one and
three steps, the divergence-free face velocities, and the Taylor-Green
vortex."""
import math

import numpy as np
import pytest

import inputs
import oracle
from helpers import Case
from oracle import ns

pytestmark = pytest.mark.gpu


def _to_dev(c, U, us):
    kF = c.k * c.m3.g.n_faces
    Ud = [c.op.to_rows(u) for u in U]
    Uf = c.op.to_rows(us[:kF], rows=c.op.F_b)
    Wz = c.op.to_rows(us[kF:]) if c.op.zfaces else None
    return Ud, Uf, Wz


def _from_dev(c, Ud, Uf, Wz):
    U = [c.op.to_planes(u) for u in Ud]
    us = c.op.to_planes(Uf, rows=c.op.F_b)
    if Wz is not None:
        us = np.concatenate([us, c.op.to_planes(Wz)])
    return U, us


@pytest.mark.parametrize("spec,k,coupling", [
    (inputs.CartSpec(16, 12, 2 * math.pi, 0.0, 2 * math.pi, 0.0, True, True), 4, 1),
    (inputs.channel_base(20, 14), 4, 1),
    (inputs.unit_square_triangles(6), 3, 1),
    (inputs.channel_base(12, 10), 3, 0),
])
@pytest.mark.parametrize("nsteps", [1, 3])
def test_step_matches_oracle(spec, k, coupling, nsteps):
    c = Case(spec, k, coupling=coupling)
    o = ns.NSOracle(spec, c.m3)
    U0 = [inputs.uniform(100, d, c.m3.N) for d in range(3)]
    U, us, _ = o.project(U0, 1.0, 1e-13)
    Ud, Uf, Wz = _to_dev(c, U, us)
    P = c.op.zeros()
    dt, nu = 0.01, 0.05
    for _ in range(nsteps):
        st = c.op.ns_step(Ud, Uf, Wz, P, dt, nu, rtol=1e-13)
        U, us, _ = o.step(U, us, dt, nu)
    Ug, usg = _from_dev(c, Ud, Uf, Wz)
    scale = max(np.abs(u).max() for u in U)
    for d in range(3):
        assert np.max(np.abs(Ug[d] - U[d])) <= 1e-9 * scale, d
    assert np.max(np.abs(usg - us)) <= 1e-9 * np.abs(us).max()
    assert np.max(np.abs(c.M @ usg)) <= 1e-10 * np.abs(c.M).max() * np.abs(usg).max()
    assert st["iters"] > 0


def test_taylor_green_vortex_on_the_gpu():
    n, nu, T, steps = 32, 0.1, 0.25, 25
    spec = inputs.CartSpec(n, n, 2 * math.pi, 0.0, 2 * math.pi, 0.0, True, True)
    c = Case(spec, 1)
    g = c.m3.g
    o = ns.NSOracle(spec, c.m3)
    U0 = [np.sin(g.cx) * np.cos(g.cy), -np.cos(g.cx) * np.sin(g.cy), np.zeros(c.m3.N)]
    U, us, _ = o.project(U0, 1.0, 1e-13)
    Ud, Uf, Wz = _to_dev(c, U, us)
    P = c.op.zeros()
    for _ in range(steps):
        c.op.ns_step(Ud, Uf, Wz, P, T / steps, nu, rtol=1e-12)
    Ug, _ = _from_dev(c, Ud, Uf, Wz)
    ex = np.sin(g.cx) * np.cos(g.cy) * math.exp(-2 * nu * T)
    err = np.max(np.abs(Ug[0] - ex))
    assert err <= 2e-3  # the scheme's O(h^2) error at n = 32 (about 1e-3)
    assert np.max(np.abs(Ug[2])) <= 1e-14


def test_step_with_a_no_slip_viscous_operator():
    """L_v from a Dirichlet-wall operator (no slip) while the pressure keeps
    zero-flux walls."""
    spec = inputs.channel_base(16, 12)
    c = Case(spec, 4)
    fvx = c.fvx
    visc = fvx.Operator(fvx.Mesh.from_spec(spec), 4, c.dz, fvx.PERIODIC_Z, fvx.DIRICHLET, with_f32=False)
    mv = oracle.Mesh3D(oracle.geometry(spec), 4, c.dz, oracle.PERIODIC_Z, True)
    o = ns.NSOracle(spec, c.m3, visc_m3=mv)
    U, us, _ = o.project([inputs.uniform(101, d, c.m3.N) for d in range(3)], 1.0, 1e-13)
    Ud, Uf, Wz = _to_dev(c, U, us)
    P = c.op.zeros()
    c.op.ns_step(Ud, Uf, Wz, P, 0.01, 0.2, visc=visc, rtol=1e-13)
    U, us, _ = o.step(U, us, 0.01, 0.2)
    Ug, _ = _from_dev(c, Ud, Uf, Wz)
    for d in range(3):
        assert np.max(np.abs(Ug[d] - U[d])) <= 1e-9 * np.abs(U[d]).max()


def test_ns_step_argument_checks():
    c = Case(inputs.channel_base(8, 8), 4)
    fvx = c.fvx
    Ud = [c.op.zeros() for _ in range(3)]
    Uf, Wz, P = c.op.zeros(c.op.F_b), c.op.zeros(), c.op.zeros()
    with pytest.raises(fvx.FvxError):
        c.op.ns_step(Ud, Uf, Wz, P, -0.1, 0.1)
    with pytest.raises(fvx.FvxError):
        c.op.ns_step(Ud, Uf, Wz, P, 0.1, 0.1, precision=fvx.MIXED)
    other = fvx.Operator(fvx.Mesh.from_spec(inputs.channel_base(8, 8)), 2, 0.5, fvx.PERIODIC_Z, with_f32=False)
    with pytest.raises(fvx.FvxError):
        c.op.ns_step(Ud, Uf, Wz, P, 0.1, 0.1, visc=other)
