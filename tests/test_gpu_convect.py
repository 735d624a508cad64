"""The convective operator C(u_s) = M U_s Pi on the GPU (fvx_convect)
against the oracle's assembled C, element by element, and its
skew-symmetry for a divergence-free field projected by the library."""
import numpy as np
import pytest

import inputs
import oracle
from helpers import Case
from oracle import ns

pytestmark = pytest.mark.gpu


def _bound(M, us, phi):
    Pi = ns.midpoint_interpolation(M)
    return abs(M) @ (np.abs(us) * (abs(Pi) @ np.abs(phi)))


@pytest.mark.parametrize("spec,k,coupling", [
    (inputs.channel_base(64, 64), 8, 1),
    (inputs.channel_base(13, 9), 1, 1),
    (inputs.channel_base(13, 9), 2, 1),
    (inputs.channel_base(13, 9), 5, 0),
    (inputs.convection_base(12, 20), 16, 1),
    (inputs.unit_square_triangles(8), 4, 1),
    (inputs.channel_base(37, 29), 66, 1),
    (inputs.channel_base(20, 12), 130, 1),
])
def test_convect_matches_oracle(spec, k, coupling):
    c = Case(spec, k, coupling=coupling)
    fvx = c.fvx
    u = inputs.normal(90, 0, c.m3.F3)
    phi = inputs.uniform(91, 0, c.m3.N)
    kF = k * c.m3.g.n_faces
    Uf = c.op.to_rows(u[:kF], rows=c.op.F_b)
    Wz = c.op.to_rows(u[kF:]) if c.op.zfaces else None
    for dtype in (fvx.F64, fvx.F32):
        if dtype == fvx.F32:
            Uf32 = c.op.to_rows(u[:kF].astype(np.float32), rows=c.op.F_b, dtype=fvx.F32)
            Wz32 = c.op.to_rows(u[kF:].astype(np.float32), dtype=fvx.F32) if c.op.zfaces else None
            P32 = c.op.to_rows(phi.astype(np.float32), dtype=fvx.F32)
            y = c.op.to_planes(c.op.convect(Uf32, Wz32, P32), dtype=fvx.F32).astype(np.float64)
            u64, p64 = u.astype(np.float32).astype(np.float64), phi.astype(np.float32).astype(np.float64)
            ref = ns.convective(c.M, u64) @ p64
            bound = _bound(c.M, u64, p64)
            n = np.diff(c.M.indptr)
            assert np.all(np.abs(y - ref) <= (3 * n + 6) * 2.0 ** -24 * bound + 1e-30)
        else:
            y = c.op.to_planes(c.op.convect(Uf, Wz, c.op.to_rows(phi)))
            ref = ns.convective(c.M, u) @ phi
            bound = _bound(c.M, u, phi)
            z = bound == 0
            assert np.all(y[z] == 0)
            assert np.max(np.abs(y - ref)[~z] / bound[~z]) <= 1e-12


def test_energy_conserving_for_a_projected_velocity():
    """Face velocities made divergence-free by the library's own Poisson
    solve: phi^T C phi vanishes and C is skew on random pairs."""
    c = Case(inputs.channel_base(48, 32), 8)
    fvx = c.fvx
    u = inputs.normal(92, 0, c.m3.F3)
    kF = 8 * c.m3.g.n_faces
    Uf, Wz = c.op.to_rows(u[:kF], rows=c.op.F_b), c.op.to_rows(u[kF:])
    D = c.op.div(Uf, Wz)
    P, st = c.op.solve(D, rtol=1e-13)
    c.op.grad_axpy(-1.0, P, Uf, Wz)
    d = c.op.to_planes(c.op.div(Uf, Wz))
    assert np.linalg.norm(d) <= 1e-11 * np.linalg.norm(c.op.to_planes(D))
    a, b = inputs.uniform(93, 0, c.m3.N), inputs.uniform(93, 1, c.m3.N)
    Ca = c.op.to_planes(c.op.convect(Uf, Wz, c.op.to_rows(a)))
    Cb = c.op.to_planes(c.op.convect(Uf, Wz, c.op.to_rows(b)))
    scale = np.abs(Ca).max() * np.abs(b).max() * c.m3.N
    assert abs(b @ Ca + a @ Cb) <= 1e-12 * scale
    assert abs(a @ Ca) <= 1e-12 * scale


def test_convect_argument_checks():
    c = Case(inputs.channel_base(8, 8), 4)
    fvx = c.fvx
    X = c.op.zeros()
    Uf = c.op.zeros(c.op.F_b)
    with pytest.raises(fvx.FvxError):
        c.op.convect(Uf, None, X)  # coupled planes need Wz
    with pytest.raises(fvx.FvxError):
        c.op.convect(Uf, X, X, Out=X)  # Out aliases an input
