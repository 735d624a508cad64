"""Pins of the oracle's convective operator C(u_s) = M U_s Pi (oracle/ns.py):
a closed form on a uniform periodic box, C 1 = M u_s, and skew-symmetry
(kinetic-energy conservation) for divergence-free face velocities obtained
by projection with a dense solve."""
import math

import numpy as np
import pytest

import inputs
import oracle
from oracle import ns


def _m3(spec, k, coupling=oracle.PERIODIC_Z):
    return oracle.Mesh3D(oracle.geometry(spec), k, 0.45, coupling)


def test_uniform_x_velocity_on_a_periodic_box_is_a_central_difference():
    nx, ny, k = 12, 5, 3
    spec = inputs.CartSpec(nx, ny, 2 * math.pi, 0.0, 1.0, 0.0, True, True)
    m3 = _m3(spec, k)
    M = m3.div()
    g = m3.g
    kF = k * g.n_faces
    us = np.zeros(m3.F3)
    # in-plane faces whose normal points along +x carry u0; the rest carry 0
    u0 = 0.7
    dx = g.cx[g.c2] - g.cx[g.c1]
    xf = np.abs(np.abs(dx) - 2 * math.pi / nx) < 1e-12
    xf |= np.abs(np.abs(dx) - (2 * math.pi - 2 * math.pi / nx)) < 1e-12  # faces across the period
    sgn = np.where(np.abs(dx) < math.pi, np.sign(dx), -np.sign(dx))  # +1 when c1 -> c2 points along +x
    per_plane = np.where(xf, u0 * sgn, 0.0)
    us[:kF] = np.tile(per_plane, k)
    x = np.tile(g.cx, k)
    phi = np.sin(x)
    hx, hy, dz = 2 * math.pi / nx, 1.0 / ny, 0.45
    expect = u0 * hy * dz * np.cos(x) * math.sin(hx)
    got = ns.convective(M, us) @ phi
    assert np.max(np.abs(got - expect)) <= 1e-13


@pytest.mark.parametrize("spec,k", [(inputs.channel_base(9, 7), 4), (inputs.unit_square_triangles(4), 3),
                                    (inputs.convection_base(5, 6), 2)])
def test_constant_field_gives_the_divergence(spec, k):
    m3 = _m3(spec, k)
    M = m3.div()
    us = inputs.normal(80, 0, m3.F3)
    assert np.max(np.abs(ns.convective(M, us) @ np.ones(m3.N) - M @ us)) <= 1e-13 * np.abs(M @ us).max()


@pytest.mark.parametrize("spec,k,coupling", [(inputs.channel_base(9, 7), 4, oracle.PERIODIC_Z),
                                             (inputs.unit_square_triangles(4), 3, oracle.PERIODIC_Z),
                                             (inputs.convection_base(5, 6), 2, oracle.PERIODIC_Z),
                                             (inputs.channel_base(6, 5), 3, oracle.NONE)])
def test_skew_symmetric_for_divergence_free_velocity(spec, k, coupling):
    m3 = _m3(spec, k, coupling)
    M, G, L = m3.div(), m3.grad(), m3.lap()
    u = inputs.normal(81, 0, m3.F3)
    p = oracle.dense_solve(L.toarray(), oracle.project_mean(M @ u, m3.n_groups()), m3.n_groups())
    us = u - G @ p
    assert np.max(np.abs(M @ us)) <= 1e-10 * np.abs(M @ u).max()
    C = ns.convective(M, us).toarray()
    assert np.max(np.abs(C + C.T)) <= 1e-10 * np.abs(C).max()
    phi = inputs.uniform(82, 0, m3.N)
    assert abs(phi @ C @ phi) <= 1e-10 * np.abs(C).max() * (phi @ phi)


def test_uniform_velocity_survives_interpolation_both_ways():
    """Gamma_sc Gamma_cs reproduces a uniform velocity on a uniform periodic
    box (the normal and volume-weight conventions of both operators)."""
    spec = inputs.CartSpec(6, 5, 1.2, 0.0, 1.0, 0.0, True, True)
    m3 = oracle.Mesh3D(oracle.geometry(spec), 4, 0.3, oracle.PERIODIC_Z)
    o = ns.NSOracle(spec, m3)
    U = np.concatenate([np.full(m3.N, 0.7), np.full(m3.N, -1.3), np.full(m3.N, 0.4)])
    assert np.max(np.abs(o.Gsc @ (o.Gcs @ U) - U)) <= 1e-13


def test_triangle_normals_are_unit_and_oriented():
    spec = inputs.unit_square_triangles(4)
    g = oracle.geometry(spec)
    nx, ny = ns.face_normals(spec, g)
    assert np.allclose(np.hypot(nx, ny), 1.0, atol=1e-14)
    assert np.all(nx * (g.cx[g.c2] - g.cx[g.c1]) + ny * (g.cy[g.c2] - g.cy[g.c1]) > 0)


def _tgv_error(n, nu=0.1, T=0.25, steps=25):
    spec = inputs.CartSpec(n, n, 2 * math.pi, 0.0, 2 * math.pi, 0.0, True, True)
    m3 = oracle.Mesh3D(oracle.geometry(spec), 1, 1.0, oracle.PERIODIC_Z)
    o = ns.NSOracle(spec, m3)
    g = m3.g
    U = [np.sin(g.cx) * np.cos(g.cy), -np.cos(g.cx) * np.sin(g.cy), np.zeros(m3.N)]
    U, us, _ = o.project(U, 1.0, 1e-13)
    dt = T / steps
    for _ in range(steps):
        U, us, _ = o.step(U, us, dt, nu)
    decay = math.exp(-2 * nu * T)
    ex = np.sin(g.cx) * np.cos(g.cy) * decay
    return np.max(np.abs(U[0] - ex)), np.max(np.abs(o.M @ us))


def test_taylor_green_vortex_second_order_and_divergence_free():
    e16, d16 = _tgv_error(16)
    e32, d32 = _tgv_error(32)
    rate = math.log2(e16 / e32)
    assert 1.8 <= rate <= 2.3, (e16, e32, rate)
    assert d16 <= 1e-11 and d32 <= 1e-11
