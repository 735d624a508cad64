"""Pins of the oracle's preconditioned CG (oracle/pcg.py) against facts that
do not come from it: the C oracle's plain CG, the identity between Jacobi-
preconditioned CG and plain CG on the symmetrically scaled system, the
closed-form residual polynomial of the Chebyshev semi-iteration, and dense
direct solves."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import inputs
import oracle
from oracle import pcg as opcg


def _case(spec, k, dirichlet=False, coupling=oracle.PERIODIC_Z):
    m3 = oracle.Mesh3D(oracle.geometry(spec), k, math.pi / k, coupling, dirichlet)
    return m3, m3.lap().tocsr()


def test_unpreconditioned_equals_the_c_oracle_cg():
    m3, L = _case(inputs.channel_base(12, 10), 4)
    b = inputs.rhs_uniform(50, m3.N)
    ref = oracle.cg(m3, L, b, 1e-10)
    got = opcg.pcg(m3, L, b, 1e-10, precond="none")
    assert got.iters == ref.iters
    assert np.max(np.abs(got.x - ref.x)) <= 1e-9 * np.max(np.abs(ref.x))


def test_jacobi_with_a_constant_diagonal_is_plain_cg():
    spec = inputs.CartSpec(8, 6, 2 * math.pi, 0.0, 2 * math.pi, 0.0, True, True)  # uniform periodic box
    m3 = oracle.Mesh3D(oracle.geometry(spec), 5, 0.7, oracle.PERIODIC_Z)
    L = m3.lap().tocsr()
    assert np.ptp(L.diagonal()) <= 1e-12 * abs(L.diagonal()).max()
    b = inputs.rhs_uniform(51, m3.N)
    a = opcg.pcg(m3, L, b, 1e-10, precond="none")
    j = opcg.pcg(m3, L, b, 1e-10, precond="jacobi")
    assert a.iters == j.iters
    assert np.max(np.abs(a.x - j.x)) <= 1e-10 * np.max(np.abs(a.x))


@pytest.mark.parametrize("m", [1, 3, 7, 15])
def test_jacobi_iterates_are_scaled_cg_iterates(m):
    """PCG with M = D and CG on S A S y = S b (S = D^-1/2) produce x = S y
    after every iteration (Dirichlet walls: nonsingular)."""
    m3, L = _case(inputs.channel_base(10, 9), 3, dirichlet=True)
    b = inputs.rhs_uniform(52, m3.N)
    got = opcg.pcg(m3, L, b, 1e-300, precond="jacobi", max_iter=m)
    s = 1.0 / np.sqrt(-L.diagonal())
    S = sp.diags(s)
    Ls = (S @ L @ S).tocsr()
    ref = oracle.cg(m3, Ls, s * b, 1e-300, max_iter=m)
    assert got.iters == [m] and ref.iters == [m]
    xs = s * ref.x
    assert np.max(np.abs(got.x - xs)) <= 1e-10 * np.max(np.abs(xs))


@pytest.mark.parametrize("degree", [1, 2, 3, 4, 6])
@pytest.mark.parametrize("ratio", [4.0, 30.0])
def test_chebyshev_apply_matches_its_closed_form_polynomial(degree, ratio):
    m3, L = _case(inputs.channel_base(6, 5), 3, dirichlet=True)
    A = (-L).tocsr()
    d = A.diagonal()
    dinv = 1.0 / d
    r = inputs.uniform(53, degree, m3.N)
    z = opcg.chebyshev_apply(A, dinv, r, degree, ratio)
    Mh = (np.diag(np.sqrt(dinv)) @ A.toarray() @ np.diag(np.sqrt(dinv)))
    lam, V = np.linalg.eigh(Mh)
    assert lam.max() <= opcg.CHEB_BMAX * (1 + 1e-12)  # the Gershgorin bound the method relies on
    p = opcg.chebyshev_polynomial(lam, degree, ratio)
    zc = np.sqrt(dinv) * (V @ (p * (V.T @ (np.sqrt(dinv) * r))))
    assert np.max(np.abs(z - zc)) <= 1e-11 * np.max(np.abs(zc))


def test_chebyshev_degree_one_is_jacobi():
    m3, L = _case(inputs.channel_base(12, 10), 4)
    b = inputs.rhs_uniform(54, m3.N)
    j = opcg.pcg(m3, L, b, 1e-10, precond="jacobi")
    c = opcg.pcg(m3, L, b, 1e-10, precond="chebyshev", degree=1)
    assert j.iters == c.iters
    assert np.max(np.abs(j.x - c.x)) <= 1e-10 * np.max(np.abs(j.x))


@pytest.mark.parametrize("precond,degree", [("jacobi", 1), ("chebyshev", 3), ("chebyshev", 5)])
@pytest.mark.parametrize("dirichlet", [False, True])
def test_pcg_matches_dense_direct_solve(precond, degree, dirichlet):
    m3, L = _case(inputs.channel_base(5, 4), 3, dirichlet=dirichlet)
    b = inputs.rhs_uniform(55, m3.N)
    got = opcg.pcg(m3, L, b, 1e-13, precond=precond, degree=degree)
    assert got.status == [0]
    xd = oracle.dense_solve(L.toarray(), b if dirichlet else oracle.project_mean(b, 1), 0 if dirichlet else 1)
    assert np.max(np.abs(got.x - xd)) <= 1e-9 * np.max(np.abs(xd))


def test_chebyshev_needs_fewer_iterations_as_the_degree_grows():
    m3, L = _case(inputs.channel_base(32, 32), 8)
    b = inputs.rhs_uniform(56, m3.N)
    its = [opcg.pcg(m3, L, b, 1e-8, precond="chebyshev", degree=d).iters[0] for d in (1, 2, 4, 8)]
    assert its[0] > its[1] > its[2] > its[3], its
