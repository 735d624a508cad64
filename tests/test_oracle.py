"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compare the oracle with itself: each checks a closed form, an
invariant, a textbook special case, a brute-force dense computation, a
convergence order, or a value the paper prints.
"""
import math
import os

import numpy as np
import pytest

import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mesh(orc, spec, k, dz, coupling=1, dirichlet=False):
    return orc.Mesh3D(orc.geometry(spec), k, dz, coupling, dirichlet)


# ---------------------------------------------------------------- geometry

def test_cell_volumes_fill_the_box(orc):
    spec = inputs.channel_base(64, 64)
    m = _mesh(orc, spec, 8, math.pi / 8)
    assert abs(m.cell_volumes().sum() - 2 * math.pi * 2 * math.pi) < 1e-12


def test_stretched_grid_symmetric_and_clustered(orc):
    g = orc.cart_geometry(inputs.channel_base(8, 32))
    cy = g.cy.reshape(32, 8)[:, 0]
    assert np.allclose(cy, -cy[::-1], atol=1e-15, rtol=0)
    dy = g.wdist.reshape(-1)  # half heights of wall cells
    h = 2 * (g.area.reshape(32, 8)[:, 0] / (2 * math.pi / 8))
    assert h[0] < h[8] < h[16]              # clustered at the walls
    assert np.all(dy > 0)


def test_channel_first_cell_matches_printed_y_plus(orc):
    """Section 4.1 prints y+ = 0.65 at the wall for 160 tanh cells, gamma 1.5."""
    vals = {}
    with open(os.path.join(GOLDEN, "channel_grid.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                key, v = line.split()
                vals[key] = float(v)
    spec = inputs.CartSpec(1, int(vals["ny"]), 1.0, -1.0, 1.0, vals["gamma"], True, False)
    g = orc.cart_geometry(spec)
    dy_wall = g.area[0]  # unit-width column: area = first cell height
    y_plus = vals["re_tau"] * dy_wall
    assert abs(y_plus - vals["y_plus_wall"]) / vals["y_plus_wall"] < 0.06


def test_triangle_geometry_tiles_the_square(orc):
    t = inputs.unit_square_triangles(4)
    g = orc.tri_geometry(t)
    assert abs(g.area.sum() - 1.0) < 1e-14
    assert abs(g.wlen.sum() - 4.0) < 1e-14   # boundary edges = perimeter
    assert np.all(g.dist > 0) and np.all(g.wdist > 0)
    # Euler: interior faces = (3 T - boundary) / 2
    assert g.n_faces == (3 * g.n_cells - g.n_walls) // 2


# ---------------------------------------------------------------- Laplacian

@pytest.mark.parametrize("k,coupling", [(1, 1), (2, 1), (3, 1), (8, 1), (4, 0)])
def test_laplacian_symmetric_zero_rowsum_nsd(orc, k, coupling):
    m = _mesh(orc, inputs.channel_base(12, 10), k, math.pi / k, coupling)
    L = m.lap()
    assert abs(L - L.T).max() == 0.0
    absrow = abs(L).sum(axis=1).A1
    assert np.all(np.abs(L.sum(axis=1).A1) <= 8 * np.finfo(float).eps * absrow)
    rng = np.random.default_rng(0)
    X = rng.standard_normal((m.N, 50))
    assert np.all(np.einsum("ij,ij->j", X, L @ X) <= 1e-12)


@pytest.mark.parametrize("k,coupling,dirichlet", [(1, 1, False), (2, 1, False), (3, 1, False),
                                                  (3, 0, False), (2, 1, True)])
def test_dense_spectrum_null_space(orc, k, coupling, dirichlet):
    m = _mesh(orc, inputs.channel_base(4, 3), k, 0.7, coupling, dirichlet)
    ev = np.linalg.eigvalsh(m.dense_lap())
    scale = abs(ev).max()
    n_zero = int(np.sum(np.abs(ev) < 1e-12 * scale))
    assert np.all(ev <= 1e-12 * scale)
    expected = 0 if dirichlet else (k if (coupling == 0 and k > 1) else 1)
    assert n_zero == expected


@pytest.mark.parametrize("a,b,c", [(1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 3, 1), (3, 5, 3)])
def test_uniform_box_fourier_eigenpairs(orc, a, b, c):
    """On a uniform mesh (periodic x and z, zero-flux walls in y) the discrete
    modes cos(2 pi a (i+1/2)/nx) cos(pi b (j+1/2)/ny) cos(2 pi c (l+1/2)/k) are
    exact eigenvectors of the assembled operator with eigenvalue
    -sum_d (face area_d / distance_d) 4 sin^2(theta_d / 2)."""
    nx, ny, k = 8, 6, 4
    Lx, Ly, dz = 2.0, 1.5, 0.3
    spec = inputs.CartSpec(nx, ny, Lx, 0.0, Ly, 0.0, True, False)
    m = _mesh(orc, spec, k, dz)
    dx, dy = Lx / nx, Ly / ny
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    l = np.arange(k)[:, None, None]
    v = (np.cos(2 * math.pi * a * (i + 0.5) / nx) * np.cos(math.pi * b * (j + 0.5) / ny)
         * np.cos(2 * math.pi * c * (l + 0.5) / k)).ravel()
    lam = -((dy * dz / dx) * 4 * math.sin(math.pi * a / nx) ** 2
            + (dx * dz / dy) * 4 * math.sin(math.pi * b / (2 * ny)) ** 2
            + (dx * dy / dz) * 4 * math.sin(math.pi * c / k) ** 2)
    Lv = orc.spmv(m.lap(), v)
    assert np.max(np.abs(Lv - lam * v)) <= 1e-13 * max(1.0, abs(lam)) * np.max(np.abs(v))


def test_dirichlet_wall_adds_half_cell_flux(orc):
    """With p = 0 on the walls, a cell next to a wall loses a/(h/2) on the
    diagonal; the rest of the row is unchanged."""
    spec = inputs.CartSpec(4, 5, 1.0, 0.0, 1.0, 0.0, True, False)
    n = _mesh(orc, spec, 2, 0.5).dense_lap()
    d = _mesh(orc, spec, 2, 0.5, 1, True).dense_lap()
    diff = d - n
    dx, dy, dz = 0.25, 0.2, 0.5
    expect = np.zeros(n.shape[0])
    for l in range(2):
        for i in range(4):
            expect[l * 20 + 0 * 4 + i] = -dx * dz / (dy / 2)
            expect[l * 20 + 4 * 4 + i] = -dx * dz / (dy / 2)
    assert np.allclose(np.diag(diff), expect, rtol=1e-14, atol=0)
    assert np.count_nonzero(diff - np.diag(np.diag(diff))) == 0


# ---------------------------------------------------------------- div / grad

@pytest.mark.parametrize("k,coupling", [(1, 1), (2, 1), (5, 1), (3, 0)])
def test_div_grad_identities(orc, k, coupling):
    m = _mesh(orc, inputs.channel_base(6, 5), k, 0.4, coupling)
    M, G, L = m.div().toarray(), m.grad().toarray(), m.lap().toarray()
    Os = m.face_volumes()
    # M = -(Omega_s G)^T with one rounding per entry
    assert np.allclose(M, -(Os[:, None] * G).T, rtol=4e-16, atol=0)
    # L = M G
    assert np.max(np.abs(M @ G - L)) <= 1e-14 * np.max(np.abs(L))
    # gradient of a constant vanishes; interior fluxes cancel in the total
    assert np.max(np.abs(G @ np.ones(m.N))) == 0.0
    u = np.random.default_rng(1).standard_normal(m.F3)
    assert abs((M @ u).sum()) <= 1e-13 * np.abs(M).sum(axis=1).max() * np.abs(u).max() * m.N


def test_sparse_matches_dense_brute_force(orc):
    for spec in (inputs.channel_base(5, 4), inputs.convection_base(3, 4),
                 inputs.unit_square_triangles(3)):
        for k, coupling, dirichlet in ((1, 1, False), (2, 1, False), (3, 1, True), (3, 0, False)):
            m = _mesh(orc, spec, k, 0.3, coupling, dirichlet)
            assert np.max(np.abs(m.lap().toarray() - m.dense_lap())) <= 4e-16 * np.abs(m.dense_lap()).max() * 4
            assert np.allclose(m.div().toarray(), m.dense_div(), rtol=0, atol=0)
            assert np.allclose(m.grad().toarray(), m.dense_grad(), rtol=1e-15, atol=0)


def test_triangle_operators(orc):
    m = _mesh(orc, inputs.unit_square_triangles(6), 3, 0.25)
    L = m.lap()
    assert abs(L - L.T).max() == 0.0
    assert np.max(np.abs(L.sum(axis=1).A1)) <= 1e-14 * abs(L).max()
    ev = np.linalg.eigvalsh(L.toarray())
    assert ev.max() <= 1e-12 * abs(ev).max()
    assert np.sum(np.abs(ev) < 1e-12 * abs(ev).max()) == 1


# ---------------------------------------------------------------- solves

@pytest.mark.parametrize("k,coupling,dirichlet", [(1, 1, False), (2, 1, False), (3, 1, False),
                                                  (4, 0, False), (3, 1, True)])
def test_cg_matches_dense_direct_solve(orc, k, coupling, dirichlet):
    m = _mesh(orc, inputs.channel_base(6, 5, 0.5), k, 0.6, coupling, dirichlet)
    L = m.lap()
    b = inputs.rhs_uniform(3, m.N)
    r = orc.cg(m, L, b, 1e-15, max_iter=5000)
    ng = m.n_groups()
    xd = orc.dense_solve(m.dense_lap(), orc.project_mean(b, ng), ng)
    assert np.linalg.norm(r.x - xd) <= 1e-12 * np.linalg.norm(xd)
    for rr in r.relres_true:
        assert rr < 1e-13


def test_cg_finite_termination_on_few_distinct_eigenvalues(orc):
    """CG in exact arithmetic ends in at most as many steps as the operator has
    distinct nonzero eigenvalues touched by b.  A uniform 4-cell periodic ring
    extruded into 4 periodic planes has eigenvalues
    -(4 sin^2(pi a/4) + 4 sin^2(pi c/4)) with sin^2 in {0, 1/2, 1}: the nonzero
    sums are {2, 4, 6, 8}, so 4 steps suffice."""
    spec = inputs.CartSpec(4, 1, 4.0, 0.0, 1.0, 0.0, True, False)
    m = _mesh(orc, spec, 4, 1.0)
    b = inputs.rhs_uniform(11, m.N)
    r = orc.cg(m, m.lap(), b, 1e-13, max_iter=50)
    assert r.iters[0] <= 4
    assert r.relres_true[0] < 1e-13


def test_cg_initial_guess_and_zero_rhs(orc):
    m = _mesh(orc, inputs.channel_base(8, 6), 4, 0.5)
    L = m.lap()
    b = inputs.rhs_uniform(5, m.N)
    ref = orc.cg(m, L, b, 1e-12)
    warm = orc.cg(m, L, b, 1e-12, x0=ref.x)
    assert warm.iters[0] <= 1
    zero = orc.cg(m, L, np.ones(m.N), 1e-12)  # constant RHS projects to zero
    assert zero.iters[0] == 0 and np.all(zero.x == 0)


def _mms_error(orc, n, kz, dirichlet):
    spec = inputs.channel_base(n, n, 1.5)
    k = kz
    m = _mesh(orc, spec, k, math.pi / k, 1, dirichlet)
    g = m.g
    z = m.z_centres()
    X = np.tile(g.cx, k)
    Y = np.tile(g.cy, k)
    Z = np.repeat(z, m.n_b)
    if dirichlet:
        p = np.cos(X) * np.cos(math.pi * Y / 2) * np.cos(2 * Z)
        f = -(1 + math.pi ** 2 / 4 + 4) * p
    else:
        p = np.cos(X) * np.cos(math.pi * Y) * np.cos(2 * Z)
        f = -(1 + math.pi ** 2 + 4) * p
    b = m.cell_volumes() * f
    r = orc.cg(m, m.lap(), b, 1e-12, max_iter=20000)
    ps = p - p.mean() if not dirichlet else p
    return np.sqrt(np.mean((r.x - ps) ** 2))


@pytest.mark.parametrize("dirichlet", [False, True])
def test_manufactured_solution_second_order(orc, dirichlet):
    e = [_mms_error(orc, n, kz, dirichlet) for n, kz in ((32, 4), (64, 8), (128, 16))]
    orders = [math.log2(e[0] / e[1]), math.log2(e[1] / e[2])]
    assert all(1.8 <= o <= 2.2 for o in orders), (e, orders)


# ---------------------------------------------------------------- Section 2 model

@pytest.mark.parametrize("nnz_row", [5, 7, 13, 27])
def test_speedup_bounds_are_intensity_ratios(orc, nnz_row):
    """Eq. 3a equals I(m)/I(1) of Eq. 2, and Eq. 3b equals the same ratio with
    the input-vector term 8 n_c m replaced by 8 nnz m (zero temporal locality)."""
    n = 1e6
    nnz = nnz_row * n
    for m in (1, 2, 3, 8, 16, 64, 128):
        ub = orc.p_spmm_ub(nnz, n, n, m)
        assert ub == pytest.approx(orc.ai_spmm(nnz, n, n, m) / orc.ai_spmm(nnz, n, n, 1), rel=1e-12)

        def ai_lb(mm):
            return (2 * nnz + 1) * mm / (12 * nnz + 4 * (n + 1) + mm * (8 * n + 8 * nnz + 8))
        lb = orc.p_spmm_lb(nnz, n, m)
        assert lb == pytest.approx(ai_lb(m) / ai_lb(1), rel=1e-12)
        assert 1.0 <= lb <= ub <= m + 1e-12
    assert orc.p_spmm_ub(nnz, n, n, 1) == pytest.approx(1.0)
    # Eq. 7: all time in SpMM (chi = 1) gives the SpMM speed-up; none gives 1.
    assert orc.p_poisson(3.0, 1.0) == pytest.approx(3.0)
    assert orc.p_poisson(3.0, 0.0) == pytest.approx(1.0)


def test_speedup_bounds_match_fig2_values(orc):
    """Eqs. 3a/3b at the Fig. 2 setting (n = 10^6, 7 and 13 nonzeros per row)
    against the values in tests/golden/spmm_bounds_fig2.txt."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "spmm_bounds_fig2.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    assert len(rows) == 8
    n = 1e6
    for r, m, ub, lb in rows:
        nnz = int(r) * n
        assert orc.p_spmm_ub(nnz, n, n, int(m)) == pytest.approx(float(ub), abs=6e-4)
        assert orc.p_spmm_lb(nnz, n, int(m)) == pytest.approx(float(lb), abs=6e-4)


def _alg1_bytes(A, m, fresh_gathers):
    """Bytes Algorithm 1 moves for an actual CSR matrix A (FP64 values, int32
    indices and row pointers) and m right-hand sides, counted from the arrays
    it touches: the matrix once, the output y and the column scale c once,
    and the input x either once per distinct element (perfect reuse) or once
    per gathered entry (every gather a fresh load)."""
    val = A.data.astype(np.float64)
    idx = A.indices.astype(np.int32)
    ptr = A.indptr.astype(np.int32)
    n_r, n_c = A.shape
    x_elems = (A.nnz if fresh_gathers else n_c) * m
    return val.nbytes + idx.nbytes + ptr.nbytes + 8 * x_elems + 8 * n_r * m + 8 * m


@pytest.mark.parametrize("shape,per_row", [((400, 400), 7), ((300, 500), 13), ((600, 200), 5)])
def test_speedup_bounds_match_counted_bytes(orc, shape, per_row):
    """Eqs. 3a/3b against a byte count of Algorithm 1 on real random CSR
    matrices: with the flops of m right-hand sides m times those of one, the
    upper bound is m B(1) / B(m) with the input read once, and the lower
    bound the same ratio with every gather a fresh load; Eq. 2's denominator
    is B(m) with the input read once."""
    import scipy.sparse as sp
    rng = np.random.default_rng(per_row)
    n_r, n_c = shape
    cols = np.stack([rng.choice(n_c, per_row, replace=False) for _ in range(n_r)])
    A = sp.csr_matrix((rng.standard_normal(n_r * per_row), cols.ravel(), np.arange(0, n_r * per_row + 1, per_row)),
                      shape=shape)
    for m in (1, 2, 5, 16, 128):
        ub = m * _alg1_bytes(A, 1, False) / _alg1_bytes(A, m, False)
        lb = m * _alg1_bytes(A, 1, True) / _alg1_bytes(A, m, True)
        assert orc.p_spmm_lb(A.nnz, n_r, m) == pytest.approx(lb, rel=1e-13)  # n_c drops out of Eq. 3b
        assert orc.p_spmm_ub(A.nnz, n_r, n_c, m) == pytest.approx(ub, rel=1e-13)
        flops = orc.ai_spmm(A.nnz, n_r, n_c, m) * _alg1_bytes(A, m, False)
        assert flops == pytest.approx((2 * A.nnz + 1) * m, rel=1e-13)
