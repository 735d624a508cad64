"""Pins of the oracle's aggregation multigrid (oracle/amg.py) against facts
that do not come from it: aggregates worked out by hand on small chains, the
structure a Galerkin product of piecewise-constant aggregates must keep (zero
row sums, symmetry, identical plane blocks coupled only to neighbouring
planes), the two-level error propagation written as the product of its three
stages, symmetry and definiteness of the cycle, exactness with one level,
and dense solves."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import inputs
import oracle
from oracle import amg
from oracle import pcg as opcg


def _chain(c):
    """Symmetric coupling matrix of a chain with couplings c[i] between i, i+1."""
    n = len(c) + 1
    r = np.arange(n - 1)
    return sp.csr_matrix((np.r_[c, c], (np.r_[r, r + 1], np.r_[r + 1, r])), shape=(n, n))


@pytest.mark.parametrize("c,expect", [
    ([1, 3, 1, 1, 2], [0, 0, 1, 1, 2, 2]),           # pairs in order
    ([1, 10, 1, 1], [0, 0, 0, 1, 1]),                # cell 2: its only free neighbour is weak (1 < 0.25 * 10),
                                                     # so it stays alone, then joins its strongest neighbour's pair
    ([1, 1, 1], [0, 0, 1, 1]),                       # ties go to the smallest index
    ([5, 1, 5, 1, 5], [0, 0, 1, 1, 2, 2]),
    ([1, 4, 4, 1], [0, 0, 1, 1, 1]),                 # cell 2 pairs with 3 (tie 4 = 4, 1 is taken); 4 alone, joins 3
    ([4, 1, 1, 4, 1, 1], [0, 0, 1, 1, 2, 2, 2]),     # 2 pairs with 3 (1 = 1, 1 is taken); 4 pairs with 5 (its
                                                     # threshold 0.25 * 4 admits 1); 6 alone, joins 5's pair
])
def test_pairwise_by_hand(c, expect):
    agg, nc = amg.pairwise(_chain(np.array(c, float)), 0.25)
    assert agg.tolist() == expect and nc == max(expect) + 1


def _sym(edges, n):
    r, c, v = zip(*edges)
    return sp.csr_matrix((np.r_[v, v], (np.r_[r, c], np.r_[c, r])), shape=(n, n))


def test_pairwise_prefers_the_strongest_free_neighbour():
    # star: 0 linked to 1 (1.0), 2 (3.0), 3 (2.0): 0 pairs with 2; 1 and 3 (their only neighbour taken) join it
    agg, nc = amg.pairwise(_sym([(0, 1, 1.0), (0, 2, 3.0), (0, 3, 2.0)], 4), 0.25)
    assert agg.tolist() == [0, 0, 0, 0] and nc == 1
    # a chain 4 - 0 - 1 - 2 - 3 with 0-1 strongest: 0 pairs with 1, 2 with 3; 4 joins 0's pair
    agg, nc = amg.pairwise(_sym([(0, 1, 5.0), (1, 2, 1.0), (2, 3, 2.0), (0, 4, 1.0)], 5), 0.25)
    assert agg.tolist() == [0, 0, 1, 1, 0] and nc == 2


def test_pairwise_breaks_ties_towards_the_smallest_index():
    # equal couplings 0-1, 0-2 and 1-3: 0 pairs with 1 (smallest), 2 joins them, 3 joins 1's aggregate
    agg, nc = amg.pairwise(_sym([(0, 1, 1.0), (0, 2, 1.0), (1, 3, 1.0)], 4), 0.25)
    assert agg.tolist() == [0, 0, 0, 0]
    # 0 - 1 - 2 and 2 - 3 equal, 3 - 4 stronger: 0 pairs with 1; 2 pairs with 3 (tie of 1 and 3: 1 is taken);
    # 4 alone joins 3's pair
    agg, nc = amg.pairwise(_sym([(0, 1, 1.0), (1, 2, 1.0), (2, 3, 1.0), (3, 4, 3.0)], 5), 0.25)
    assert agg.tolist() == [0, 0, 1, 1, 1] and nc == 2
    # equal within the relative tie tolerance counts as a tie: with 0-2 stronger by 1e-12, 0 still pairs with 1
    # (2 then pairs with 4, 3 joins 1's pair); stronger by 1e-6, 0 pairs with 2 (1 with 3, 4 joins 2's pair)
    e = lambda d: _sym([(0, 1, 1.0), (0, 2, 1.0 + d), (1, 3, 1.0), (2, 4, 1.0)], 5)
    assert amg.pairwise(e(1e-12), 0.25)[0].tolist() == [0, 0, 1, 0, 1]
    assert amg.pairwise(e(1e-6), 0.25)[0].tolist() == [0, 1, 0, 1, 0]


def test_lonely_cells_do_not_stall_coarsening():
    """A graph where index order strands many cells (each cell 2m links
    strongly to 2m - 1, taken first by 2m - 2): without the second phase
    every other cell would stay alone on every level."""
    n = 40
    e = [(i, i + 1, 1.0 if i % 2 == 0 else 3.0) for i in range(n - 1)]
    agg, nc = amg.aggregate(_sym(e, n), 0.25)
    assert nc <= n // 3
    assert np.bincount(agg).min() >= 2


def test_double_pairwise_on_a_uniform_grid_makes_2x2_boxes():
    nx, ny = 8, 6
    idx = np.arange(nx * ny).reshape(ny, nx)
    rows, cols = [], []
    for a, b in ((idx[:, :-1], idx[:, 1:]), (idx[:-1, :], idx[1:, :])):
        rows += [a.ravel(), b.ravel()]
        cols += [b.ravel(), a.ravel()]
    r, c = np.concatenate(rows), np.concatenate(cols)
    T = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(nx * ny, nx * ny))
    agg, nc = amg.aggregate(T, 0.25)
    assert nc == nx * ny // 4
    for a in range(nc):
        m = np.flatnonzero(agg == a)
        j, i = m // nx, m % nx
        assert len(m) == 4 and np.ptp(i) == 1 and np.ptp(j) == 1


def _case(spec, k, dz=None, dirichlet=False, coupling=oracle.PERIODIC_Z):
    m3 = oracle.Mesh3D(oracle.geometry(spec), k, dz or math.pi / k, coupling, dirichlet)
    return m3, (-m3.lap()).tocsr()


@pytest.mark.parametrize("dirichlet", [False, True])
def test_galerkin_levels_keep_the_extruded_form(dirichlet):
    m3, A = _case(inputs.channel_base(24, 20), 16, dz=0.02, dirichlet=dirichlet)
    h = amg.build(A, m3.n_b, m3.k, True, amg.AmgOpts(coarse_max=40))
    kinds = [lv.kind for lv in h.levels]
    assert "z" in kinds and "xy" in kinds and len(h.levels) >= 4
    for lv in h.levels:
        B = lv.A.toarray()
        n, k = lv.n_b, lv.k
        assert np.allclose(B, B.T, rtol=0, atol=1e-13 * np.abs(B).max())
        if not dirichlet:
            assert np.abs(B.sum(axis=1)).max() <= 1e-12 * np.abs(B).max()
        blk = lambda a, b: B[a * n:(a + 1) * n, b * n:(b + 1) * n]
        for l in range(k):
            assert np.array_equal(blk(l, l), blk(0, 0))
            for m in range(k):
                d = min((l - m) % k, (m - l) % k)
                if d > 1:
                    assert not blk(l, m).any()
                elif d == 1:
                    c = blk(l, m)
                    assert np.count_nonzero(c - np.diag(np.diag(c))) == 0  # planes couple cell to same cell
    for lv in h.levels[:-1]:
        P = lv.P.toarray()
        assert np.array_equal(P.sum(axis=1), np.ones(P.shape[0]))      # one aggregate per unknown
        if lv.kind == "xy":
            sizes = np.bincount(lv.agg)
            assert sizes.min() >= 1 and sizes.sum() == lv.n_b
            T, _ = amg.couplings(lv.A, lv.n_b, lv.k)
            for a in range(sizes.size):                                  # aggregates are connected
                m = np.flatnonzero(lv.agg == a)
                if len(m) > 1:
                    sub = T[m][:, m]
                    ncomp, _ = sp.csgraph.connected_components(sub, directed=False)
                    assert ncomp == 1


def test_z_coarsening_follows_the_dominant_coupling():
    spec = inputs.CartSpec(16, 16, 1.0, 0.0, 1.0, 0.0, True, True)
    _, A = _case(spec, 8, dz=0.01)           # planes 0.01 apart, cells 1/16: plane coupling dominates
    _, B = _case(spec, 8, dz=1.0)            # planes far apart: in-plane coupling dominates
    ha = amg.build(A, 256, 8, True, amg.AmgOpts(coarse_max=16))
    hb = amg.build(B, 256, 8, True, amg.AmgOpts(coarse_max=16))
    assert ha.levels[0].kind == "z" and hb.levels[0].kind == "xy"
    assert ha.levels[1].k == 4 and hb.levels[1].k == 8


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_two_level_cycle_equals_the_product_of_its_stages(degree):
    m3, A = _case(inputs.channel_base(8, 6), 4)
    h = amg.build(A, m3.n_b, m3.k, True, amg.AmgOpts(degree=degree, coarse_max=60))
    assert len(h.levels) == 2
    n = A.shape[0]
    Minv = np.column_stack([amg.vcycle(h, e) for e in np.eye(n)])
    E = np.eye(n) - Minv @ A.toarray()
    Eref = amg.two_level_error(h)
    # on the complement of the constants (the cycle's range there is what CG uses)
    Q = np.eye(n) - np.ones((n, n)) / n
    assert np.abs(Q @ (E - Eref) @ Q).max() <= 1e-10
    ev = np.linalg.eigvals(Q @ Eref @ Q)
    assert ev.real.min() >= -1e-10 and ev.real.max() < 1.0


@pytest.mark.parametrize("dirichlet", [False, True])
def test_cycle_is_symmetric_and_positive_definite(dirichlet):
    m3, A = _case(inputs.channel_base(10, 8), 6, dirichlet=dirichlet)
    h = amg.build(A, m3.n_b, m3.k, True, amg.AmgOpts(coarse_max=20))
    assert len(h.levels) >= 3
    n = A.shape[0]
    M = np.column_stack([amg.vcycle(h, e) for e in np.eye(n)])
    assert np.abs(M - M.T).max() <= 1e-10 * np.abs(M).max()
    if not dirichlet:
        Q = np.eye(n) - np.ones((n, n)) / n
        M = Q @ M @ Q
        ev = np.linalg.eigvalsh((M + M.T) / 2)
        assert np.sum(ev > 1e-12 * ev.max()) == n - 1 and ev.min() > -1e-10 * ev.max()
    else:
        assert np.linalg.eigvalsh((M + M.T) / 2).min() > 0


def test_one_level_is_the_pseudo_inverse():
    m3, A = _case(inputs.channel_base(6, 5), 3)
    h = amg.build(A, m3.n_b, m3.k, True, amg.AmgOpts(coarse_max=1000))
    assert len(h.levels) == 1
    r = oracle.project_mean(inputs.rhs_uniform(90, m3.N), 1)
    x = amg.vcycle(h, r)
    assert np.linalg.norm(A @ x - r) <= 1e-12 * np.linalg.norm(r)
    assert abs(x.mean()) <= 1e-14 * np.abs(x).max()
    got = opcg.pcg(m3, -A, -r, 1e-12, precond="amg", amg_opts=amg.AmgOpts(coarse_max=1000))
    assert got.iters == [1]


def test_smoother_from_a_guess_is_the_smoother_of_the_residual():
    m3, A = _case(inputs.channel_base(9, 7), 4)
    dinv = 1.0 / A.diagonal()
    r = inputs.rhs_uniform(91, m3.N)
    z0 = inputs.uniform(92, 0, m3.N)
    for degree in (1, 2, 4):
        a = amg.chebyshev_smooth(A, dinv, r, degree, 8.0, z0=z0)
        b = z0 + opcg.chebyshev_apply(A, dinv, r - A @ z0, degree, 8.0)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
        assert np.array_equal(amg.chebyshev_smooth(A, dinv, r, degree, 8.0),
                              amg.chebyshev_smooth(A, dinv, r, degree, 8.0, z0=None))


@pytest.mark.parametrize("spec,k,coupling,dirichlet", [
    (inputs.channel_base(16, 12), 8, oracle.PERIODIC_Z, False),
    (inputs.channel_base(16, 12), 6, oracle.PERIODIC_Z, True),
    (inputs.channel_base(12, 10), 4, oracle.NONE, False),
    (inputs.unit_square_triangles(7), 4, oracle.PERIODIC_Z, False),
])
def test_amg_pcg_matches_dense_solve(spec, k, coupling, dirichlet):
    m3 = oracle.Mesh3D(oracle.geometry(spec), k, math.pi / k, coupling, dirichlet)
    L = m3.lap().tocsr()
    b = inputs.rhs_uniform(93, m3.N)
    got = opcg.pcg(m3, L, b, 1e-12, precond="amg", amg_opts=amg.AmgOpts(coarse_max=30))
    ng = m3.n_groups()
    xd = oracle.dense_solve(L.toarray(), oracle.project_mean(b, ng) if m3.singular else b, ng)
    assert np.max(np.abs(got.x - xd)) <= 1e-9 * np.max(np.abs(xd))
    plain = opcg.pcg(m3, L, b, 1e-12, precond="none")
    assert max(got.iters) < max(plain.iters)


@pytest.mark.parametrize("k", [1, 2, 3, 8])
def test_level_couplings_are_the_geometric_coefficients(k):
    """t_ij = dz len_f / dist_f and w_i = area_i / dz, read from the assembled
    operator (for two planes the two plane faces of a cell meet the same
    neighbour)."""
    spec = inputs.channel_base(6, 5)
    g = oracle.geometry(spec)
    dz = 0.3
    m3 = oracle.Mesh3D(g, k, dz, oracle.PERIODIC_Z)
    T, w = amg.couplings((-m3.lap()).tocsr(), m3.n_b, k)
    ref = np.zeros((m3.n_b, m3.n_b))
    for f in range(g.n_faces):
        a, b = g.c1[f], g.c2[f]
        if a != b:
            ref[a, b] += dz * g.len[f] / g.dist[f]
            ref[b, a] += dz * g.len[f] / g.dist[f]
    assert np.allclose(T.toarray(), ref, rtol=1e-14, atol=0)
    assert np.allclose(w, g.area / dz if k >= 2 else 0.0, rtol=1e-14, atol=0)


def test_prolongation_maps_each_plane_to_the_same_plane():
    """Base aggregation acts within every plane: unknown (l, c) feeds coarse
    unknown (l, agg[c]); plane merging sends plane l to plane l // 2."""
    m3, A = _case(inputs.channel_base(12, 10), 4, dz=0.05)
    h = amg.build(A, m3.n_b, m3.k, True, amg.AmgOpts(coarse_max=40, z_rule=1e9))
    lv = h.levels[0]
    assert lv.kind == "xy"
    nc = h.levels[1].n_b
    P = lv.P.tocoo()
    l, c = P.row // m3.n_b, P.row % m3.n_b
    assert np.array_equal(P.col, l * nc + lv.agg[c])
    h = amg.build(A, m3.n_b, m3.k, True, amg.AmgOpts(coarse_max=40, z_rule=-1.0))
    lv = h.levels[0]
    assert lv.kind == "z"
    P = lv.P.tocoo()
    l, c = P.row // m3.n_b, P.row % m3.n_b
    assert np.array_equal(P.col, (l // 2) * m3.n_b + c)


def test_unstructured_mesh_coarsens_steadily():
    """On a Delaunay mesh around an airfoil (cells of very different sizes)
    every base-plane level at least halves the cells, down to the coarsest."""
    spec = inputs.naca_delaunay(seed=3, n_interior=1500, n_surface=60, n_box_side=16)
    m3 = oracle.Mesh3D(oracle.geometry(spec), 4, 0.2, oracle.PERIODIC_Z)
    h = amg.build((-m3.lap()).tocsr(), m3.n_b, 4, True, amg.AmgOpts(coarse_max=40))
    assert h.levels[-1].n_b * h.levels[-1].k <= 40
    for a, b in zip(h.levels, h.levels[1:]):
        if a.kind == "xy":
            assert b.n_b <= a.n_b // 2


def test_galerkin_level_of_a_uniform_periodic_box_is_the_closed_form_stencil():
    """On a uniform box periodic in x, y and z, two pairwise passes give
    aligned 2 x 2 aggregates, and the Galerkin product P^T A P of the
    piecewise-constant prolongation is again the 7-point operator on the
    half-size box, worked out by hand: across an x-face pair of aggregates
    two cell faces of coupling t_x = dz h_y / h_x each (-2 t_x), likewise
    -2 t_y in y, four cells of plane coupling w = h_x h_y / dz each between
    planes (-4 w), and the diagonal the negated sum of those (the internal
    faces of an aggregate cancel).  Checked entry by entry on the oracle's
    level-1 operator, with the aggregates mapped to their (I, J) by their
    member cells."""
    nx, ny, k, dz = 8, 6, 4, 1.0
    spec = inputs.CartSpec(nx, ny, 1.0, 0.0, 1.0, 0.0, True, True)   # h_x = 1/8, h_y = 1/6, uniform
    hx, hy = 1.0 / nx, 1.0 / ny
    tx, ty, w = dz * hy / hx, dz * hx / hy, hx * hy / dz
    assert 2 * ty > tx > ty >= 0.25 * tx   # x pairs first, then the pairs pair along y: 2 x 2 boxes
    m3 = oracle.Mesh3D(oracle.geometry(spec), k, dz, oracle.PERIODIC_Z)
    A0 = (-m3.lap()).tocsr()
    h = amg.build(A0, nx * ny, k, True, amg.AmgOpts(coarse_max=16))
    lev = h.levels[0]
    assert lev.kind == "xy" and len(h.levels) >= 2
    cx, cy = nx // 2, ny // 2
    nc = cx * cy
    pos = np.empty(nc, dtype=int)   # aggregate -> coarse cell J * cx + I
    for a in range(nc):
        m = np.flatnonzero(lev.agg == a)
        j, i = m // nx, m % nx
        assert len(m) == 4 and np.ptp(i) == 1 and np.ptp(j) == 1 and i.min() % 2 == 0 and j.min() % 2 == 0
        pos[a] = (j.min() // 2) * cx + i.min() // 2
    assert sorted(pos) == list(range(nc))
    E = np.zeros((k * nc, k * nc))
    for l in range(k):
        for J in range(cy):
            for I in range(cx):
                r = l * nc + J * cx + I
                E[r, r] = 2 * (2 * tx) + 2 * (2 * ty) + 2 * (4 * w)
                E[r, l * nc + J * cx + (I + 1) % cx] -= 2 * tx
                E[r, l * nc + J * cx + (I - 1) % cx] -= 2 * tx
                E[r, l * nc + ((J + 1) % cy) * cx + I] -= 2 * ty
                E[r, l * nc + ((J - 1) % cy) * cx + I] -= 2 * ty
                E[r, ((l + 1) % k) * nc + J * cx + I] -= 4 * w
                E[r, ((l - 1) % k) * nc + J * cx + I] -= 4 * w
    perm = np.concatenate([l * nc + pos for l in range(k)])   # oracle row l*nc + a is expected row l*nc + pos[a]
    A1 = np.zeros_like(E)
    A1[np.ix_(perm, perm)] = h.levels[1].A.toarray()
    np.testing.assert_allclose(A1, E, rtol=0, atol=1e-13 * np.abs(E).max())


def test_mode_rule_stops_at_the_first_level_with_few_base_cells():
    m3, A = _case(inputs.channel_base(32, 24), 8)
    full = amg.build(A, m3.n_b, m3.k, True, amg.AmgOpts(coarse_max=40))
    for cells in (1000, 200, 50):
        h = amg.build(A, m3.n_b, m3.k, True, amg.AmgOpts(coarse_max=40, mode_cells=cells))
        first = next(i for i, lv in enumerate(full.levels) if lv.n_b <= cells)
        assert len(h.levels) == first + 1
        for a, b in zip(h.levels, full.levels):
            assert (a.n_b, a.k) == (b.n_b, b.k)
            assert (a.A != b.A).nnz == 0
    # within mode_cells but above the mode terms: coarsening goes on
    h = amg.build(A, m3.n_b, m3.k, True, amg.AmgOpts(coarse_max=40, mode_cells=2048), solve_coarsest=False)
    sizes = [(lv.n_b, lv.k) for lv in h.levels]
    last = next(i for i, lv in enumerate(full.levels) if (lv.k // 2 + 1) * lv.n_b ** 2 <= amg.MODE_TERMS)
    assert sizes == [(lv.n_b, lv.k) for lv in full.levels[:last + 1]] and h.pinv is None
    assert (m3.k // 2 + 1) * m3.n_b ** 2 <= amg.MODE_TERMS              # this case: level 0 within both
    m32, A32 = _case(inputs.channel_base(32, 24), 32)                   # 17 modes of 768^2 > 2^23 terms
    h32 = amg.build(A32, m32.n_b, 32, True, amg.AmgOpts(coarse_max=40, mode_cells=2048), solve_coarsest=False)
    assert [(lv.n_b, lv.k) for lv in h32.levels][0] == (768, 32) and len(h32.levels) >= 2
    assert (h32.levels[-1].k // 2 + 1) * h32.levels[-1].n_b ** 2 <= amg.MODE_TERMS
    assert 17 * 768 ** 2 > amg.MODE_TERMS
    # independent planes: the planes counted in pairs, n_b^2 per pair
    n_b = m3.n_b
    A0 = A[:n_b, :n_b].tocsr()
    ha = amg.build(A0, n_b, 1, False, amg.AmgOpts(coarse_max=20), columns=8)
    for cols, cells in ((8, 2000), (8, 100), (64, 2000), (1, 2000)):
        hb = amg.build(A0, n_b, 1, False, amg.AmgOpts(coarse_max=20, mode_cells=cells), columns=cols,
                       solve_coarsest=False)
        full = amg.build(A0, n_b, 1, False, amg.AmgOpts(coarse_max=20), columns=cols, solve_coarsest=False)
        first = next(i for i, lv in enumerate(full.levels)
                     if lv.n_b <= cells and (cols + 1) // 2 * lv.n_b ** 2 <= amg.MODE_TERMS)
        assert [lv.n_b for lv in hb.levels] == [lv.n_b for lv in full.levels[:first + 1]]
        assert all(lv.k == 1 for lv in hb.levels)
    assert (64 + 1) // 2 * 768 ** 2 > amg.MODE_TERMS >= 4 * 768 ** 2     # 64 planes coarsen further than 8


@pytest.mark.parametrize("k,dirichlet", [(8, False), (5, False), (6, True), (2, False)])
def test_coarsest_pinv_is_blockwise_by_plane_modes(k, dirichlet):
    """The coarsest level of coupled planes is block circulant over the
    planes, so its pseudo-inverse is the inverse discrete Fourier transform
    (numpy's FFT over the plane offset) of the pseudo-inverses of the mode
    blocks sum_d C_d exp(-2 pi i m d / k) -- the closed form the library's
    per-mode solve relies on, here pinned against the oracle's
    eigen-decomposition of the whole level."""
    m3, A = _case(inputs.channel_base(12, 10), k, dirichlet=dirichlet)
    h = amg.build(A, m3.n_b, m3.k, True, amg.AmgOpts(coarse_max=40, mode_cells=40))
    lv = h.levels[-1]
    n = lv.n_b
    assert lv.k == k and n <= 40 and len(h.levels) >= 2
    B = lv.A.toarray()
    C = np.stack([B[:n, d * n:(d + 1) * n] for d in range(k)])      # block (0, d) = C_d
    for l in range(k):                                                # block (l, l + d) = C_d
        for d in range(k):
            assert np.array_equal(B[l * n:(l + 1) * n, ((l + d) % k) * n:((l + d) % k + 1) * n], C[d])
    Mhat = np.fft.fft(C, axis=0)                                      # mode m: sum_d C_d e^{-2 pi i m d / k}
    Phat = np.stack([np.linalg.pinv(Mhat[m], rcond=1e-10) for m in range(k)])
    Pd = np.fft.ifft(Phat, axis=0)                                    # offset d block of the pseudo-inverse
    assert np.abs(Pd.imag).max() <= 1e-12 * np.abs(Pd.real).max()
    for l in range(k):
        for d in range(k):
            got = h.pinv[l * n:(l + 1) * n, ((l + d) % k) * n:((l + d) % k + 1) * n]
            assert np.allclose(got, Pd[d].real, rtol=0, atol=1e-9 * np.abs(Pd.real).max())
