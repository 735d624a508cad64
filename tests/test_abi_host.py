"""CPU-side checks of the C-ABI library: it loads, exports every entry point
declared in include/fvx.h, and its host-only logic (mesh builders, size
queries, argument validation) agrees with the oracle.  No GPU calls."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            txt = open(os.path.join(inc, f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(fvx_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def fvx():
    import paper_2508_06710_amd as fvx
    fvx.lib()
    return fvx


def test_exports_every_declared_symbol(fvx):
    from paper_2508_06710_amd import _lib
    names = _declared()
    assert len(names) >= 20
    L = fvx.lib()
    for n in names:
        assert hasattr(L, n), f"{n} missing from libfvx.so"
        assert n in _lib.SIGNATURES, f"{n} has no ctypes signature"


def test_status_strings(fvx):
    L = fvx.lib()
    assert L.fvx_status_str(0) == b"ok"
    assert L.fvx_status_str(-5) == b"CG breakdown"
    assert L.fvx_version() >= 10000


@pytest.mark.parametrize("spec", [inputs.channel_base(7, 5), inputs.convection_base(4, 6),
                                  inputs.CartSpec(3, 4, 1.0, 0.0, 2.0, 0.7, True, True)])
def test_cartesian_mesh_matches_oracle_geometry(fvx, orc, spec):
    m = fvx.Mesh.from_spec(spec)
    g = orc.cart_geometry(spec)
    area, c1, c2, ln, ds = m.faces()
    cx, cy = m.centroids()
    assert np.array_equal(c1, g.c1) and np.array_equal(c2, g.c2)
    for a, b in ((area, g.area), (ln, g.len), (ds, g.dist), (cx, g.cx), (cy, g.cy)):
        assert np.allclose(a, b, rtol=4e-16, atol=1e-300)


def test_triangle_mesh_matches_oracle_geometry(fvx, orc):
    t = inputs.unit_square_triangles(5)
    m = fvx.Mesh.from_spec(t)
    g = orc.tri_geometry(t)
    area, c1, c2, ln, ds = m.faces()
    assert np.array_equal(c1, g.c1) and np.array_equal(c2, g.c2)
    assert np.allclose(area, g.area, rtol=1e-15) and np.allclose(ln, g.len, rtol=1e-15)
    assert np.allclose(ds, g.dist, rtol=1e-13)


def test_mesh_errors(fvx):
    from paper_2508_06710_amd._lib import E_ARG, E_MESH
    L = fvx.lib()
    h = C.c_void_p()
    assert L.fvx_mesh_cartesian(0, 4, 0.0, 1.0, 0.0, 1.0, 0.0, 1, 0, C.byref(h)) == E_ARG
    assert b"nx" in L.fvx_last_error()
    xy = np.array([[0, 0], [1, 0], [0, 1.0]])
    tri = np.array([[0, 1, 5]], np.int32)
    assert L.fvx_mesh_triangles(3, xy.ctypes.data, 1, tri.ctypes.data, C.byref(h)) == E_MESH
    with pytest.raises(fvx.FvxError):
        fvx.Mesh.from_faces([1.0, -1.0], [0], [1], [1.0], [1.0])


def test_op_bytes_independent_of_k(fvx):
    """Operator storage is that of the base block only (fields grow with k, operators do not)."""
    from paper_2508_06710_amd import _lib
    m = fvx.Mesh.from_spec(inputs.channel_base(32, 16))
    sizes = []
    for k in (1, 4, 64, 128):
        d = _lib.OpDesc()
        d.k, d.coupling, d.dz, d.wall_bc, d.with_f32 = k, 1, 0.1, 0, 1
        n = C.c_size_t()
        assert fvx.lib().fvx_op_bytes(m._h, C.byref(d), C.byref(n)) == 0
        sizes.append(n.value)
    assert len(set(sizes)) == 1
    d.k = 0
    assert fvx.lib().fvx_op_bytes(m._h, C.byref(d), C.byref(n)) == _lib.E_ARG


@pytest.mark.parametrize("spec", [inputs.channel_base(9, 7), inputs.convection_base(5, 6),
                                  inputs.unit_square_triangles(4)])
@pytest.mark.parametrize("k,coupling,dirichlet", [(1, 1, False), (2, 1, False), (3, 1, False),
                                                  (8, 1, False), (3, 0, False), (4, 1, True)])
def test_kronecker_expansion_matches_oracle_assembly(fvx, orc, spec, k, coupling, dirichlet):
    """The builder's base block, expanded as I_k (x) A_b + C, equals the oracle's
    face-by-face 3D assembly: same pattern, values within 2 ulp."""
    dz = 0.37
    m = fvx.Mesh.from_spec(spec)
    ptr, col, val = fvx.expand_csr(m, k, dz, coupling, fvx.DIRICHLET if dirichlet else fvx.NEUMANN)
    L = orc.Mesh3D(orc.geometry(spec), k, dz, coupling, dirichlet).lap()
    assert np.array_equal(ptr, L.indptr) and np.array_equal(col, L.indices)
    ulp = np.spacing(np.abs(L.data))
    assert np.all(np.abs(val - L.data) <= 2 * ulp + 1e-300 * 0), float(np.max(np.abs(val - L.data) / ulp))


def test_one_hip_runtime_whatever_the_import_order():
    """torch's wheel carries its own HIP runtime; loading the library must not
    bring a second one into the process (device memory from one runtime is
    unknown to the other).  No device call is made."""
    import subprocess
    import sys
    code = ("import paper_2508_06710_amd as f; f.lib(); import torch\n"
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=root, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == "1"



@pytest.mark.parametrize("stencil", [13, 27])
@pytest.mark.parametrize("spec", [inputs.channel_base(7, 9), inputs.convection_base(6, 5),
                                  inputs.CartSpec(3, 4, 2.0, 0.0, 1.5, 0.0, True, True),
                                  inputs.CartSpec(1, 2, 1.0, 0.0, 1.0, 0.0, True, True)])
@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_structured_stencil_expansion_matches_oracle(fvx, orc, stencil, spec, k):
    """The builder's 13/27-point base blocks (in-plane entries, coefficients of
    the neighbouring planes), expanded over k planes, equal the oracle's
    assembly; short periodic axes merge neighbours like the oracle does."""
    dz = 0.61
    m = fvx.Mesh.from_spec(spec)
    ptr, col, val = fvx.expand_csr(m, k, dz, fvx.PERIODIC_Z, fvx.NEUMANN, stencil=stencil)
    import scipy.sparse as sp
    n = spec.nx * spec.ny * k
    A = sp.csr_matrix((val, col, ptr), shape=(n, n)).toarray()
    B = orc.stencil_lap(spec, k, dz, stencil).toarray()
    assert np.max(np.abs(A - B)) <= 4e-15 * np.max(np.abs(B))


def test_structured_stencil_rejections(fvx):
    tri = fvx.Mesh.from_spec(inputs.unit_square_triangles(3))
    cart = fvx.Mesh.from_spec(inputs.channel_base(4, 4))
    for mesh, kw in ((tri, {}), (cart, {"coupling": fvx.NONE}), (cart, {"wall_bc": fvx.DIRICHLET}),
                     (cart, {"k": 200})):
        args = dict(k=4, dz=0.5, coupling=fvx.PERIODIC_Z, wall_bc=fvx.NEUMANN)
        args.update(kw)
        with pytest.raises(fvx.FvxError):
            fvx.expand_csr(mesh, args["k"], args["dz"], args["coupling"], args["wall_bc"], stencil=27)
    with pytest.raises(fvx.FvxError):
        fvx.expand_csr(cart, 4, 0.5, stencil=9)


@pytest.mark.parametrize("b", [1, 2, 3, 5])
def test_hilbert_order_on_a_grid_is_the_hilbert_curve(fvx, b):
    """On the 2^b x 2^b grid of integer points (shuffled), the order visits
    every point once, each step goes to a unit neighbour, and the walk runs
    from (0, 0) to (2^b - 1, 0): the defining properties of the Hilbert
    curve in its standard orientation."""
    n = 1 << b
    gx, gy = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x, y = gx.ravel().astype(float), gy.ravel().astype(float)
    shuffle = np.random.default_rng(b).permutation(n * n)
    x, y = x[shuffle], y[shuffle]
    perm = fvx.hilbert_order(x, y)
    assert sorted(perm.tolist()) == list(range(n * n))
    px, py = x[perm], y[perm]
    steps = np.abs(np.diff(px)) + np.abs(np.diff(py))
    assert np.all(steps == 1)
    assert (px[0], py[0]) == (0, 0) and (px[-1], py[-1]) == (n - 1, 0)


def test_hilbert_order_edge_cases(fvx):
    assert len(fvx.hilbert_order(np.zeros(0), np.zeros(0))) == 0
    # equal points (and a zero-width box): index order
    assert fvx.hilbert_order(np.ones(5), np.ones(5)).tolist() == [0, 1, 2, 3, 4]
    # points on a horizontal line: sorted by x along the curve's bottom edge
    x = np.array([3.0, 0.0, 2.0, 1.0])
    assert fvx.hilbert_order(x, np.zeros(4)).tolist() == [1, 3, 2, 0]
    with pytest.raises(fvx.FvxError):
        fvx.hilbert_order(np.array([0.0, np.nan]), np.zeros(2))


def test_hilbert_order_keeps_neighbours_close(fvx):
    """Random points: consecutive points in the order are on average far
    closer than in index order (about n^-1/2 of the box against a third)."""
    rng = np.random.default_rng(3)
    x, y = rng.random(20000), rng.random(20000)
    perm = fvx.hilbert_order(x, y)
    assert sorted(perm.tolist()) == list(range(len(x)))
    step = np.hypot(np.diff(x[perm]), np.diff(y[perm])).mean()
    assert step < 0.03 < np.hypot(np.diff(x), np.diff(y)).mean()


def test_mesh_in_hilbert_order_renumbers_cells(fvx):
    """A triangle mesh built with order="hilbert": cell i is input triangle
    cell_perm[i] (centroids, areas and the face graph follow the permutation)."""
    spec = inputs.unit_square_triangles(6)
    m0 = fvx.Mesh.from_spec(spec)
    m1 = fvx.Mesh.from_spec(spec, order="hilbert")
    perm = m1.cell_perm
    assert sorted(perm.tolist()) == list(range(len(spec.triangles)))
    c0, c1 = m0.centroids(), m1.centroids()
    assert np.array_equal(c1[0], c0[0][perm]) and np.array_equal(c1[1], c0[1][perm])
    a0, f10, f20 = m0.faces()[:3]
    a1, f11, f21 = m1.faces()[:3]
    assert np.array_equal(a1, a0[perm])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    e0 = sorted(tuple(sorted(e)) for e in zip(inv[f10], inv[f20]))
    e1 = sorted(tuple(sorted(e)) for e in zip(f11, f21))
    assert e0 == e1


def test_multigrid_defaults(fvx):
    """fvx_amg_opts_default against the values the header states, and the
    oracle's defaults for the options both sides share (the oracle leaves
    the plane-mode rule off unless asked: comparisons pass it)."""
    from paper_2508_06710_amd import _lib
    from oracle import amg as oamg
    o = _lib.AmgOpts()
    assert fvx.lib().fvx_amg_opts_default(C.byref(o)) == 0
    got = (o.degree, o.ratio, o.beta, o.z_rule, o.coarse_max, o.max_levels, o.mode_cells)
    assert got == (2, 8.0, 0.75, 1.0, 2048, 16, 2048)
    d = oamg.AmgOpts()
    assert (d.degree, d.ratio, d.beta, d.z_rule, d.coarse_max, d.max_levels) == got[:6]
    assert d.mode_cells == 0
    assert fvx.lib().fvx_amg_opts_default(None) != 0
