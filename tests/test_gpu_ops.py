"""GPU parity of the SpMM operators (lap, div, grad) against the oracle's
assembled 3D matrices, element by element, through the C ABI."""
import math

import numpy as np
import pytest
import torch

import inputs
from helpers import Case, componentwise, fp32_bound_factor

pytestmark = pytest.mark.gpu

TOL64 = 1e-12

# (label, spec) -- ragged sizes that do not fill whole tiles, walls on all
# sides, unstructured triangles, and the 64x64 stretched channel base.
BASES = {
    "chan13x9": inputs.channel_base(13, 9),
    "box7x11": inputs.convection_base(7, 11),
    "tri6": inputs.unit_square_triangles(6),
    "chan64": inputs.channel_base(64, 64),
}


def _lap_check(c: Case, seed=0, dtype=None, colscale=None):
    fvx = c.fvx
    x = inputs.uniform(seed, 0, c.m3.N)
    if dtype == fvx.F32:
        x = x.astype(np.float32).astype(np.float64)
        X = c.op.to_rows(x, dtype=fvx.F32)
        y = c.op.to_planes(c.op.lap(X, colscale=colscale), dtype=fvx.F32).astype(np.float64)
    else:
        X = c.op.to_rows(x)
        y = c.op.to_planes(c.op.lap(X, colscale=colscale))
    from oracle import spmv
    ref = spmv(c.L, x)
    if colscale is not None:
        s = colscale.cpu().numpy()
        ref = ref * np.repeat(s, c.m3.n_b)
        A = c.L.multiply(np.repeat(np.abs(s), c.m3.n_b)[:, None]).tocsr()
    else:
        A = c.L
    return y, ref, A, x


@pytest.mark.parametrize("base", list(BASES))
@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 16, 64])
def test_lap_f64_periodic(base, k):
    c = Case(BASES[base], k)
    y, ref, A, x = _lap_check(c, seed=k)
    assert componentwise(y, ref, A, x) <= TOL64
    assert np.linalg.norm(y - ref) <= TOL64 * np.linalg.norm(ref)


@pytest.mark.parametrize("base", ["chan13x9", "tri6"])
@pytest.mark.parametrize("k", [1, 4, 7])
def test_lap_f64_independent_planes_colscale(base, k):
    c = Case(BASES[base], k, coupling=0)
    cs = torch.tensor(inputs.uniform(9, 0, k, 0.5, 2.0), dtype=torch.float64, device="cuda")
    for scale in (None, cs):
        y, ref, A, x = _lap_check(c, seed=1, colscale=scale)
        assert componentwise(y, ref, A, x) <= TOL64


@pytest.mark.parametrize("k", [2, 5, 16])
def test_lap_dirichlet(k):
    c = Case(BASES["box7x11"], k, dirichlet=True)
    y, ref, A, x = _lap_check(c, seed=3)
    assert componentwise(y, ref, A, x) <= TOL64


@pytest.mark.parametrize("k", [128, 130])
def test_lap_wide_k(k):
    c = Case(BASES["chan13x9"], k)
    y, ref, A, x = _lap_check(c, seed=4)
    assert componentwise(y, ref, A, x) <= TOL64


@pytest.mark.parametrize("k", [8, 16, 64])
def test_every_tile_gives_the_same_product(k):
    """Tiles are interchangeable: each valid tile reproduces the oracle, and
    single-pass and multi-pass row groups agree."""
    c = Case(BASES["chan13x9"], k)
    fvx = c.fvx
    outs = []
    for vec in (1, 2):
        for lpr in (1, 2, 4, 8, 16, 32, 64):
            for block in (64, 256, 1024):
                if block < lpr:
                    continue
                for remap in (0, 1):
                    for stage in (0, 1):
                        if stage and block // lpr > 64:
                            continue
                        cap = (0, 3, 7)[(lpr + block + stage) % 3]  # caps give several tiles per block
                        nt = (remap + stage) % 2
                        c.op.set_tile(vec, lpr, block, remap, cap, stage, nt, dtype=fvx.F64)
                        y, ref, A, x = _lap_check(c, seed=5)
                        assert componentwise(y, ref, A, x) <= TOL64, (vec, lpr, block, remap, cap, stage, nt)
                        outs.append(y)
    # same order of operations per element in every tile: bit-identical results
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    with pytest.raises(fvx.FvxError):
        c.op.set_tile(4, 8, 256, 1, dtype=fvx.F64)  # 32-byte vectors are not offered
    with pytest.raises(fvx.FvxError):
        c.op.set_tile(2, 3, 256, 1, dtype=fvx.F64)  # lanes per row must be a power of two
    with pytest.raises(fvx.FvxError):
        c.op.set_tile(2, 8, 256, 1, 0, 2, dtype=fvx.F64)  # stage_lds is 0 or 1
    with pytest.raises(fvx.FvxError):
        c.op.set_tile(2, 1, 256, 1, 0, 1, dtype=fvx.F64)  # 256 rows per tile do not fit the stage


def _cart_lines(n_b, nx, ny, rows_per_tile, cap):
    """Grid lines per row group the Cartesian kernel takes under a workgroup
    cap (1 without one, else the fewest of 2 or 4 that fits, at most ny)."""
    if cap <= 0 or -(-n_b // rows_per_tile) <= cap:
        return 1
    xt = -(-nx // rows_per_tile)
    r = 2 if xt * -(-ny // 2) <= cap else 4
    while r > ny:
        r //= 2
    return r


CART_SPECS = {
    "chan13x9": inputs.channel_base(13, 9),                                    # periodic x, walls y
    "box7x11": inputs.convection_base(7, 11),                                  # walls on all sides
    "torus11x7": inputs.CartSpec(11, 7, 1.0, 0.0, 1.0, 0.0, True, True),       # periodic x and y
    "torus5x3": inputs.CartSpec(5, 3, 1.0, 0.0, 1.0, 0.0, True, True),         # ny = 3: wraps past the last line
    "pery6x10": inputs.CartSpec(6, 10, 1.0, 0.0, 1.0, 1.2, False, True),       # walls x, periodic y
}


@pytest.mark.parametrize("spec", list(CART_SPECS))
@pytest.mark.parametrize("k,coupling", [(16, 1), (64, 1), (16, 0)])
def test_cartesian_line_tiles_give_the_same_product(spec, k, coupling):
    """Workgroup caps on a Cartesian 5-point base give each row group 2 or 4
    grid lines along y (ragged last tiles in x and y, walls and periodic
    wraps): the product is the oracle's and bitwise that of the one-line
    kernel and of the ELL kernel (LDS-staged tile)."""
    c = Case(CART_SPECS[spec], k, coupling=coupling)
    fvx = c.fvx
    sp_ = CART_SPECS[spec]
    cs = torch.tensor(inputs.uniform(11, 0, k, 0.5, 2.0), dtype=torch.float64, device="cuda")
    for scale in (None, cs):  # the column scale applies to coupled planes as well
        c.op.set_tile(2, 8, 64, 1, 0, 1, 0, dtype=fvx.F64)   # ELL kernel, rows staged in LDS
        y_ell, ref, A, x = _lap_check(c, seed=12, colscale=scale)
        assert componentwise(y_ell, ref, A, x) <= TOL64
        seen = set()
        for vec, lpr in ((2, k // 2), (1, min(64, k))):
            if lpr * vec != k:
                continue
            for block in (64, 128, 256):
                if block < lpr:
                    continue
                for cap in (0, 1, 3, 12, 24, 40):
                    for remap, nt in ((0, 1), (1, 0)):
                        c.op.set_tile(vec, lpr, block, remap, cap, 0, nt, dtype=fvx.F64)
                        y, _, _, _ = _lap_check(c, seed=12, colscale=scale)
                        key = (vec, lpr, block, cap, remap, nt)
                        assert np.array_equal(y, y_ell), key
                        seen.add(_cart_lines(sp_.nx * sp_.ny, sp_.nx, sp_.ny, block // lpr, cap))
        assert seen == ({1, 2} if sp_.ny < 4 else {1, 2, 4}), seen


@pytest.mark.parametrize("spec", ["chan13x9", "torus5x3", "pery6x10"])
@pytest.mark.parametrize("k", [16, 64])
def test_cartesian_line_tiles_fp32(spec, k):
    """The FP32 product (the mixed solve's inner SpMM) on the same line
    tiles: within the FP32 rounding bound of the oracle and bitwise that of
    the FP32 ELL kernel."""
    c = Case(CART_SPECS[spec], k)
    fvx = c.fvx
    c.op.set_tile(2, 8, 64, 1, 0, 1, 0, dtype=fvx.F32)   # ELL kernel, rows staged in LDS
    y_ell, ref, A, x = _lap_check(c, seed=13, dtype=fvx.F32)
    assert componentwise(y_ell, ref, A, x) <= float(np.max(fp32_bound_factor(A)))
    for vec in (4, 2):
        lpr = k // vec
        if lpr < 8 or lpr > 64:
            continue
        for block in (64, 256):
            for cap in (0, 1, 12, 40):
                c.op.set_tile(vec, lpr, block, cap % 2, cap, 0, 1, dtype=fvx.F32)
                y, _, _, _ = _lap_check(c, seed=13, dtype=fvx.F32)
                assert np.array_equal(y, y_ell), (vec, lpr, block, cap)


@pytest.mark.parametrize("k,dtype", [(16, 0), (5, 1), (64, 1)])
def test_tuner_keeps_the_fastest_candidate(k, dtype):
    """The autotuner's two stages: every row mapping with default options,
    then the options around the stage-1 winner; the op keeps the fastest
    candidate, and the tuned product is the oracle's (tiles only change speed)."""
    c = Case(inputs.channel_base(40, 24), k)
    fvx = c.fvx
    res = c.op.tune(dtype, scratch_bytes=32 << 20, reps=1)
    tiles = [t for t, _ in res]
    assert len(set(tiles)) == len(tiles)
    stage1 = [t for t in tiles if t[3:] == (1, 0, 0, 0)]
    first = min(((us, t) for t, us in res if t in stage1))[1]
    for t in tiles[len(stage1):]:  # options around the stage-1 row mapping; on a Cartesian base also
        assert t[:2] == first[:2]    # the line caps at the other workgroup sizes
        assert t[2] == first[2] or (t[4] in (1024, 2048) and t[5] == 0), t
    assert c.op.get_tile(dtype) == min(res, key=lambda r: r[1])[0]
    y, ref, A, x = _lap_check(c, seed=7, dtype=dtype)
    tol = TOL64 if dtype == fvx.F64 else float(np.max(fp32_bound_factor(A)))
    assert componentwise(y, ref, A, x) <= tol


@pytest.mark.parametrize("base", list(BASES))
@pytest.mark.parametrize("k", [1, 3, 8, 64])
def test_lap_f32_within_rounding_bound(base, k):
    c = Case(BASES[base], k)
    y, ref, A, x = _lap_check(c, seed=6, dtype=c.fvx.F32)
    bound = abs(A) @ np.abs(x)
    err = np.abs(y - ref)
    fac = fp32_bound_factor(A)
    assert np.all(err <= fac * bound + 1e-30), float(np.max(err / (fac * bound + 1e-300)))


def _faces_vec(c, seed):
    """Random face velocities, plane-major over the oracle's 3D face numbering."""
    return inputs.normal(seed, 0, c.m3.F3)


def _split_faces(c, u):
    kF = c.k * c.m3.g.n_faces
    return u[:kF], u[kF:]


@pytest.mark.parametrize("base", list(BASES))
@pytest.mark.parametrize("k,coupling", [(1, 1), (2, 1), (3, 1), (8, 1), (64, 1), (4, 0)])
def test_div_and_grad(base, k, coupling):
    c = Case(BASES[base], k, coupling=coupling)
    fvx = c.fvx
    from oracle import spmv
    u = _faces_vec(c, 11)
    uf, wz = _split_faces(c, u)
    Uf = c.op.to_rows(uf, rows=c.op.F_b)
    Wz = c.op.to_rows(wz) if c.op.zfaces else None
    D = c.op.to_planes(c.op.div(Uf, Wz))
    assert componentwise(D, spmv(c.M, u), c.M, u) <= TOL64

    p = inputs.uniform(12, 0, c.m3.N)
    Gf, Gz = c.op.grad(c.op.to_rows(p))
    g = c.op.to_planes(Gf, rows=c.op.F_b)
    if c.op.zfaces:
        g = np.concatenate([g, c.op.to_planes(Gz)])
    assert componentwise(g, spmv(c.G, p), c.G, p) <= TOL64

    # FP32 versions within a rounding bound.
    U32 = c.op.to_rows(uf.astype(np.float32), rows=c.op.F_b, dtype=fvx.F32)
    W32 = c.op.to_rows(wz.astype(np.float32), dtype=fvx.F32) if c.op.zfaces else None
    D32 = c.op.to_planes(c.op.div(U32, W32), dtype=fvx.F32).astype(np.float64)
    u32 = np.concatenate([uf.astype(np.float32), wz.astype(np.float32)]).astype(np.float64)
    ref32 = spmv(c.M, u32)
    assert np.all(np.abs(D32 - ref32) <= 16 * 2.0 ** -24 * (abs(c.M) @ np.abs(u32)) + 1e-30)


@pytest.mark.parametrize("k,vec,lpr", [(64, 2, 4), (7, 1, 2), (130, 2, 16), (9, 2, 1)])
def test_multi_pass_row_groups(k, vec, lpr):
    """Row groups that cover the k columns in several passes take the plane
    neighbours at the pass edges from memory: lap, div and grad against the
    oracle with such tiles."""
    c = Case(BASES["chan13x9"], k)
    fvx = c.fvx
    from oracle import spmv
    c.op.set_tile(vec, lpr, 64, 1, dtype=fvx.F64)
    y, ref, A, x = _lap_check(c, seed=21)
    assert componentwise(y, ref, A, x) <= TOL64
    u = _faces_vec(c, 22)
    uf, wz = _split_faces(c, u)
    D = c.op.to_planes(c.op.div(c.op.to_rows(uf, rows=c.op.F_b), c.op.to_rows(wz)))
    assert componentwise(D, spmv(c.M, u), c.M, u) <= TOL64
    p = inputs.uniform(23, 0, c.m3.N)
    Gf, Gz = c.op.grad(c.op.to_rows(p))
    g = np.concatenate([c.op.to_planes(Gf, rows=c.op.F_b), c.op.to_planes(Gz)])
    assert componentwise(g, spmv(c.G, p), c.G, p) <= TOL64


def test_lap_equals_div_of_grad():
    """L = M G through the GPU operators themselves."""
    c = Case(BASES["chan13x9"], 6)
    p = c.op.to_rows(inputs.uniform(13, 0, c.m3.N))
    Gf, Gz = c.op.grad(p)
    D = c.op.to_planes(c.op.div(Gf, Gz))
    Lp = c.op.to_planes(c.op.lap(p))
    assert np.max(np.abs(D - Lp)) <= 1e-12 * np.max(np.abs(Lp))


def test_small_channel_full_size():
    """The 64x64 base with 8 periodic planes (32,768 cells), all elements."""
    c = Case(inputs.channel_base(64, 64), 8, math.pi / 8)
    y, ref, A, x = _lap_check(c, seed=0)
    assert componentwise(y, ref, A, x) <= TOL64
    assert np.linalg.norm(y - ref) <= TOL64 * np.linalg.norm(ref)


def test_bad_arguments_are_rejected():
    c = Case(BASES["chan13x9"], 4)
    fvx = c.fvx
    X = c.op.empty()
    with pytest.raises(fvx.FvxError):
        c.op.lap(X, X)                      # in place
    with pytest.raises(fvx.FvxError):
        c.op.lap(X[:, 1:], dtype=fvx.F64)  # misaligned
    c2 = Case(BASES["chan13x9"], 4, with_f32=False)
    with pytest.raises(fvx.FvxError):
        c2.op.lap(c2.op.empty(dtype=fvx.F32), dtype=fvx.F32)


@pytest.mark.parametrize("k", [1, 8, 32])
def test_operators_on_a_mesh_in_hilbert_order(k):
    """A Delaunay airfoil mesh with its cells renumbered along a Hilbert curve
    (the layout the airfoil benchmark uses): lap in both precisions, div and
    the solve against the oracle assembled on the same numbering."""
    spec = inputs.naca_delaunay(seed=3, n_interior=1500, n_surface=60, n_box_side=16)
    c = Case(spec, k, order="hilbert")
    fvx = c.fvx
    assert c.op.mesh.cell_perm is not None
    y, ref, A, x = _lap_check(c, seed=k)
    assert componentwise(y, ref, A, x) <= TOL64
    y32, ref32, A32, x32 = _lap_check(c, seed=k, dtype=fvx.F32)
    assert np.all(np.abs(y32 - ref32) <= fp32_bound_factor(A32) * (abs(A32) @ np.abs(x32)) + 1e-30)
    from oracle import spmv, project_mean
    b = inputs.rhs_uniform(11, c.m3.N)
    X, st = c.op.solve(c.op.to_rows(b), rtol=1e-10)
    bp = project_mean(b, c.m3.n_groups())
    r = bp - spmv(c.L, c.op.to_planes(X))
    assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(bp)


def test_tile_cache_file(tmp_path):
    """fvx_tune_cached / fvx_tune_cg_cached: tune and store on a miss, set
    without timing on a hit; a file written by Python (other entries, other
    members) is read, kept and rewritten in the same layout as Python's
    json.dump(indent=1, sort_keys=True); a malformed file is an error."""
    import json
    c = Case(inputs.channel_base(13, 9), 8)
    fvx = c.fvx
    path = str(tmp_path / "tiles.json")
    other = {"gfx950|f64|k=1|ld=1|n_b=1|nnz_b=1|stencil=7": {"tile": [1, 1, 64, 1, 0, 0, 0], "us": 3.3057108521461487,
                                                             "candidates": 15, "source": "refined"}}
    with open(path, "w") as fh:
        json.dump(other, fh, indent=1, sort_keys=True)
    t1, src1 = c.op.tune_cached(fvx.F64, path, scratch_bytes=64 << 20)
    assert src1 == "tuned" and t1 == c.op.get_tile(fvx.F64)
    doc = json.load(open(path))
    key = [k for k in doc if k.endswith(f"|f64|k=8|ld={c.op.ld}|n_b={c.op.n_b}|nnz_b={c.op.nnz_b}|stencil=7")]
    assert len(key) == 1 and tuple(doc[key[0]]["tile"]) == t1 and doc[key[0]]["candidates"] >= 1
    assert doc[key[0]]["us"] > 0 and key[0].split("|")[0].startswith("gfx")
    for k, v in other.items():
        assert doc[k] == v  # kept, numbers included
    text = open(path).read()
    assert text == json.dumps(doc, indent=1, sort_keys=True)
    c.op.set_tile(1, 8, 64, 0, 0, 0, 0)
    t2, src2 = c.op.tune_cached(fvx.F64, path)
    assert src2 == "cache" and t2 == t1 and c.op.get_tile(fvx.F64) == t1
    assert open(path).read() == text  # a hit does not rewrite the file
    tc, srcc = c.op.tune_cg_cached(fvx.F64, path, iters=8)
    assert srcc == "tuned" and tc == c.op.get_cg_tile(fvx.F64)
    doc2 = json.load(open(path))
    ck = [k for k in doc2 if k.startswith("cg|") and k.endswith(f"|n_b={c.op.n_b}|nnz_b={c.op.nnz_b}|coupling=1")]
    assert len(ck) == 1 and doc2[ck[0]]["us_per_iter"] > 0
    assert c.op.tune_cg_cached(fvx.F64, path, iters=8) == (tc, "cache")
    bad = str(tmp_path / "bad.json")
    open(bad, "w").write('{"a": [1, 2,')
    with pytest.raises(fvx.FvxError):
        c.op.tune_cached(fvx.F64, bad)
