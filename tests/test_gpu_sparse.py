"""The general sparse-matrix SpMM (fvx_sparse_*) against the oracle's CSR
product, column by column: random rectangular matrices with empty and long
rows and repeated columns, every lane-group width and vector width, column
scaling, padded strides, and the coarse-to-fine state mapping of the inline
mesh refinement applied to all k states."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import inputs
import oracle
from helpers import componentwise
from oracle import refine as orf

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _random_csr(seed, n_rows, n_cols, max_len):
    lens = (inputs.u64(seed, 0, n_rows) % np.uint64(max_len + 1)).astype(np.int64)
    lens[:3] = [0, max_len, 1]  # an empty row, a long row, a single entry
    ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    nnz = int(ptr[-1])
    col = (inputs.u64(seed, 1, nnz) % np.uint64(n_cols)).astype(np.int32)
    val = inputs.uniform(seed, 2, nnz)
    return ptr, col, val


def _ref(A, X):
    """Column-by-column oracle product of a host [n_cols][k] array."""
    return np.stack([oracle.spmv(A, np.ascontiguousarray(X[:, c])) for c in range(X.shape[1])], axis=1)


def _check64(A, X, Y):
    for c in range(X.shape[1]):
        assert componentwise(Y[:, c], oracle.spmv(A, np.ascontiguousarray(X[:, c])), A, X[:, c]) <= 1e-12, c


@pytest.mark.parametrize("k", [1, 2, 3, 8, 17, 64, 130])
def test_rectangular_random_f64(k):
    import paper_2508_06710_amd as fvx
    ptr, col, val = _random_csr(70, 1001, 677, 20)
    A = sp.csr_matrix((val, col, ptr), shape=(1001, 677))
    M = fvx.SparseMatrix(ptr, col, val, 677)
    ld = k + (-k) % 4
    Xh = np.zeros((677, ld))
    Xh[:, :k] = inputs.uniform(71, k, 677 * k).reshape(677, k)
    Y = M.spmm(torch.as_tensor(Xh).cuda(), k=k).cpu().numpy()
    _check64(A, Xh[:, :k], Y[:, :k])
    assert np.all(Y[:, k:] == 0)  # columns past k are not written


@pytest.mark.parametrize("k", [4, 16, 64])
def test_rectangular_random_f32_within_rounding_bound(k):
    import paper_2508_06710_amd as fvx
    ptr, col, val = _random_csr(72, 800, 1200, 12)
    A = sp.csr_matrix((val.astype(np.float32).astype(np.float64), col, ptr), shape=(800, 1200))
    M = fvx.SparseMatrix(ptr, col, val, 1200)
    Xh = inputs.uniform(73, k, 1200 * k).reshape(1200, k).astype(np.float32)
    Y = M.spmm(torch.as_tensor(Xh).cuda()).cpu().numpy().astype(np.float64)
    X64 = Xh.astype(np.float64)
    n = np.diff(ptr)
    for c in range(k):
        ref = oracle.spmv(A, np.ascontiguousarray(X64[:, c]))
        bound = abs(A) @ np.abs(X64[:, c])
        assert np.all(np.abs(Y[:, c] - ref) <= (n + 1) * U32 * bound + 1e-30)


@pytest.mark.parametrize("k", [1, 3, 24])
def test_tiles_with_the_same_split_give_the_same_product(k):
    """Tiles that differ in vector width, lanes per column pass, workgroup,
    remap, grid cap or store kind give bitwise the same product when they
    split the rows' nonzeros the same way; every split matches the oracle."""
    import paper_2508_06710_amd as fvx
    ptr, col, val = _random_csr(74, 513, 300, 9)
    A = sp.csr_matrix((val, col, ptr), shape=(513, 300))
    M = fvx.SparseMatrix(ptr, col, val, 300)
    ld = k if k < 4 else k + (-k) % 4
    for dtype, tdt, vecs in ((fvx.F64, torch.float64, (1, 2)), (fvx.F32, torch.float32, (1, 2, 4))):
        Xh = np.zeros((300, ld))
        Xh[:, :k] = inputs.uniform(75, k, 300 * k).reshape(300, k)
        X = torch.as_tensor(Xh).to(tdt).cuda()
        refs = {}
        n = 0
        for vec in vecs:
            if ld % vec:
                continue
            c = 1
            while c < -(-k // vec):
                c *= 2
            for lpr in (1, 2, 4, 8, 16, 32, 64):
                split = max(1, lpr // c)
                for block in (64, 256, 1024):
                    for remap in (0, 1):
                        for cap in (0, 5):
                            for nt in (0, 1):
                                if block < lpr:
                                    continue
                                M.set_tile(vec, lpr, block, remap, cap, nt, dtype=dtype)
                                Y = M.spmm(X, k=k).cpu().numpy()
                                ref = refs.setdefault(split, Y)
                                assert np.array_equal(Y, ref), (dtype, vec, lpr, block, remap, cap, nt)
                                n += 1
        M.set_tile(0, dtype=dtype)  # back to the default (no split)
        assert np.array_equal(M.spmm(X, k=k).cpu().numpy(), refs[1])
        if dtype == fvx.F64:
            for Y in refs.values():
                _check64(A, Xh[:, :k], Y[:, :k])
        assert n > 50 and len(refs) >= 2


def test_column_scaling():
    import paper_2508_06710_amd as fvx
    ptr, col, val = _random_csr(76, 400, 400, 7)
    A = sp.csr_matrix((val, col, ptr), shape=(400, 400))
    M = fvx.SparseMatrix(ptr, col, val, 400)
    k = 6
    Xh = inputs.uniform(77, 0, 400 * k).reshape(400, k)
    cs = np.array([1.0, -2.0, 0.5, 0.0, 3.25, 1e-3])
    Y = M.spmm(torch.as_tensor(Xh).cuda(), colscale=torch.as_tensor(cs).cuda()).cpu().numpy()
    for c in range(k):
        ref = cs[c] * oracle.spmv(A, np.ascontiguousarray(Xh[:, c]))
        bound = abs(cs[c]) * (abs(A) @ np.abs(Xh[:, c]))
        assert np.all(np.abs(Y[:, c] - ref) <= 2e-16 * 8 * bound + 1e-300)


@pytest.mark.parametrize("spec,rf,k", [(inputs.channel_base(24, 16), 2, 8), (inputs.convection_base(9, 7), 3, 5),
                                       (inputs.channel_base(96, 64), 2, 64)])
def test_prolongation_of_all_states(spec, rf, k):
    """The coarse-to-fine mapping built by the library, applied to k flow
    states at once, equals the oracle's mapping applied state by state."""
    import paper_2508_06710_amd as fvx
    m = fvx.Mesh.from_spec(spec)
    ptr, col, val = m.prolongation(rf)
    P = fvx.SparseMatrix(ptr, col, val, m.n_cells)
    Pref = orf.prolongation(spec, rf)
    ld = k + (-k) % 4
    Xh = np.zeros((m.n_cells, ld))
    Xh[:, :k] = inputs.uniform(78, k, m.n_cells * k).reshape(m.n_cells, k)
    Y = P.spmm(torch.as_tensor(Xh).cuda(), k=k).cpu().numpy()
    _check64(Pref, Xh[:, :k], Y[:, :k])


def test_bad_arguments_are_rejected():
    import paper_2508_06710_amd as fvx
    ptr, col, val = _random_csr(79, 50, 40, 5)
    with pytest.raises(fvx.FvxError):
        fvx.SparseMatrix(ptr, np.where(col == col.max(), 40, col), val, 40)  # column out of range
    bad = ptr.copy()
    bad[5], bad[6] = bad[6], bad[5] - 1
    with pytest.raises(fvx.FvxError):
        fvx.SparseMatrix(bad, col, val, 40)  # decreasing row pointers
    v2 = val.copy()
    v2[0] = np.nan
    with pytest.raises(fvx.FvxError):
        fvx.SparseMatrix(ptr, col, v2, 40)
    M = fvx.SparseMatrix(ptr, col, val, 40, with_f32=False)
    X = torch.zeros((40, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(fvx.FvxError):
        M.spmm(X, Y=X)  # aliasing
    with pytest.raises(fvx.FvxError):
        M.spmm(X.float())  # no FP32 copy
    with pytest.raises(fvx.FvxError):
        M.spmm(X, k=5)  # ldx 4 < k
    with pytest.raises(fvx.FvxError):
        M.set_tile(4, 8, 256, dtype=fvx.F64)  # 32-byte vectors


@pytest.mark.parametrize("k", [1, 8, 64])
def test_tuned_tile_matches_the_oracle(k):
    import paper_2508_06710_amd as fvx
    ptr, col, val = _random_csr(80, 3000, 2000, 13)
    A = sp.csr_matrix((val, col, ptr), shape=(3000, 2000))
    M = fvx.SparseMatrix(ptr, col, val, 2000)
    ld = max(k, 4) if k > 1 else 1
    Xh = np.zeros((2000, ld))
    Xh[:, :k] = inputs.uniform(81, k, 2000 * k).reshape(2000, k)
    X = torch.as_tensor(Xh).cuda()
    Y0 = M.spmm(X, k=k).cpu().numpy()
    Y = torch.zeros((3000, ld), dtype=torch.float64, device="cuda")
    n = M.tune(X, Y, k=k, reps=2)
    assert n >= 4
    Y1 = M.spmm(X, k=k).cpu().numpy()
    _check64(A, Xh[:, :k], Y0[:, :k])
    _check64(A, Xh[:, :k], Y1[:, :k])  # the tuned tile may split rows: same bound, other rounding
