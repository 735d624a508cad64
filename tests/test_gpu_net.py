"""Learned initial guess on the GPU against the FP64 reference network.

The HIP network computes in FP32 (weights, activations, accumulation); the
oracle computes the same network in FP64 from the same FP32 parameters and
inputs.  Tolerances: a dot product of n FP32 terms has a typical relative
error of about sqrt(n) u (u = 2^-24, Higham and Mary's probabilistic bound),
n = 27 * 32 = 864 per output here, so about 2e-6 per layer and under 1e-5
through four layers (normwise).  Gradients are sums over every position of
the batch (thousands of terms, partial sums per block) of FP32 products of
quantities that carry the forward error: 1e-4 normwise per layer."""
import math

import numpy as np
import pytest
import torch

import inputs
import oracle
import oracle.net as onet
from helpers import Case

pytestmark = pytest.mark.gpu

FWD_TOL = 1e-5
GRAD_TOL = 1e-4


def _net(nx, ny, nz, batch, params):
    import paper_2508_06710_amd as fvx
    return fvx.GuessNet(nx, ny, nz, batch=batch, params=params)


def _params(seed=6, bias=0.05):
    p = inputs.net_init(seed, zero_output_layer=False)
    o = 0
    for ci, co, _ in onet.LAYERS:
        o += co * ci * 27
        p[o:o + co] = (bias * inputs.uniform(seed + 1, o, co)).astype(np.float32)
        o += co
    return p


def _identity_params():
    """Weights whose network output is exactly its second input channel: a
    zero output layer leaves the previous-pressure skip alone."""
    return np.zeros(onet.n_params(), np.float32)


def _samples(ns, nz, ny, nx, stream, ch=2):
    return inputs.uniform(41, stream, ns * ch * nz * ny * nx).reshape(ns, ch, nz, ny, nx).astype(np.float32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _layer_slices():
    out, o = [], 0
    for ci, co, _ in onet.LAYERS:
        out.append((slice(o, o + co * ci * 27), slice(o + co * ci * 27, o + co * ci * 27 + co)))
        o += co * ci * 27 + co
    return out


# Grids: several 256-thread blocks with a ragged tail; odd sizes; single
# rows, planes and columns (every padding rule degenerates there).
GRIDS = [(12, 10, 4, 3), (7, 5, 3, 2), (9, 1, 2, 2), (1, 6, 1, 1), (16, 8, 8, 1)]


@pytest.mark.parametrize("nx,ny,nz,ns", GRIDS)
def test_forward_matches_oracle(nx, ny, nz, ns):
    p = _params()
    x = _samples(ns, nz, ny, nx, 1)
    net = _net(nx, ny, nz, ns, p)
    out = net.forward(_dev(x)).cpu().numpy()
    ref = onet.forward(p.astype(np.float64), x.astype(np.float64))[-1]
    for n in range(ns):
        assert _rel(out[n], ref[n]) <= FWD_TOL, n


def test_forward_full_size_batch_sampled():
    """The training batch of the 64 x 64 x 8 channel (16 samples, two MFMA
    column blocks per wave): outputs at sampled cells against the oracle's
    receptive-field evaluation."""
    nx, ny, nz, ns = 64, 64, 8, 16
    p = _params()
    x = _samples(ns, nz, ny, nx, 12)
    net = _net(nx, ny, nz, ns, p)
    out = net.forward(_dev(x)).cpu().numpy()
    pick = inputs.u64(13, 0, 4 * 24).reshape(24, 4)
    got, ref = [], []
    for n_, z, y, xx in pick:
        n_, z, y, xx = int(n_ % ns), int(z % nz), int(y % ny), int(xx % nx)
        got.append(out[n_, 0, z, y, xx])
        ref.append(onet.forward_at(p.astype(np.float64), x.astype(np.float64), n_, z, y, xx))
    got, ref = np.array(got, np.float64), np.array(ref)
    # edges of the grid are always sampled too
    for n_, z, y, xx in ((0, 0, 0, 0), (ns - 1, nz - 1, ny - 1, nx - 1), (3, 0, ny - 1, 0)):
        got = np.append(got, out[n_, 0, z, y, xx])
        ref = np.append(ref, onet.forward_at(p.astype(np.float64), x.astype(np.float64), n_, z, y, xx))
    assert np.max(np.abs(got - ref)) <= FWD_TOL * np.max(np.abs(ref))


# (32, 16, 8, 5): 20,480 positions, more than the 256 position blocks of the
# 32 -> 32 layers' weight gradient hold in one 64-position chunk each, so each
# block takes a full chunk and a ragged one.
@pytest.mark.parametrize("nx,ny,nz,ns", GRIDS[:4] + [(32, 16, 8, 5)])
def test_gradients_match_oracle(nx, ny, nz, ns):
    p = _params()
    x = _samples(ns, nz, ny, nx, 2)
    t = _samples(ns, nz, ny, nx, 3, ch=1)
    net = _net(nx, ny, nz, ns, p)
    loss = net.gradients(_dev(x), _dev(t))
    g = net.grads()
    ref_loss, ref = onet.loss_and_grads(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    for w, b in _layer_slices():
        assert _rel(g[w], ref[w]) <= GRAD_TOL
        assert _rel(g[b], ref[b]) <= GRAD_TOL


def test_gradients_are_deterministic():
    p = _params()
    x, t = _samples(3, 4, 10, 12, 4), _samples(3, 4, 10, 12, 5, ch=1)
    net = _net(12, 10, 4, 3, p)
    net.gradients(_dev(x), _dev(t))
    g1 = net.grads()
    net.gradients(_dev(x), _dev(t))
    assert np.array_equal(g1, net.grads())


def test_adam_matches_oracle_on_given_gradients():
    """Adam alone: three steps from gradients that come from the input
    generator, written into the network's gradient buffer."""
    import torch as th
    nx, ny, nz, lr = 5, 4, 3, 1e-3
    p = _params()
    net = _net(nx, ny, nz, 1, p)
    pr, m, v = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    for step in (1, 2, 3):
        g = (inputs.normal(70, step, p.size) * 10.0 ** inputs.uniform(71, step, p.size, -6, 0)).astype(np.float32)
        net.grads_tensor().copy_(th.from_numpy(g))
        net.apply_adam(lr)
        pr, m, v = onet.adam(pr, g.astype(np.float64), m, v, step, lr)
    got = net.params().astype(np.float64)
    assert np.max(np.abs(got - pr)) <= 1e-4 * lr + 1e-6 * np.max(np.abs(pr))


def test_train_step_matches_oracle():
    """One training step end to end.  Adam's first step moves every parameter
    by lr * g / (|g| + eps), about lr times the sign of its gradient, so
    components whose gradient is within rounding of zero may move either way
    (|diff| <= 2 lr); the others must agree closely."""
    nx, ny, nz, ns, lr = 12, 10, 4, 3, 1e-3
    p = _params()
    x, t = _samples(ns, nz, ny, nx, 6), _samples(ns, nz, ny, nx, 7, ch=1)
    net = _net(nx, ny, nz, ns, p)
    loss = net.train_step(_dev(x), _dev(t), lr)
    got = net.params().astype(np.float64)
    ref_loss, g = onet.loss_and_grads(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    pr, _, _ = onet.adam(p.astype(np.float64), g, np.zeros(p.size), np.zeros(p.size), 1, lr)
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    for w, b in _layer_slices():
        for sl in (w, b):
            clear = np.abs(g[sl]) > 1e-3 * np.max(np.abs(g[sl]))
            d = np.abs(got[sl] - pr[sl])
            assert np.all(d[clear] <= 1e-3 * lr + 1e-6 * np.abs(pr[sl][clear]))
            assert np.all(d <= 2 * lr + 1e-6 * np.abs(pr[sl]))
            assert np.mean(clear) > 0.5


def _channel_case(nx=12, ny=10, k=4):
    spec = inputs.channel_base(nx, ny)
    return Case(spec, k, math.pi / k), spec


def test_prepare_and_guess_match_oracle():
    c, spec = _channel_case()
    nx, ny, k = spec.nx, spec.ny, c.k
    area = oracle.geometry(spec).area
    n = c.op.n_b * k
    b, pp, xs = (inputs.uniform(50, s, n) for s in (1, 2, 3))
    b += 0.3  # nonzero mean, removed for the singular operator
    p = _params()
    net = _net(nx, ny, k, 1, p)
    B, P, XS = c.op.to_rows(b), c.op.to_rows(pp), c.op.to_rows(xs)
    inp, tgt = net.prepare(c.op, B, P, XS)
    ref, s = onet.prepare(b, pp, area, c.dz, nx, ny, k, True)
    assert _rel(inp.cpu().numpy(), ref[0]) <= 1e-6
    assert _rel(tgt.cpu().numpy()[0], xs.reshape(k, ny, nx) / s) <= 1e-6
    inp0, _ = net.prepare(c.op, B)
    assert np.all(inp0.cpu().numpy()[1] == 0.0)
    X0 = net.guess(c.op, B, P)
    got = c.op.to_planes(X0)
    want = onet.guess(p.astype(np.float64), b, pp, area, c.dz, nx, ny, k, True)
    assert _rel(got, want) <= FWD_TOL
    X0n = net.guess(c.op, B)
    want_n = onet.guess(p.astype(np.float64), b, None, area, c.dz, nx, ny, k, True)
    assert _rel(c.op.to_planes(X0n), want_n) <= FWD_TOL


def _solve_case():
    c, spec = _channel_case(16, 12, 8)
    b = inputs.rhs_uniform(60, c.op.n_b * c.k)
    return c, spec, b


def _half_params():
    """Weights whose network output is half its second input channel:
    relu(p) and relu(-p) carried through the centre taps, the output layer
    subtracting half of p from the previous-pressure skip."""
    layers = [(np.zeros((co, ci, 3, 3, 3)), np.zeros(co)) for ci, co, _ in onet.LAYERS]
    layers[0][0][0, 1, 1, 1, 1] = 1.0
    layers[0][0][1, 1, 1, 1, 1] = -1.0
    for l in (1, 2):
        layers[l][0][0, 0, 1, 1, 1] = 1.0
        layers[l][0][1, 1, 1, 1, 1] = 1.0
    layers[3][0][0, 0, 1, 1, 1] = -0.5
    layers[3][0][0, 1, 1, 1, 1] = 0.5
    return onet.pack(layers).astype(np.float32)


@pytest.mark.parametrize("which", ["zero", "nan"])
def test_fallback_is_the_zero_guess_solve(which):
    """A useless guess (the network returns a random previous pressure) or a
    non-finite one loses to zero, and the solve is exactly the zero-guess
    solve."""
    import paper_2508_06710_amd as fvx
    c, spec, b = _solve_case()
    p = _identity_params()
    if which == "nan":
        p = _params()
        p[5] = np.nan
    net = _net(spec.nx, spec.ny, c.k, 1, p)
    B = c.op.to_rows(b)
    X, st = net.solve(c.op, B, c.op.to_rows(inputs.uniform(61, 1, b.size)), rtol=1e-10)
    X0, st0 = c.op.solve(B, rtol=1e-10)
    assert st["source"] == fvx.GUESS_ZERO
    assert st["iters"] == st0["iters"]
    assert torch.equal(X, X0)


def test_exact_previous_pressure_beats_its_fp32_copy():
    """The untrained network returns p_prev rounded to FP32; the exact
    previous pressure itself has the smaller residual and is chosen."""
    import paper_2508_06710_amd as fvx
    c, spec, b = _solve_case()
    B = c.op.to_rows(b)
    Xs, _ = c.op.solve(B, rtol=1e-12)
    net = _net(spec.nx, spec.ny, c.k, 1, _identity_params())
    X, st = net.solve(c.op, B, Xs.clone(), rtol=1e-10)
    assert st["source"] == fvx.GUESS_GIVEN
    assert st["r0_over_b"] < 1e-10
    assert st["iters"] <= 2
    # the network's own guess is p_prev with its mean removed, to FP32 rounding
    X0 = net.guess(c.op, B, Xs)
    xs = c.op.to_planes(Xs)
    assert _rel(c.op.to_planes(X0), xs - xs.mean()) <= 1e-6


def test_network_guess_is_used_when_best():
    """With weights that halve p_prev, p_prev = 2 x* gives a network guess
    accurate to FP32 rounding while p_prev itself is as bad as zero: the
    network's guess is chosen and CG needs fewer iterations than from zero."""
    import paper_2508_06710_amd as fvx
    c, spec, b = _solve_case()
    B = c.op.to_rows(b)
    Xs, _ = c.op.solve(B, rtol=1e-12)
    net = _net(spec.nx, spec.ny, c.k, 1, _half_params())
    X, st = net.solve(c.op, B, 2.0 * Xs, rtol=1e-10)
    assert st["source"] == fvx.GUESS_NET
    # FP32 rounding of the guess, amplified by at most cond(L)
    assert st["r0_over_b"] < 1e-2
    _, stz = c.op.solve(B, rtol=1e-10)
    assert st["iters"] < stz["iters"]
    x = c.op.to_planes(X)
    bp = oracle.project_mean(b, 1)
    assert np.linalg.norm(bp - oracle.spmv(c.L, x)) <= 1.0001e-10 * np.linalg.norm(bp)


def test_net_argument_errors():
    import paper_2508_06710_amd as fvx
    c, spec, b = _solve_case()
    net = _net(spec.nx, spec.ny, c.k, 2, _params())
    B = c.op.to_rows(b)
    other = Case(inputs.channel_base(spec.nx, spec.ny), 4, math.pi / 4)
    with pytest.raises(fvx.FvxError) as e:
        net.guess(other.op, other.op.to_rows(np.zeros(other.op.n_b * 4)))
    assert e.value.code == fvx._lib.E_ARG
    tri = Case(inputs.unit_square_triangles(2), c.k, 0.1)
    with pytest.raises(fvx.FvxError):
        net.solve(tri.op, tri.op.to_rows(np.zeros(tri.op.n_b * c.k)))
    x = _dev(_samples(3, c.k, spec.ny, spec.nx, 9))
    with pytest.raises(fvx.FvxError):
        net.forward(x)
    with pytest.raises(ValueError):
        net.set_params(np.zeros(10, np.float32))


def test_checkpoint_resumes_training_exactly(tmp_path):
    """fvx_net_save / fvx_net_load: a network restored from a checkpoint
    (parameters, Adam moments, step count) takes the same next training step
    as the one that kept training, bitwise; a checkpoint loads into a network
    of another grid; a file that is not a checkpoint, or is truncated, is
    refused and leaves the network unchanged."""
    nx, ny, nz, ns = 12, 10, 4, 3
    p = _params()
    x, t = _samples(ns, nz, ny, nx, 21), _samples(ns, nz, ny, nx, 22, ch=1)
    a = _net(nx, ny, nz, ns, p)
    for _ in range(2):
        a.train_step(_dev(x), _dev(t), 1e-3)
    path = str(tmp_path / "net.ckpt")
    a.save(path)
    b = _net(nx, ny, nz, ns, np.zeros_like(p))
    b.load(path)
    saved = a.params()
    assert np.array_equal(saved, b.params())
    a.train_step(_dev(x), _dev(t), 1e-3)
    b.train_step(_dev(x), _dev(t), 1e-3)
    assert np.array_equal(a.params(), b.params())
    other = _net(7, 5, 3, 1, np.zeros_like(p))
    other.load(path)
    assert np.array_equal(other.params(), saved)
    raw = open(path, "rb").read()
    assert raw[:8] == b"FVXNET01" and len(raw) == 16 + 3 * 4 * p.size
    before = b.params()
    bad = str(tmp_path / "bad.ckpt")
    open(bad, "wb").write(b"NOTANET!" + raw[8:])
    from paper_2508_06710_amd import FvxError
    with pytest.raises(FvxError):
        b.load(bad)
    open(bad, "wb").write(raw[:len(raw) // 2])
    with pytest.raises(FvxError):
        b.load(bad)
    with pytest.raises(FvxError):
        b.load(str(tmp_path / "missing.ckpt"))
    assert np.array_equal(b.params(), before)
