"""Pins of the reference network (oracle/net.py) against facts that do not
come from the oracle itself: torch's conv3d with torch's own padding modes,
torch autograd, torch's Adam, central finite differences and the adjoint
identity.  None of these call into the oracle; the oracle calls none of
them."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import inputs
import oracle.net as onet

RNG_SEED = 31


def _rand(shape, stream):
    return inputs.uniform(RNG_SEED, stream, int(np.prod(shape))).reshape(shape)


def _torch_pad(a):
    a = F.pad(a, (1, 1, 0, 0, 1, 1), mode="circular")     # x and z periodic
    return F.pad(a, (0, 0, 1, 1, 0, 0), mode="replicate")  # y edge copy


def _torch_net(params, inp):
    x = inp
    for (W, b), (_, _, relu) in zip(params, onet.LAYERS):
        x = F.conv3d(_torch_pad(x), W, b)
        if relu:
            x = torch.relu(x)
    return x + inp[:, 1:2]


def _torch_params(flat):
    return [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True))
            for W, b in onet.unpack(flat)]


def _params(scale_bias=0.1):
    p = inputs.net_init(6, zero_output_layer=False).astype(np.float64)
    # nonzero biases so that the bias paths are exercised
    o = 0
    for ci, co, _ in onet.LAYERS:
        o += co * ci * 27
        p[o:o + co] = scale_bias * inputs.uniform(7, o, co)
        o += co
    return p


@pytest.mark.parametrize("shape", [(4, 3, 5), (1, 4, 3), (3, 1, 2), (2, 3, 1), (1, 1, 1)])
def test_conv_matches_torch_conv3d(shape):
    Z, Y, X = shape
    a = _rand((2, 3, Z, Y, X), 1)
    W = _rand((4, 3, 3, 3, 3), 2)
    b = _rand((4,), 3)
    ref = F.conv3d(_torch_pad(torch.tensor(a)), torch.tensor(W), torch.tensor(b)).numpy()
    out = onet.conv(a, W, b)
    assert np.max(np.abs(out - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_forward_matches_torch():
    p = _params()
    inp = _rand((2, 2, 3, 5, 6), 4)
    ref = _torch_net(_torch_params(p), torch.tensor(inp)).detach().numpy()
    out = onet.forward(p, inp)[-1]
    assert out.shape == (2, 1, 3, 5, 6)
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("shape", [(3, 5, 6), (1, 1, 4), (2, 1, 1)])
def test_gradients_match_torch_autograd(shape):
    p = _params()
    inp = _rand((2, 2) + shape, 5)
    tgt = _rand((2, 1) + shape, 6)
    tp = _torch_params(p)
    loss_t = torch.mean((_torch_net(tp, torch.tensor(inp)) - torch.tensor(tgt)) ** 2)
    loss_t.backward()
    ref = np.concatenate([np.concatenate([W.grad.numpy().ravel(), b.grad.numpy().ravel()]) for W, b in tp])
    loss, g = onet.loss_and_grads(p, inp, tgt)
    assert abs(loss - loss_t.item()) <= 1e-14 * loss
    assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_gradients_match_central_differences():
    p = _params()
    inp = _rand((2, 2, 3, 4, 5), 8)
    tgt = _rand((2, 1, 3, 4, 5), 9)
    _, g = onet.loss_and_grads(p, inp, tgt)
    idx = (inputs.u64(3, 10, 40) % np.uint64(p.size)).astype(np.int64)
    # include every bias block and the first weight of every layer
    o = 0
    extra = []
    for ci, co, _ in onet.LAYERS:
        extra += [o, o + co * ci * 27]
        o += co * ci * 27 + co
    h = 1e-6
    for i in np.concatenate([idx, extra]):
        e = np.zeros_like(p)
        e[i] = h
        lp = np.mean((onet.forward(p + e, inp)[-1] - tgt) ** 2)
        lm = np.mean((onet.forward(p - e, inp)[-1] - tgt) ** 2)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3 * np.max(np.abs(g))), i


@pytest.mark.parametrize("shape", [(3, 4, 5), (1, 1, 1), (2, 1, 3), (1, 2, 1)])
def test_pad_adjoint_identity(shape):
    a = _rand((2, 3) + shape, 11)
    gshape = (2, 3) + tuple(s + 2 for s in shape)
    g = _rand(gshape, 12)
    lhs = float(np.sum(onet.pad(a) * g))
    rhs = float(np.sum(a * onet.pad_adjoint(g)))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1.0)


def test_constant_field_reduces_to_tap_sums():
    # padding copies or wraps cells, so a constant input stays constant and
    # every output is the bias plus the sum of all taps times the constant
    W = _rand((3, 2, 3, 3, 3), 13)
    b = _rand((3,), 14)
    a = np.full((1, 2, 3, 4, 5), 0.7)
    out = onet.conv(a, W, b)
    expect = b + 0.7 * W.sum(axis=(1, 2, 3, 4))
    assert np.allclose(out, expect[None, :, None, None, None], rtol=0, atol=1e-14)


def test_periodic_shift_equivariance():
    p = _params()
    inp = _rand((1, 2, 4, 5, 6), 15)
    out = onet.forward(p, inp)[-1]
    sx = onet.forward(p, np.roll(inp, 2, axis=-1))[-1]
    sz = onet.forward(p, np.roll(inp, 1, axis=-3))[-1]
    assert np.allclose(np.roll(out, 2, axis=-1), sx, rtol=0, atol=1e-13)
    assert np.allclose(np.roll(out, 1, axis=-3), sz, rtol=0, atol=1e-13)


def test_adam_matches_torch_adam():
    p0 = _rand((50,), 16)
    grads = [_rand((50,), 17 + t) for t in range(3)]
    tp = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = onet.adam(p, g, m, v, t, 1e-3)
    assert np.max(np.abs(p - tp.detach().numpy())) <= 1e-15


def test_prepare_and_guess_scaling():
    nx, ny, k, dz = 6, 5, 3, 0.4
    area = 0.5 + _rand((nx * ny,), 20) ** 2
    b = _rand((k * nx * ny,), 21)
    pp = _rand((k * nx * ny,), 22)
    inp, s = onet.prepare(b, pp, area, dz, nx, ny, k, True)
    f = (b.reshape(k, ny, nx) - b.mean()) / (area.reshape(1, ny, nx) * dz)
    assert np.isclose(s, np.sqrt(np.mean(f * f)), rtol=1e-15)
    assert np.allclose(inp[0, 0], f / s, rtol=1e-14, atol=0)
    assert np.allclose(inp[0, 1], pp.reshape(k, ny, nx) / s, rtol=1e-14, atol=0)
    # the input is invariant and the guess equivariant under a common scaling
    p = _params()
    g1 = onet.guess(p, b, pp, area, dz, nx, ny, k, True)
    g2 = onet.guess(p, 8.0 * b, 8.0 * pp, area, dz, nx, ny, k, True)
    assert np.allclose(g2, 8.0 * g1, rtol=1e-13, atol=1e-15 * np.max(np.abs(g2)))
    assert abs(g1.mean()) <= 1e-15 * np.max(np.abs(g1)) * g1.size
    # zero right-hand side: scale 1
    _, s0 = onet.prepare(np.zeros_like(b), None, area, dz, nx, ny, k, True)
    assert s0 == 1.0


def test_n_params_matches_layer_shapes():
    assert onet.n_params() == 2 * 32 * 27 + 32 + 2 * (32 * 32 * 27 + 32) + 32 * 27 + 1
    assert inputs.net_init(6).size == onet.n_params()


def test_untrained_network_returns_the_previous_pressure():
    # zero output layer: out = input channel 1 exactly
    inp = _rand((2, 2, 3, 4, 5), 30)
    out = onet.forward(inputs.net_init(6).astype(np.float64), inp)[-1]
    assert np.array_equal(out[:, 0], inp[:, 1])


@pytest.mark.parametrize("shape", [(3, 5, 6), (1, 2, 3)])
def test_forward_at_one_cell_equals_whole_grid_forward(shape):
    p = _params()
    inp = _rand((2,) + (2,) + shape, 31)
    full = onet.forward(p, inp)[-1]
    Z, Y, X = shape
    for n in range(2):
        for z in range(Z):
            for y in range(Y):
                for x in range(X):
                    assert abs(onet.forward_at(p, inp, n, z, y, x) - full[n, 0, z, y, x]) <= 1e-12
