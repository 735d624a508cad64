"""Pins of the oracle's 13- and 27-point operators (the higher-order stencils
of the paper's Section 4.1) against closed forms: their Fourier symbols on a
uniform periodic box, the order of accuracy on smooth fields, symmetry, zero
row sums and (27-point) negative semidefiniteness on stretched meshes."""
import math

import numpy as np
import pytest

import inputs
import oracle


def _box(n, m, periodic=True):
    return inputs.CartSpec(n, m, 2 * math.pi, 0.0, 2 * math.pi, 0.0, periodic, periodic)


def _symbol(stencil, th, h):
    if stencil == 27:
        kk = [(2 - 2 * math.cos(t)) / hh for t, hh in zip(th, h)]
        mm = [hh * (4 + 2 * math.cos(t)) / 6 for t, hh in zip(th, h)]
        return -(kk[0] * mm[1] * mm[2] + mm[0] * kk[1] * mm[2] + mm[0] * mm[1] * kk[2])
    vol = h[0] * h[1] * h[2]
    return vol * sum((4 / 3) * (2 * math.cos(t) - 2) / hh ** 2 - (1 / 6) * (2 * math.cos(2 * t) - 2) / (2 * hh ** 2)
                     for t, hh in zip(th, h))


@pytest.mark.parametrize("stencil", [13, 27])
@pytest.mark.parametrize("mode", [(1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 3, 1), (3, 1, 2), (4, 2, 2)])
def test_fourier_eigenpairs_on_uniform_periodic_box(stencil, mode):
    nx, ny, k = 8, 6, 5
    spec = _box(nx, ny)
    dz = 2 * math.pi / k
    A = oracle.stencil_lap(spec, k, dz, stencil)
    th = [2 * math.pi * mode[0] / nx, 2 * math.pi * mode[1] / ny, 2 * math.pi * mode[2] / k]
    h = [2 * math.pi / nx, 2 * math.pi / ny, dz]
    l, j, i = np.meshgrid(np.arange(k), np.arange(ny), np.arange(nx), indexing="ij")
    v = np.cos(th[0] * i + th[1] * j + th[2] * l).ravel()
    lam = _symbol(stencil, th, h)
    assert np.max(np.abs(A @ v - lam * v)) <= 1e-12 * max(1.0, abs(lam))


@pytest.mark.parametrize("stencil,order", [(13, 4.0), (27, 2.0)])
def test_order_of_accuracy_on_a_smooth_periodic_field(stencil, order):
    errs = []
    for n in (16, 32):
        spec = _box(n, n)
        dz = 2 * math.pi / n
        A = oracle.stencil_lap(spec, n, dz, stencil)
        c = (np.arange(n) + 0.5) * 2 * math.pi / n
        z, y, x = np.meshgrid(c, c, c, indexing="ij")
        f = np.sin(x) * np.cos(2 * y) * np.sin(z + 0.3)
        exact = -6.0 * f * (2 * math.pi / n) ** 3
        errs.append(np.max(np.abs(A @ f.ravel() - exact.ravel())) / (2 * math.pi / n) ** 3)
    p = math.log2(errs[0] / errs[1])
    assert abs(p - order) <= 0.2, (errs, p)


@pytest.mark.parametrize("stencil", [13, 27])
@pytest.mark.parametrize("spec", [inputs.channel_base(7, 9), inputs.convection_base(6, 5), _box(3, 4)])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_symmetric_with_zero_row_sums(stencil, spec, k):
    A = oracle.stencil_lap(spec, k, 0.37, stencil)
    assert A.shape == (spec.nx * spec.ny * k,) * 2
    scale = abs(A).max()
    assert abs(A - A.T).max() <= 1e-14 * scale
    assert np.max(np.abs(A @ np.ones(A.shape[0]))) <= 1e-13 * scale


@pytest.mark.parametrize("spec", [inputs.channel_base(5, 6), inputs.convection_base(4, 5)])
def test_27_point_negative_semidefinite_on_stretched_meshes(spec):
    A = oracle.stencil_lap(spec, 3, 0.4, 27).toarray()
    ev = np.linalg.eigvalsh(A)
    assert ev.max() <= 1e-12 * abs(ev).max()
    assert np.sum(np.abs(ev) <= 1e-10 * abs(ev).max()) == 1  # only the constants


def test_stencil_nonzeros_per_row():
    spec = _box(8, 7)
    for stencil in (13, 27):
        A = oracle.stencil_lap(spec, 6, 0.5, stencil)
        assert set(np.diff(A.indptr)) == {stencil}
