"""Inline mesh refinement on a Cartesian base (Section 3.3): the refined mesh
and the coarse-to-fine state mapping, written independently of the library
(TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
leg may use it).

The refined mesh splits every coarse cell into rf x rf equal children, as
classical adaptive mesh refinement does.  The mapping evaluates, at every
fine cell centre, the piecewise-linear interpolant of the coarse cell-centre
values along each axis (the tensor product of the two 1D interpolants):
periodic axes interpolate across the period, wall-bounded axes keep the end
centre's value beyond it.  Each 1D interpolant is np.interp of the unit
vectors on the (periodically extended) coarse centres; the 2D operator is the
Kronecker product of the y and x operators in the j*nx+i cell order.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def cart_faces(spec):
    """Face coordinates of an inputs.CartSpec: x uniform on [x0, x0+Lx];
    y on [y0, y1] with y_j = y0 + (y1-y0)(1 + tanh(s(2j/n - 1))/tanh s)/2
    (uniform when s == 0)."""
    xf = spec.x0 + spec.Lx * np.arange(spec.nx + 1) / spec.nx
    t = np.arange(spec.ny + 1) / spec.ny
    if spec.stretch == 0.0:
        yf = spec.y0 + (spec.y1 - spec.y0) * t
    else:
        s = spec.stretch
        yf = spec.y0 + (spec.y1 - spec.y0) * 0.5 * (1.0 + np.tanh(s * (2.0 * t - 1.0)) / math.tanh(s))
    return xf, yf


def split_faces(f, rf):
    """Every interval of f split into rf equal parts."""
    f = np.asarray(f, dtype=np.float64)
    parts = [f[:-1, None] + (f[1:, None] - f[:-1, None]) * (np.arange(rf)[None, :] / rf)]
    return np.concatenate([np.concatenate(parts, axis=None), f[-1:]])


def interp_1d(f_coarse, f_fine, periodic):
    """Dense [n_fine, n_coarse] matrix of the piecewise-linear interpolation
    of coarse centre values at fine centres."""
    c = 0.5 * (f_coarse[1:] + f_coarse[:-1])
    x = 0.5 * (f_fine[1:] + f_fine[:-1])
    n = len(c)
    P = np.zeros((len(x), n))
    if n == 1:
        P[:, 0] = 1.0
        return P
    L = f_coarse[-1] - f_coarse[0]
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        if periodic:
            nodes = np.concatenate([[c[-1] - L], c, [c[0] + L]])
            vals = np.concatenate([[e[-1]], e, [e[0]]])
        else:
            nodes, vals = c, e
        P[:, i] = np.interp(x, nodes, vals)
    return P


def prolongation(spec, rf: int) -> sp.csr_matrix:
    """The coarse-to-fine mapping of an inputs.CartSpec refined rf times."""
    xf, yf = cart_faces(spec)
    Px = interp_1d(xf, split_faces(xf, rf), spec.periodic_x)
    Py = interp_1d(yf, split_faces(yf, rf), spec.periodic_y)
    P = sp.kron(sp.csr_matrix(Py), sp.csr_matrix(Px), format="csr")
    P.eliminate_zeros()
    return P


def fine_centres(spec, rf: int):
    """Centres (x, y) of the refined cells in j*nx+i order."""
    xf, yf = cart_faces(spec)
    X, Y = split_faces(xf, rf), split_faces(yf, rf)
    cx, cy = 0.5 * (X[1:] + X[:-1]), 0.5 * (Y[1:] + Y[:-1])
    gx, gy = np.meshgrid(cx, cy)
    return gx.ravel(), gy.ravel()


def coarse_centres(spec):
    xf, yf = cart_faces(spec)
    cx, cy = 0.5 * (xf[1:] + xf[:-1]), 0.5 * (yf[1:] + yf[:-1])
    gx, gy = np.meshgrid(cx, cy)
    return gx.ravel(), gy.ravel()
