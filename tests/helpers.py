"""Shared helpers of the GPU parity tests: build the same case on both sides
and compare element by element.  Inputs come from the seeded generators in
``inputs``; expected values come only from ``oracle``."""
import math

import numpy as np

import inputs
import oracle

U32 = 2.0 ** -24


class Case:
    """One (base mesh, k, dz, coupling, wall) case, on the GPU and in the oracle."""

    def __init__(self, spec, k, dz=None, coupling=1, dirichlet=False, with_f32=True, order=None):
        import paper_2508_06710_amd as fvx
        self.fvx = fvx
        self.k = k
        self.dz = dz if dz is not None else math.pi / k
        self.coupling, self.dirichlet = coupling, dirichlet
        mesh = fvx.Mesh.from_spec(spec, order=order)
        if mesh.cell_perm is not None:
            # the oracle assembles the same numbering from the renumbered triangles
            spec = type(spec)(spec.points, np.ascontiguousarray(spec.triangles[mesh.cell_perm]), spec.name)
        self.spec = spec
        self.op = fvx.Operator(mesh, k, self.dz, coupling, fvx.DIRICHLET if dirichlet else fvx.NEUMANN,
                               with_f32=with_f32)
        self.m3 = oracle.Mesh3D(oracle.geometry(spec), k, self.dz, coupling, dirichlet)
        self._L = self._M = self._G = None

    @property
    def L(self):
        if self._L is None:
            self._L = self.m3.lap()
        return self._L

    @property
    def M(self):
        if self._M is None:
            self._M = self.m3.div()
        return self._M

    @property
    def G(self):
        if self._G is None:
            self._G = self.m3.grad()
        return self._G

    def __repr__(self):
        return f"Case({self.spec}, k={self.k}, coupling={self.coupling}, dirichlet={self.dirichlet})"


def componentwise(y, ref, A, x):
    """max_i |y_i - ref_i| / (|A| |x|)_i (rows with a zero bound must match exactly)."""
    bound = abs(A) @ np.abs(x)
    d = np.abs(y - ref)
    z = bound == 0
    assert np.all(d[z] == 0), "nonzero result where |A||x| vanishes"
    return float(np.max(d[~z] / bound[~z])) if np.any(~z) else 0.0


def row_nnz(A):
    return np.diff(A.indptr)


def fp32_bound_factor(A):
    """Per-row FP32 bound on |y32 - y| / (|A||x|): the products and sums of a
    row of n entries (Higham's gamma_n) plus one rounding per stored entry and
    the FP32 rebuild of the diagonal from the off-diagonal sum -- (2n + 3) u."""
    n = row_nnz(A) + 2
    return (2 * n + 3) * U32


def stream_of(seed, stream, n):
    return inputs.uniform(seed, stream, n)
