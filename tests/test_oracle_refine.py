"""Pins of the oracle's coarse-to-fine mapping (oracle/refine.py) against
facts independent of it: partition of unity, exact reproduction of fields
that are linear between the coarse centres, the identity for rf = 1,
second-order accuracy on a smooth periodic field, children that tile their
parent; and host parity of the library's mapping and refined mesh with it."""
import math

import numpy as np
import pytest

import inputs
import oracle
from oracle import refine as orf

SPECS = [inputs.channel_base(12, 10), inputs.convection_base(9, 7),
         inputs.CartSpec(5, 4, 2.0, 0.0, 1.0, 0.0, True, True), inputs.CartSpec(1, 3, 1.0, 0.0, 1.0, 0.5, True, False)]


@pytest.mark.parametrize("spec", SPECS)
@pytest.mark.parametrize("rf", [1, 2, 3])
def test_rows_are_convex_weights(spec, rf):
    P = orf.prolongation(spec, rf)
    assert P.shape == (spec.nx * spec.ny * rf * rf, spec.nx * spec.ny)
    assert np.all(P.data > 0) and np.all(P.data <= 1 + 1e-15)
    assert np.max(np.abs(P @ np.ones(P.shape[1]) - 1.0)) <= 1e-14
    assert P.getnnz(axis=1).max() <= 4


@pytest.mark.parametrize("spec", SPECS[:3])
def test_identity_for_rf_one(spec):
    P = orf.prolongation(spec, 1)
    assert abs(P - np.eye(P.shape[0])).max() <= 1e-15


@pytest.mark.parametrize("spec", [inputs.channel_base(12, 10), inputs.convection_base(9, 7)])
def test_fields_linear_in_y_are_reproduced_between_centres(spec):
    P = orf.prolongation(spec, 2)
    cx, cy = orf.coarse_centres(spec)
    fx, fy = orf.fine_centres(spec, 2)
    a, b = 0.3, -1.7
    fine = P @ (a + b * cy)
    inside = (fy >= cy.min()) & (fy <= cy.max())
    assert np.max(np.abs(fine[inside] - (a + b * fy[inside]))) <= 1e-13
    # beyond the end centres (walls): the end value
    assert np.allclose(fine[fy < cy.min()], a + b * cy.min(), atol=1e-13)


def test_second_order_on_a_smooth_periodic_field():
    errs = []
    for n in (16, 32, 64):
        spec = inputs.CartSpec(n, n, 2 * math.pi, 0.0, 2 * math.pi, 0.0, True, True)
        P = orf.prolongation(spec, 2)
        cx, cy = orf.coarse_centres(spec)
        fx, fy = orf.fine_centres(spec, 2)
        f = lambda x, y: np.sin(x) * np.cos(2 * y)
        errs.append(np.max(np.abs(P @ f(cx, cy) - f(fx, fy))))
    p = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(q - 2.0) <= 0.1 for q in p), (errs, p)


@pytest.mark.parametrize("spec", SPECS)
@pytest.mark.parametrize("rf", [2, 3])
def test_library_mapping_and_mesh_match_the_oracle(spec, rf):
    import paper_2508_06710_amd as fvx
    m = fvx.Mesh.from_spec(spec)
    ptr, col, val = m.prolongation(rf)
    import scipy.sparse as sp
    A = sp.csr_matrix((val, col, ptr), shape=(spec.nx * spec.ny * rf * rf, spec.nx * spec.ny))
    B = orf.prolongation(spec, rf)
    assert abs(A - B).max() <= 1e-14
    f = m.refine(rf)
    cx, cy = f.centroids()
    fx, fy = orf.fine_centres(spec, rf)
    assert np.max(np.abs(cx - fx)) <= 1e-13 and np.max(np.abs(cy - fy)) <= 1e-13
    # the children tile their parent: fine areas summed per parent equal the coarse areas
    area_f = f.faces()[0]
    area_c = m.faces()[0]
    I, J = np.meshgrid(np.arange(spec.nx * rf), np.arange(spec.ny * rf))
    parent = ((J // rf) * spec.nx + (I // rf)).ravel()
    assert np.allclose(np.bincount(parent, weights=area_f), area_c, rtol=1e-13, atol=0)


def test_refinement_rejects_unstructured_meshes():
    import paper_2508_06710_amd as fvx
    m = fvx.Mesh.from_spec(inputs.unit_square_triangles(3))
    with pytest.raises(fvx.FvxError):
        m.refine(2)
    with pytest.raises(fvx.FvxError):
        m.prolongation(2)
