"""Pins of the oracle's det J (the change of variables of Sec. 2.2) and of its
count of elements with det J <= 0 (signed determinant, integrated as
written), against closed forms that do not go through the shape functions."""
import numpy as np
import pytest

import oracle
from paper_1504_01023_amd import inputs

TET_REF = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
PRISM_REF = np.array([[0, 0, -1], [1, 0, -1], [0, 1, -1], [0, 0, 1], [1, 0, 1], [0, 1, 1]],
                     dtype=np.float64)


def soa(verts):
    """(n, n_vert, 3) vertex coordinates -> SoA (3 n_vert, n)."""
    v = np.asarray(verts, dtype=np.float64)
    return np.ascontiguousarray(v.reshape(v.shape[0], -1).T)


@pytest.mark.parametrize("elem,ref,n_q", [("tet4", TET_REF, 4), ("prism6", PRISM_REF, 6)])
def test_reference_element_has_unit_det(elem, ref, n_q):
    d = oracle.jacobian_dets(elem, soa(ref[None]), oracle.quad_rule(elem, n_q))
    assert np.allclose(d, 1.0, rtol=0, atol=1e-15)


def test_tet_det_is_the_edge_triple_product():
    rng = np.random.default_rng(5)
    v = rng.normal(size=(200, 4, 3))
    e = v[:, 1:] - v[:, :1]
    triple = np.einsum("ei,ei->e", e[:, 0], np.cross(e[:, 1], e[:, 2]))
    d = oracle.jacobian_dets("tet4", soa(v), oracle.quad_rule("tet4", 4))
    for q in range(d.shape[1]):
        assert np.allclose(d[:, q], triple, rtol=1e-12, atol=1e-13)


def test_affine_prism_det_is_constant_triple_product():
    # top = bottom + h: J = [X1 - X0, X2 - X0, h / 2] at every point
    rng = np.random.default_rng(6)
    b = rng.normal(size=(100, 3, 3))
    h = rng.normal(size=(100, 1, 3))
    v = np.concatenate([b, b + h], axis=1)
    e1, e2 = b[:, 1] - b[:, 0], b[:, 2] - b[:, 0]
    triple = np.einsum("ei,ei->e", e1, np.cross(e2, 0.5 * h[:, 0]))
    d = oracle.jacobian_dets("prism6", soa(v), oracle.quad_rule("prism6", 6))
    assert np.allclose(d, triple[:, None], rtol=1e-12, atol=1e-13)


def vertical_prisms(rng, n, heights):
    """Prisms with a horizontal bottom triangle at z = 0 and vertical edges of
    heights h_i: det J(xi, eta, zeta) = 2 A_signed h(xi, eta) / 2 with
    h = sum_i N_i h_i, and the volume is A |mean h| for h of one sign."""
    b = np.concatenate([rng.uniform(-1, 1, size=(n, 3, 2)), np.zeros((n, 3, 1))], axis=2)
    top = b.copy()
    top[:, :, 2] = heights
    return b, np.concatenate([b, top], axis=1)


def test_vertical_prism_det_and_volume():
    rng = np.random.default_rng(7)
    n = 64
    hts = rng.uniform(0.2, 2.0, size=(n, 3))
    b, v = vertical_prisms(rng, n, hts)
    xi, w = oracle.quad_rule("prism6", 6)
    d = oracle.jacobian_dets("prism6", soa(v), (xi, w))
    e1, e2 = b[:, 1, :2] - b[:, 0, :2], b[:, 2, :2] - b[:, 0, :2]
    twice_area = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    N = np.stack([1 - xi[:, 0] - xi[:, 1], xi[:, 0], xi[:, 1]], axis=1)   # (n_q, 3)
    h_at = hts @ N.T                                                       # (n, n_q)
    assert np.allclose(d, 0.5 * twice_area[:, None] * h_at, rtol=1e-12, atol=1e-14)
    # sum_q w_q det_q = signed volume = area * mean height (the top is planar)
    vol = 0.5 * twice_area * hts.mean(axis=1)
    assert np.allclose(d @ w, vol, rtol=1e-12, atol=1e-14)


def test_vertex_swap_negates_det():
    for wl, swap, n_q in ((inputs.tet_poisson(3, seed=2), (1, 2), 4),
                          (inputs.prism_cdr_qp(4, 3, seed=2), (1, 2, 4, 5), 6)):
        c = wl.mesh.coords
        nv = c.shape[0] // 3
        v = c.reshape(nv, 3, -1).copy()
        perm = list(range(nv))
        for a, bb in zip(swap[::2], swap[1::2]):
            perm[a], perm[bb] = perm[bb], perm[a]
        rule = oracle.quad_rule(wl.elem, n_q)
        d0 = oracle.jacobian_dets(wl.elem, c, rule)
        d1 = oracle.jacobian_dets(wl.elem, v[perm].reshape(nv * 3, -1), rule)
        # the swap mirrors the reference element (xi <-> eta); the rules are
        # symmetric under that mirror, so the values per element match as sets
        assert np.allclose(np.sort(d1, axis=1), np.sort(-d0, axis=1), rtol=1e-11, atol=0)


@pytest.mark.parametrize("make,n_q", [(lambda: inputs.tet_poisson(4, seed=3), 1),
                                      (lambda: inputs.prism_cdr_qp(6, 4, seed=3), 6),
                                      (lambda: inputs.prism_elasticity(5, 4, seed=4), 6)])
def test_generated_meshes_have_no_inverted_elements(make, n_q):
    wl = make()
    assert oracle.count_inverted(wl.elem, wl.mesh.coords, oracle.quad_rule(wl.elem, n_q)) == 0


def test_count_semantics_on_planted_cases():
    rng = np.random.default_rng(8)
    xi, w = oracle.quad_rule("prism6", 6)
    N = np.stack([1 - xi[:, 0] - xi[:, 1], xi[:, 0], xi[:, 1]], axis=1)
    # heights where mean h > 0 but h < 0 near vertex 0: det changes sign inside
    hts = np.tile([-2.0, 3.0, 3.0], (32, 1)) + rng.uniform(-0.1, 0.1, size=(32, 3))
    _, v = vertical_prisms(rng, 32, hts)
    # orient every bottom triangle counter-clockwise so that det > 0 where h > 0
    e1, e2 = v[:, 1, :2] - v[:, 0, :2], v[:, 2, :2] - v[:, 0, :2]
    cw = (e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]) < 0
    v[cw] = v[cw][:, [0, 2, 1, 3, 5, 4]]
    hts[cw] = hts[cw][:, [0, 2, 1]]
    neg_somewhere = ((hts @ N.T) <= 0).any(axis=1)
    assert neg_somewhere.any()
    assert oracle.count_inverted("prism6", soa(v), (xi, w)) == int(neg_somewhere.sum())
    # a flat tetrahedron (all vertices in one plane z = const) has det J = 0 exactly
    t = rng.normal(size=(5, 4, 3))
    t[:, :, 2] = 0.75
    assert np.all(oracle.jacobian_dets("tet4", soa(t), oracle.quad_rule("tet4", 1)) == 0.0)
    assert oracle.count_inverted("tet4", soa(t), oracle.quad_rule("tet4", 1)) == 5
