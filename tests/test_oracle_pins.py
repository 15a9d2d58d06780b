"""Pins of the CPU oracle against what the paper and the mathematics fix:
closed forms, invariants, brute-force quadrature, rule moments and
metamorphic relations. No GPU; no part of the GPU library is used."""
import math

import numpy as np
import pytest

import oracle
from paper_1504_01023_amd import inputs
from tests import _witness as W

REF_TET = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
REF_PRISM = np.array([[0, 0, -1], [1, 0, -1], [0, 1, -1], [0, 0, 1], [1, 0, 1], [0, 1, 1]], float)


def soa(X):
    """One element's vertex rows (n_vert, 3) -> SoA (n_vert*3, 1)."""
    return np.ascontiguousarray(X.reshape(-1, 1))


def slots_with(**kw):
    u = np.zeros(20)
    names = {"c00": 0, "d0": 16}
    for k, v in kw.items():
        if k in names:
            u[names[k]] = v
        elif k.startswith("c") and len(k) == 3:
            u[4 * int(k[1]) + int(k[2])] = v
        elif k.startswith("d"):
            u[16 + int(k[1])] = v
    return u


LAPLACE = slots_with(c11=1, c22=1, c33=1)


# ---------------------------------------------------------------- rules
def _tet_monomial(a, b, c):
    return math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)


def _prism_monomial(a, b, c):
    tri = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
    line = (1 - (-1) ** (c + 1)) / (c + 1)
    return tri * line


@pytest.mark.parametrize("n_q,deg", [(1, 1), (4, 2)])
def test_tet_rule_moments(n_q, deg):
    xi, w = oracle.quad_rule("tet4", n_q)
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            for c in range(deg + 1 - a - b):
                got = np.sum(w * xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c)
                assert got == pytest.approx(_tet_monomial(a, b, c), rel=1e-14, abs=1e-16)
    # and not exact one degree higher (the rule's degree is what is claimed)
    got = np.sum(w * xi[:, 0] ** (deg + 1))
    assert abs(got - _tet_monomial(deg + 1, 0, 0)) > 1e-6


def test_prism_rule_moments():
    xi, w = oracle.quad_rule("prism6", 6)
    for a in range(3):
        for b in range(3 - a):
            for c in range(4):
                got = np.sum(w * xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c)
                assert got == pytest.approx(_prism_monomial(a, b, c), rel=1e-14, abs=1e-16)
    assert abs(np.sum(w * xi[:, 2] ** 4) - _prism_monomial(0, 0, 4)) > 1e-3


def test_collapsed_rules_are_accurate():
    # the witnesses' own brute-force rules, pinned by monomials
    xi, w = W.collapsed_tet_rule(8)
    assert np.sum(w * xi[:, 0] ** 3 * xi[:, 1] ** 2 * xi[:, 2]) == pytest.approx(
        _tet_monomial(3, 2, 1), rel=1e-13)
    xi, w = W.collapsed_prism_rule(8, 6)
    assert np.sum(w * xi[:, 0] ** 4 * xi[:, 1] ** 3 * xi[:, 2] ** 6) == pytest.approx(
        _prism_monomial(4, 3, 6), rel=1e-13)


def test_shape_partition_of_unity_and_nodal():
    for elem, V in (("tet4", REF_TET), ("prism6", REF_PRISM)):
        for r, x in enumerate(V):
            phi, dphi = oracle.shape(elem, x)
            expect = np.zeros(len(V))
            expect[r] = 1.0
            np.testing.assert_allclose(phi, expect, atol=1e-15)
        rng = np.random.default_rng(0)
        for _ in range(5):
            p = rng.uniform(0, 0.3, 3)
            phi, dphi = oracle.shape(elem, p)
            assert phi.sum() == pytest.approx(1.0, abs=1e-15)
            np.testing.assert_allclose(dphi.sum(0), 0, atol=1e-15)
            # linear reproduction: sum_r X_r phi_r(p) = x(p) = p on the reference element
            np.testing.assert_allclose(V.T @ phi, p, atol=1e-15)


# ---------------------------------------------------------------- P1 / P3
def test_reference_tet_closed_forms():
    g = W.load_golden("reference_tet.txt")
    c = soa(REF_TET)
    r1, r4 = oracle.quad_rule("tet4", 1), oracle.quad_rule("tet4", 4)
    for rule in (r1, r4):
        K, F = oracle.integrate("tet4", "scalar", c, rule, uniform=slots_with(c11=1, c22=1, c33=1, d0=1))
        np.testing.assert_allclose(K[0], g["laplace"], rtol=0, atol=1e-15)
        np.testing.assert_allclose(F[0], g["load_d0"][0], rtol=0, atol=1e-16)
    K, _ = oracle.integrate("tet4", "scalar", c, r4, uniform=slots_with(c00=1))
    np.testing.assert_allclose(K[0], g["mass_exact"], atol=1e-16)
    K, _ = oracle.integrate("tet4", "scalar", c, r1, uniform=slots_with(c00=1))
    np.testing.assert_allclose(K[0], g["mass_1pt"], atol=1e-16)
    for rule in (r1, r4):
        K, _ = oracle.integrate("tet4", "scalar", c, rule, uniform=slots_with(c10=1))
        np.testing.assert_allclose(K[0], g["convection_c10"], atol=1e-16)
        K, _ = oracle.integrate("tet4", "scalar", c, rule, uniform=slots_with(c01=1))
        np.testing.assert_allclose(K[0], g["convection_c01"], atol=1e-16)
        _, F = oracle.integrate("tet4", "scalar", c, rule, uniform=slots_with(d1=1))
        np.testing.assert_allclose(F[0], g["load_d1"][0], atol=1e-16)


def test_reference_prism_closed_forms():
    g = W.load_golden("reference_prism.txt")
    c = soa(REF_PRISM)
    rule = oracle.quad_rule("prism6", 6)
    K, F = oracle.integrate("prism6", "scalar", c, rule, uniform=slots_with(c11=1, c22=1, c33=1, d0=1))
    np.testing.assert_allclose(K[0], g["laplace"], atol=1e-15)
    np.testing.assert_allclose(F[0], g["load_d0"][0], atol=1e-16)
    K, _ = oracle.integrate("prism6", "scalar", c, rule, uniform=slots_with(c00=1))
    np.testing.assert_allclose(K[0], g["mass"], atol=1e-16)


# ---------------------------------------------------------------- P2
def _random_affine_tets(n, seed):
    rng = np.random.default_rng(seed)
    X = np.empty((n, 4, 3))
    for e in range(n):
        while True:
            P = rng.uniform(-1, 1, (4, 3))
            vol = np.linalg.det(np.hstack([np.ones((4, 1)), P])) / 6
            if vol > 0.02:
                break
        X[e] = P
    coords = np.ascontiguousarray(X.transpose(1, 2, 0).reshape(12, n))
    return X, coords


def test_affine_tet_all_terms_match_closed_form():
    n = 40
    X, coords = _random_affine_tets(n, 11)
    rng = np.random.default_rng(12)
    coeffs = inputs.cdr_per_element(n, rng)
    K, F = oracle.integrate("tet4", "scalar", coords, oracle.quad_rule("tet4", 4), "element",
                            inputs.ALL_SCALAR_MASK, None, coeffs)
    for e in range(n):
        Kc, Fc = W.tet_closed_form_scalar(X[e], coeffs[:, e])
        np.testing.assert_allclose(K[e], Kc, rtol=0, atol=1e-13 * np.abs(Kc).max())
        np.testing.assert_allclose(F[e], Fc, rtol=0, atol=1e-13 * np.abs(Fc).max())
    # the 1-point rule is exact whenever there is no reaction term
    coeffs[0] = 0.0
    K1, F1 = oracle.integrate("tet4", "scalar", coords, oracle.quad_rule("tet4", 1), "element",
                              inputs.ALL_SCALAR_MASK, None, coeffs)
    for e in range(n):
        Kc, Fc = W.tet_closed_form_scalar(X[e], coeffs[:, e])
        np.testing.assert_allclose(K1[e], Kc, atol=1e-13 * np.abs(Kc).max())
        np.testing.assert_allclose(F1[e], Fc, atol=1e-13 * np.abs(Fc).max())


def test_mesh_tets_match_closed_form():
    wl = inputs.tet_cdr(3, seed=5)
    K, F = oracle.integrate_workload(wl)
    X = wl.mesh.coords.reshape(4, 3, -1)
    for e in range(0, wl.n_elem, 7):
        Kc, Fc = W.tet_closed_form_scalar(X[:, :, e], wl.coeffs[:, e])
        np.testing.assert_allclose(K[e], Kc, atol=1e-12 * np.abs(Kc).max())
        np.testing.assert_allclose(F[e], Fc, atol=1e-12 * np.abs(Fc).max())


def test_per_qp_coefficients_follow_rule_order():
    # a per-point d^0 that is nonzero at one point only picks out that point's
    # weighted shape-function values: F_r = det * w_q * phi_r(xi_q)
    X, coords = _random_affine_tets(3, 21)
    xi, w = oracle.quad_rule("tet4", 4)
    for q in range(4):
        c = np.zeros((4, 3))
        c[q] = 1.0
        _, F = oracle.integrate("tet4", "scalar", coords, (xi, w), "qp", 1 << 16, None, c)
        for e in range(3):
            _, V = W.barycentric_gradients(X[e])
            phi, _ = oracle.shape("tet4", xi[q])
            np.testing.assert_allclose(F[e], 6 * V * w[q] * phi, rtol=1e-14)


# ---------------------------------------------------------------- elasticity
def test_tet_elasticity_closed_form_and_voigt():
    wl = inputs.tet_elasticity(2, seed=9)
    K, F = oracle.integrate_workload(wl)
    X = wl.mesh.coords.reshape(4, 3, -1)
    for e in range(wl.n_elem):
        E, nu = wl.coeffs[0, e], wl.coeffs[1, e]
        Kc, Fc = W.tet_closed_form_elasticity(X[:, :, e], E, nu, wl.coeffs[2:5, e])
        np.testing.assert_allclose(K[e], Kc, atol=1e-12 * np.abs(Kc).max())
        np.testing.assert_allclose(F[e], Fc, atol=1e-13 * np.abs(Fc).max())
    Kv, Fv = oracle.elasticity_voigt("tet4", wl.mesh.coords, oracle.quad_rule("tet4", 1), "element",
                                     31, None, wl.coeffs)
    np.testing.assert_allclose(K, Kv, rtol=0, atol=1e-14 * np.abs(K).max())
    np.testing.assert_allclose(F, Fv, rtol=0, atol=1e-14 * np.abs(F).max())


def test_prism_elasticity_voigt_route():
    wl = inputs.prism_elasticity(2, 2, seed=13)
    K, F = oracle.integrate_workload(wl)
    Kv, Fv = oracle.elasticity_voigt("prism6", wl.mesh.coords, oracle.quad_rule("prism6", 6),
                                     "element", 31, None, wl.coeffs)
    for e in range(wl.n_elem):
        s = np.abs(K[e]).max()
        np.testing.assert_allclose(K[e], Kv[e], rtol=0, atol=1e-14 * s)
        np.testing.assert_allclose(F[e], Fv[e], rtol=0, atol=1e-14 * np.abs(F[e]).max())


# ---------------------------------------------------------------- P4 / P8
def _affine_prism(rng):
    while True:
        B = rng.uniform(-1, 1, (3, 3))
        t = rng.uniform(-0.3, 0.3, 3) + np.array([0, 0, 1.0])
        X = np.vstack([B, B + t])
        tri = np.cross(B[1] - B[0], B[2] - B[0])
        if tri @ t > 0.05:
            return X


def test_affine_prism_matches_brute_force():
    rng = np.random.default_rng(31)
    xi_b, w_b = W.collapsed_prism_rule(10, 6)
    rule = oracle.quad_rule("prism6", 6)
    for _ in range(5):
        X = _affine_prism(rng)
        sl = inputs.cdr_per_element(1, rng)[:, 0]
        K, F = oracle.integrate("prism6", "scalar", soa(X), rule, uniform=sl)
        Kb, Fb, det = W.prism_brute_scalar(X, sl, xi_b, w_b)
        np.testing.assert_allclose(K[0], Kb, atol=1e-13 * np.abs(Kb).max())
        np.testing.assert_allclose(F[0], Fb, atol=1e-13 * np.abs(Fb).max())


def test_tet_cube_brute_force():
    # 1x1x1 cube -> 6 tets, all terms, collapsed 12^3 Gauss rule in NumPy
    wl = inputs.tet_cdr(1, seed=3)
    K, F = oracle.integrate_workload(wl)
    xi_b, w_b = W.collapsed_tet_rule(12)
    X = wl.mesh.coords.reshape(4, 3, -1)
    for e in range(6):
        Xe = X[:, :, e]
        # tet shape functions via barycentric maps of the collapsed points
        phi = np.stack([1 - xi_b.sum(1), xi_b[:, 0], xi_b[:, 1], xi_b[:, 2]], 1)
        G, V = W.barycentric_gradients(Xe)
        Phi = np.concatenate([phi[:, :, None], np.broadcast_to(G, (len(w_b), 4, 3))], 2)
        c = wl.coeffs[:16, e].reshape(4, 4)
        d = wl.coeffs[16:, e]
        vol = 6 * V * w_b
        Kb = np.einsum("m,mra,ab,msb->rs", vol, Phi, c, Phi)
        Fb = np.einsum("m,mra,a->r", vol, Phi, d)
        np.testing.assert_allclose(K[e], Kb, atol=1e-13 * np.abs(Kb).max())
        np.testing.assert_allclose(F[e], Fb, atol=1e-13 * np.abs(Fb).max())


def test_nonaffine_prism_high_order_and_convergence():
    rng = np.random.default_rng(41)
    xi_b, w_b = W.collapsed_prism_rule(14, 10)
    sl = inputs.cdr_per_element(1, rng)[:, 0]
    gaps = []
    for amp in (0.2, 0.05, 0.0125):
        X = REF_PRISM + amp * rng.uniform(-1, 1, (6, 3))
        # the oracle with a caller-supplied high-order rule vs the NumPy brute force
        K_hi, F_hi = oracle.integrate("prism6", "scalar", soa(X), (xi_b, w_b), uniform=sl)
        Kb, Fb, det = W.prism_brute_scalar(X, sl, xi_b, w_b)
        assert det.min() > 0
        np.testing.assert_allclose(K_hi[0], Kb, atol=1e-13 * np.abs(Kb).max())
        np.testing.assert_allclose(F_hi[0], Fb, atol=1e-13 * np.abs(Fb).max())
        K6, _ = oracle.integrate("prism6", "scalar", soa(X), oracle.quad_rule("prism6", 6), uniform=sl)
        gaps.append(np.abs(K6[0] - Kb).max() / np.abs(Kb).max())
    # the 6-point result converges to the exact integral as the distortion vanishes
    assert gaps[0] > gaps[1] > gaps[2]
    assert gaps[2] < 1e-4


# ---------------------------------------------------------------- P5 invariants
def _diffusion_only(n, rng):
    c = inputs.cdr_per_element(n, rng)
    keep = [5, 6, 7, 9, 10, 11, 13, 14, 15]
    out = np.zeros_like(c)
    out[keep] = c[keep]
    return out


@pytest.mark.parametrize("elem", ["tet4", "prism6"])
def test_pure_diffusion_zero_row_sums_and_symmetry(elem):
    rng = np.random.default_rng(51)
    mesh = inputs.tet_cube(2, rng) if elem == "tet4" else inputs.prism_layers(3, 4, rng)
    c = _diffusion_only(mesh.n_elem, rng)
    nq = 4 if elem == "tet4" else 6
    K, _ = oracle.integrate(elem, "scalar", mesh.coords, oracle.quad_rule(elem, nq), "element",
                            inputs.ALL_SCALAR_MASK, None, c)
    s = np.abs(K).max(axis=(1, 2))
    assert np.all(np.abs(K.sum(axis=2)) <= 1e-14 * s[:, None] * 8)
    assert np.all(np.abs(K.sum(axis=1)) <= 1e-14 * s[:, None] * 8)
    np.testing.assert_allclose(K, np.transpose(K, (0, 2, 1)), rtol=0, atol=1e-15 * s.max() * 8)


def _rigid_modes(X):
    n = X.shape[0]
    modes = []
    for a in range(3):
        u = np.zeros((n, 3))
        u[:, a] = 1.0
        modes.append(u.reshape(-1))
    for a in range(3):
        om = np.zeros(3)
        om[a] = 1.0
        modes.append(np.cross(om, X).reshape(-1))
    return np.array(modes)


@pytest.mark.parametrize("elem", ["tet4", "prism6"])
def test_elasticity_rigid_body_modes_and_rank(elem):
    wl = inputs.tet_elasticity(2, seed=61) if elem == "tet4" else inputs.prism_elasticity(2, 3, seed=61)
    K, _ = oracle.integrate_workload(wl)
    nv = 4 if elem == "tet4" else 6
    X = wl.mesh.coords.reshape(nv, 3, -1)
    for e in range(0, wl.n_elem, 3):
        Ke = K[e]
        s = np.abs(Ke).max()
        for m in _rigid_modes(X[:, :, e].copy()):
            assert np.abs(Ke @ m).max() <= 1e-13 * s * np.abs(m).max() * 4
        ev = np.linalg.eigvalsh(0.5 * (Ke + Ke.T))
        assert ev.min() > -1e-12 * s
        assert np.sum(ev > 1e-9 * s) == 3 * nv - 6


# ---------------------------------------------------------------- P6 volume
@pytest.mark.parametrize("elem", ["tet4", "prism6"])
def test_volume_sums_to_domain(elem):
    mesh = inputs.tet_cube(4, 71) if elem == "tet4" else inputs.prism_layers(5, 6, 71, sliver=True)
    nq = 4 if elem == "tet4" else 6
    _, F = oracle.integrate(elem, "scalar", mesh.coords, oracle.quad_rule(elem, nq),
                            uniform=slots_with(d0=1))
    assert F.sum() == pytest.approx(1.0, rel=1e-13)
    # every element and every point positively oriented (generators' promise)
    xi, w = oracle.quad_rule(elem, nq)
    for q in range(nq):
        wq = np.zeros(nq)
        wq[q] = 1.0
        _, Fq = oracle.integrate(elem, "scalar", mesh.coords, (xi, wq), uniform=slots_with(d0=1))
        assert Fq.sum(axis=1).min() > 0


# ---------------------------------------------------------------- P7 patch test
@pytest.mark.parametrize("elem", ["tet4", "prism6"])
def test_patch_test_linear_field(elem):
    mesh = inputs.tet_cube(3, 81) if elem == "tet4" else inputs.prism_layers(3, 4, 81, sliver=True)
    nq = 4 if elem == "tet4" else 6
    K, _ = oracle.integrate(elem, "scalar", mesh.coords, oracle.quad_rule(elem, nq), uniform=LAPLACE)
    a, b = np.array([0.3, -1.2, 0.7]), 0.4
    u = mesh.nodes @ a + b
    r = np.zeros(len(mesh.nodes))
    for e in range(mesh.n_elem):
        idx = mesh.conn[e]
        r[idx] += K[e] @ u[idx]
    interior = ~mesh.boundary
    assert interior.sum() > 0
    scale = np.abs(K).max() * np.abs(u).max()
    assert np.abs(r[interior]).max() <= 1e-12 * scale


# ---------------------------------------------------------------- P9 metamorphic
def _rot(rng):
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    return Q


@pytest.mark.parametrize("elem", ["tet4", "prism6"])
def test_rigid_motion_and_scaling(elem):
    rng = np.random.default_rng(91)
    mesh = inputs.tet_cube(2, rng) if elem == "tet4" else inputs.prism_layers(2, 2, rng)
    nv = 4 if elem == "tet4" else 6
    nq = 4 if elem == "tet4" else 6
    rule = oracle.quad_rule(elem, nq)
    u = slots_with(c11=1, c22=1, c33=1, d0=1)
    K0, F0 = oracle.integrate(elem, "scalar", mesh.coords, rule, uniform=u)
    X = mesh.coords.reshape(nv, 3, -1)
    Q = _rot(rng)
    t = rng.uniform(-5, 5, 3)
    Xm = np.einsum("ij,vjn->vin", Q, X) + t[None, :, None]
    K1, F1 = oracle.integrate(elem, "scalar", Xm.reshape(nv * 3, -1), rule, uniform=u)
    np.testing.assert_allclose(K1, K0, atol=1e-12 * np.abs(K0).max())
    np.testing.assert_allclose(F1, F0, atol=1e-12 * np.abs(F0).max())
    s = 2.5
    K2, F2 = oracle.integrate(elem, "scalar", (s * X).reshape(nv * 3, -1), rule, uniform=u)
    np.testing.assert_allclose(K2, s * K0, atol=1e-12 * s * np.abs(K0).max())
    np.testing.assert_allclose(F2, s ** 3 * F0, atol=1e-12 * s ** 3 * np.abs(F0).max())


def test_vertex_relabelling_permutes_matrices():
    rng = np.random.default_rng(101)
    # tet: even permutation keeps orientation
    wl = inputs.tet_cdr(1, seed=7)
    perm = [1, 2, 0, 3]
    X = wl.mesh.coords.reshape(4, 3, -1)
    Xp = X[perm]
    K1, F1 = oracle.integrate("tet4", "scalar", Xp.reshape(12, -1), oracle.quad_rule("tet4", 1),
                              "element", inputs.ALL_SCALAR_MASK, None, wl.coeffs)
    K0b, F0b = oracle.integrate("tet4", "scalar", wl.mesh.coords, oracle.quad_rule("tet4", 1),
                                "element", inputs.ALL_SCALAR_MASK, None, wl.coeffs)
    np.testing.assert_allclose(K1, K0b[:, perm][:, :, perm], atol=1e-13 * np.abs(K0b).max())
    np.testing.assert_allclose(F1, F0b[:, perm], atol=1e-13 * np.abs(F0b).max())
    # prism: rotate the triangle (0->1->2) on both levels; and swap levels with
    # a triangle reflection (orientation kept)
    m = inputs.prism_layers(2, 2, rng)
    c = inputs.cdr_per_element(m.n_elem, rng)
    X = m.coords.reshape(6, 3, -1)
    rule = oracle.quad_rule("prism6", 6)
    K0, F0 = oracle.integrate("prism6", "scalar", m.coords, rule, "element", inputs.ALL_SCALAR_MASK,
                              None, c)
    for perm in ([1, 2, 0, 4, 5, 3], [3, 5, 4, 0, 2, 1]):
        K1, F1 = oracle.integrate("prism6", "scalar", X[perm].reshape(18, -1), rule, "element",
                                  inputs.ALL_SCALAR_MASK, None, c)
        # the 6-point rule is symmetric under these maps, so results permute
        np.testing.assert_allclose(K1, K0[:, perm][:, :, perm], atol=1e-12 * np.abs(K0).max())
        np.testing.assert_allclose(F1, F0[:, perm], atol=1e-12 * np.abs(F0).max())


def test_element_permutation_is_bit_exact():
    wl = inputs.prism_cdr_qp(3, 2, seed=111)
    K0, F0 = oracle.integrate_workload(wl, threads=3)
    p = np.random.default_rng(112).permutation(wl.n_elem)
    K1, F1 = oracle.integrate("prism6", "scalar", wl.mesh.coords[:, p], oracle.quad_rule("prism6", 6),
                              "qp", wl.mask, None, wl.coeffs[:, p], threads=2)
    assert np.array_equal(K1, K0[p]) and np.array_equal(F1, F0[p])


def test_sentinel_element_id():
    # d^0 = element id: F_r(e) = e * V_e / 4 for every tet
    mesh = inputs.tet_cube(2, 121)
    n = mesh.n_elem
    c = np.arange(n, dtype=np.float64)[None, :]
    _, F = oracle.integrate("tet4", "scalar", mesh.coords, oracle.quad_rule("tet4", 1), "element",
                            1 << 16, None, c)
    X = mesh.coords.reshape(4, 3, -1)
    for e in range(n):
        _, V = W.barycentric_gradients(X[:, :, e])
        np.testing.assert_allclose(F[e], e * V / 4, rtol=1e-13, atol=1e-300)


def test_inverted_element_uses_signed_determinant():
    # reading of vol = det J * w with det J signed: swapping two vertices of a
    # tet flips the orientation, so every term changes sign (after relabelling)
    wl = inputs.tet_cdr(1, seed=131)
    X = wl.mesh.coords.reshape(4, 3, -1)
    perm = [1, 0, 2, 3]
    rule = oracle.quad_rule("tet4", 4)
    K0, F0 = oracle.integrate("tet4", "scalar", wl.mesh.coords, rule, "element",
                              inputs.ALL_SCALAR_MASK, None, wl.coeffs)
    K1, F1 = oracle.integrate("tet4", "scalar", X[perm].reshape(12, -1), rule, "element",
                              inputs.ALL_SCALAR_MASK, None, wl.coeffs)
    np.testing.assert_allclose(K1, -K0[:, perm][:, :, perm], atol=1e-13 * np.abs(K0).max())
    np.testing.assert_allclose(F1, -F0[:, perm], atol=1e-13 * np.abs(F0).max())


def test_sliver_prisms_match_extended_precision():
    # thin (aspect ~1e3) non-affine prisms with per-point coefficients: the
    # FP64 oracle stays within 1e-14 (relative Frobenius) of a long-double
    # evaluation of the same quadrature sum
    wl = inputs.prism_cdr_qp(9, 8, seed=3)
    K, F = oracle.integrate_workload(wl)
    xi, w = oracle.quad_rule("prism6", 6)
    X = wl.mesh.coords.reshape(6, 3, -1)
    n_col = 2 * 9 * 9
    sliver = range(4 * n_col, 5 * n_col, 17)   # layer L // 2
    for e in list(sliver) + [3, 100]:
        cq = wl.coeffs[:, e].reshape(20, 6).T
        Kx, Fx = W.prism_extended(X[:, :, e], cq, xi, w)
        ek = np.sqrt(((K[e] - Kx) ** 2).sum() / (Kx ** 2).sum())
        ef = np.sqrt(((F[e] - Fx) ** 2).sum() / (Fx ** 2).sum())
        assert ek < 1e-14 and ef < 1e-14, (e, float(ek), float(ef))


# ---------------------------------------------------------------- coefficient functions
def test_function_mode_matches_values_at_the_points():
    # the function mode evaluates the same fields that smooth_cdr_per_qp
    # samples at the 6-point rule's points: same parameters -> same matrices
    seed = 17
    rng = np.random.default_rng(seed)
    mesh = inputs.prism_layers(3, 4, rng)
    vals = inputs.smooth_cdr_per_qp(mesh.coords, inputs.prism_sample_weights(), rng)
    rng2 = np.random.default_rng(seed)
    inputs.prism_layers(3, 4, rng2)
    params = inputs.smooth_cdr_params(rng2)
    rule = oracle.quad_rule("prism6", 6)
    Kv, Fv = oracle.integrate("prism6", "scalar", mesh.coords, rule, "qp", inputs.ALL_SCALAR_MASK,
                              None, vals)
    Kf, Ff = oracle.integrate("prism6", "scalar", mesh.coords, rule, "function",
                              inputs.ALL_SCALAR_MASK, None, params)
    np.testing.assert_allclose(Kf, Kv, rtol=0, atol=1e-12 * np.abs(Kv).max())
    np.testing.assert_allclose(Ff, Fv, rtol=0, atol=1e-12 * np.abs(Fv).max())


def test_function_mode_constant_fields_reduce_to_uniform():
    # beta = 0 and no SPD transform: every slot is its alpha everywhere
    rng = np.random.default_rng(19)
    mesh = inputs.tet_cube(2, rng)
    p = np.zeros(122)
    alpha = inputs.cdr_per_element(1, rng)[:, 0]
    for k in range(20):
        p[6 * k] = alpha[k]
        p[6 * k + 2: 6 * k + 5] = (1, 2, 3)
        p[6 * k + 5] = 0.3
    rule = oracle.quad_rule("tet4", 4)
    Ku, Fu = oracle.integrate("tet4", "scalar", mesh.coords, rule, uniform=alpha)
    Kf, Ff = oracle.integrate("tet4", "scalar", mesh.coords, rule, "function",
                              inputs.ALL_SCALAR_MASK, None, p)
    assert np.array_equal(Kf, Ku) and np.array_equal(Ff, Fu)
    # slots outside the mask take their uniform values
    Km, Fm = oracle.integrate("tet4", "scalar", mesh.coords, rule, "function", 1 << 16, alpha, p)
    assert np.array_equal(Km, Ku) and np.array_equal(Fm, Fu)


def test_function_mode_spd_transform():
    # with the transform the diffusion block is A A^T + s I: a field with
    # A = a constant lower-triangular matrix gives c^{i;j} = (A A^T + s I)_ij
    rng = np.random.default_rng(23)
    mesh = inputs.tet_cube(2, rng)
    A = np.tril(rng.uniform(-1, 1, (3, 3)))
    p = np.zeros(122)
    for i in range(3):
        for j in range(3):
            p[6 * (4 * (i + 1) + 1 + j)] = A[i, j]
    p[120], p[121] = 0.25, 1.0
    u = np.zeros(20)
    C = A @ A.T + 0.25 * np.eye(3)
    for i in range(3):
        for j in range(3):
            u[4 * (i + 1) + 1 + j] = C[i, j]
    rule = oracle.quad_rule("tet4", 4)
    Ku, _ = oracle.integrate("tet4", "scalar", mesh.coords, rule, uniform=u)
    Kf, _ = oracle.integrate("tet4", "scalar", mesh.coords, rule, "function",
                             inputs.ALL_SCALAR_MASK, None, p)
    np.testing.assert_allclose(Kf, Ku, rtol=0, atol=1e-15 * np.abs(Ku).max())
