"""Pins of the oracle's assembled operator application (y = sum_e P_e^T K^e
P_e x) against what the mathematics fixes: the 7-point stencil of the Kuhn
triangulation, constants and linear fields in the kernel of diffusion,
the mass of the whole domain, and the adjoint of convection. CPU only."""
import numpy as np
import pytest

import oracle
from paper_1504_01023_amd import inputs

LAPLACE = np.zeros(20)
LAPLACE[[5, 10, 15]] = 1.0


def _apply(mesh, kind, rule, mode, mask, uniform, coeffs, x):
    return oracle.apply_assembled(mesh.elem, kind, mesh.nodes, mesh.conn, rule, mode, mask,
                                  uniform, coeffs, x)


def test_kuhn_laplacian_is_the_seven_point_stencil():
    # P1 elements on the Kuhn (Freudenthal) subdivision of a uniform grid give
    # the 7-point finite-difference Laplacian scaled by h at every interior
    # node (the face-diagonal couplings cancel)
    N = 5
    mesh = inputs.tet_cube(N, 1, jitter=0.0)
    h = 1.0 / N
    x = np.random.default_rng(2).standard_normal(mesh.nodes.shape[0])
    y, _ = _apply(mesh, "scalar", oracle.quad_rule("tet4", 1), "uniform", 0, LAPLACE, None, x)
    n1 = N + 1
    X = x.reshape(n1, n1, n1)     # [k, j, i]
    Y = y.reshape(n1, n1, n1)
    c = X[1:-1, 1:-1, 1:-1]
    st = 6 * c - X[2:, 1:-1, 1:-1] - X[:-2, 1:-1, 1:-1] - X[1:-1, 2:, 1:-1] - X[1:-1, :-2, 1:-1] \
        - X[1:-1, 1:-1, 2:] - X[1:-1, 1:-1, :-2]
    np.testing.assert_allclose(Y[1:-1, 1:-1, 1:-1], h * st, rtol=0, atol=1e-13 * np.abs(h * st).max())


@pytest.mark.parametrize("elem", ["tet4", "prism6"])
def test_diffusion_kernel_and_patch_test(elem):
    if elem == "tet4":
        wl = inputs.tet_cdr(3, seed=3)
    else:
        wl = inputs.prism_cdr_element(4, 3, seed=4)
    c = wl.coeffs.copy()
    c[[0, 1, 2, 3, 4, 8, 12]] = 0.0          # diffusion only (per element, SPD)
    rule = oracle.quad_rule(wl.elem, wl.n_q)
    ones = np.ones(wl.mesh.nodes.shape[0])
    y, _ = _apply(wl.mesh, "scalar", rule, "element", inputs.ALL_SCALAR_MASK, None, c, ones)
    assert np.abs(y).max() < 1e-13
    # a linear field is reproduced exactly: residual zero at interior nodes
    # (the identity diffusion; per-element tensors would leave interface jumps)
    lin = wl.mesh.nodes @ np.array([0.3, -1.2, 0.7]) + 0.4
    y, _ = _apply(wl.mesh, "scalar", rule, "uniform", 0, LAPLACE, None, lin)
    inner = ~wl.mesh.boundary
    assert np.abs(y[inner]).max() < 1e-12 * np.abs(lin).max()
    assert np.abs(y[wl.mesh.boundary]).max() > 1e-3


@pytest.mark.parametrize("elem", ["tet4", "prism6"])
def test_mass_and_load_of_the_domain(elem):
    mesh = inputs.tet_cube(3, 5) if elem == "tet4" else inputs.prism_layers(4, 3, 6)
    rule = oracle.quad_rule(elem, 4 if elem == "tet4" else 6)
    u = np.zeros(20)
    u[0] = 1.0      # c^{0;0}
    u[16] = 1.0     # d^0
    ones = np.ones(mesh.nodes.shape[0])
    y, b = _apply(mesh, "scalar", rule, "uniform", 0, u, None, ones)
    assert ones @ y == pytest.approx(1.0, rel=1e-13)
    assert b.sum() == pytest.approx(1.0, rel=1e-13)


def test_convection_adjoint():
    # exchanging c^{i;0} and c^{0;i} transposes the assembled operator
    wl = inputs.tet_cdr(2, seed=7)
    rule = oracle.quad_rule("tet4", 4)
    sw = wl.coeffs.copy()
    for i in range(1, 4):
        sw[4 * i], sw[i] = wl.coeffs[i], wl.coeffs[4 * i]
    rng = np.random.default_rng(8)
    n = wl.mesh.nodes.shape[0]
    x, z = rng.standard_normal(n), rng.standard_normal(n)
    Ax, _ = _apply(wl.mesh, "scalar", rule, "element", inputs.ALL_SCALAR_MASK, None, wl.coeffs, x)
    Bz, _ = _apply(wl.mesh, "scalar", rule, "element", inputs.ALL_SCALAR_MASK, None, sw, z)
    assert z @ Ax == pytest.approx(x @ Bz, rel=1e-12)
    Az, _ = _apply(wl.mesh, "scalar", rule, "element", inputs.ALL_SCALAR_MASK, None, wl.coeffs, z)
    assert abs(z @ Ax - x @ Az) > 1e-6 * abs(z @ Ax)      # not symmetric by itself


def test_elasticity_rigid_modes_in_the_kernel():
    wl = inputs.prism_elasticity(3, 2, seed=9)
    rule = oracle.quad_rule("prism6", 6)
    X = wl.mesh.nodes
    for mode in range(6):
        u = np.zeros((X.shape[0], 3))
        if mode < 3:
            u[:, mode] = 1.0
        else:
            w = np.zeros(3)
            w[mode - 3] = 1.0
            u = np.cross(w, X)
        y, _ = _apply(wl.mesh, "elasticity", rule, "element", inputs.ALL_ELAST_MASK, None,
                      wl.coeffs, u.ravel())
        assert np.abs(y).max() < 1e-11 * np.abs(wl.coeffs[0]).max()


def test_reordering_leaves_the_operator_unchanged():
    # Z-order renumbering of nodes and elements is a relabelling: the
    # assembled operator applied to the relabelled vector is the relabelled
    # result, and every element matrix is bit-identical
    wl = inputs.tet_cdr(3, seed=12)
    mesh, perm = inputs.morton_order(wl.mesh)
    wr = inputs.reordered(wl)
    rule = oracle.quad_rule("tet4", 4)
    x = np.random.default_rng(13).standard_normal(wl.mesh.nodes.shape[0])
    y, _ = _apply(wl.mesh, "scalar", rule, "element", inputs.ALL_SCALAR_MASK, None, wl.coeffs, x)
    # node i of the new numbering is old node node_perm[i]
    node_perm = np.array([np.nonzero((wl.mesh.nodes == p).all(axis=1))[0][0] for p in mesh.nodes])
    yr, _ = _apply(wr.mesh, "scalar", rule, "element", inputs.ALL_SCALAR_MASK, None, wr.coeffs,
                   x[node_perm])
    np.testing.assert_allclose(yr, y[node_perm], rtol=0, atol=1e-13 * np.abs(y).max())
    K0, _ = oracle.integrate_workload(wl)
    K1, _ = oracle.integrate_workload(wr)
    assert np.array_equal(K1, K0[perm])
