"""Test-side witnesses that pin the oracle from outside: closed forms and
brute-force quadrature written with NumPy along routes different from the
oracle's (barycentric coordinates instead of the Jacobian, collapsed Gauss
rules instead of the built-in rules). Nothing here is used by the GPU path."""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name: str) -> dict:
    """Parse a golden fixture: ``[section]`` headers followed by rows of
    rational numbers; ``#`` starts a comment."""
    out, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("["):
                cur = line.strip("[]").strip()
                out[cur] = []
                continue
            out[cur].append([float(Fraction(t)) for t in line.split()])
    return {k: np.array(v) for k, v in out.items()}


def tet_vertices(coords, e):
    return coords.reshape(4, 3, -1)[:, :, e]


def barycentric_gradients(X):
    """Affine tetrahedron with vertex rows X (4, 3): the gradients of the
    barycentric coordinates (4, 3) and the signed volume, from the inverse of
    the 4x4 matrix [[1, x_r, y_r, z_r]] (no Jacobian involved)."""
    T = np.hstack([np.ones((4, 1)), X])
    Tinv = np.linalg.inv(T)          # lambda_r(x) = Tinv[0, r] + Tinv[1:, r] . x
    G = Tinv[1:, :].T                # (4, 3)
    V = np.linalg.det(T) / 6.0
    return G, V


def tet_closed_form_scalar(X, slots):
    """Exact integrals of the scalar weak-form terms over one affine tet.
    slots: the 20 coefficient values (4a+b -> c[a][b], 16+a -> d[a])."""
    G, V = barycentric_gradients(X)
    c = np.asarray(slots[:16]).reshape(4, 4)
    d = np.asarray(slots[16:20])
    C = c[1:, 1:]
    ci0 = c[1:, 0]
    c0i = c[0, 1:]
    one = np.ones(4)
    M = V / 20.0 * (np.outer(one, one) + np.eye(4))
    K = V * G @ C @ G.T + (V / 4) * np.outer(G @ ci0, one) + (V / 4) * np.outer(one, G @ c0i) \
        + c[0, 0] * M
    F = V * G @ d[1:] + (V / 4) * d[0] * one
    return K, F


def tet_closed_form_vector(X, slots):
    """Exact integrals of the general 3-component weak form over one affine
    tet. slots: the 156 values ((4a+b)*9 + 3 alpha + beta -> c^{a;b}_{alpha
    beta}, 144 + 3a + alpha -> d^a_alpha). Unknowns node-major (3r + alpha);
    every (alpha, beta) block is the scalar closed form with that block's
    coefficients."""
    slots = np.asarray(slots, dtype=np.float64)
    K = np.zeros((12, 12))
    F = np.zeros(12)
    for al in range(3):
        for be in range(3):
            sl = np.zeros(20)
            for ab in range(16):
                sl[ab] = slots[ab * 9 + 3 * al + be]
            Kb, _ = tet_closed_form_scalar(X, sl)
            K[al::3, be::3] = Kb
        sl = np.zeros(20)
        for a in range(4):
            sl[16 + a] = slots[144 + 3 * a + al]
        _, Fb = tet_closed_form_scalar(X, sl)
        F[al::3] = Fb
    return K, F


def lame(E, nu):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def tet_closed_form_elasticity(X, E, nu, f):
    """K = V B^T D B with strain-displacement B built from barycentric
    gradients, F_(r, alpha) = V f_alpha / 4."""
    G, V = barycentric_gradients(X)
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] = lam + 2 * mu
    D[3:, 3:] = np.eye(3) * mu
    B = np.zeros((6, 12))
    for r in range(4):
        gx, gy, gz = G[r]
        B[0, 3 * r] = gx
        B[1, 3 * r + 1] = gy
        B[2, 3 * r + 2] = gz
        B[3, 3 * r + 1], B[3, 3 * r + 2] = gz, gy
        B[4, 3 * r], B[4, 3 * r + 2] = gz, gx
        B[5, 3 * r], B[5, 3 * r + 1] = gy, gx
    K = V * B.T @ D @ B
    F = np.tile(np.asarray(f), 4) * V / 4
    return K, F


def gauss_legendre01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1), 0.5 * w


def collapsed_tet_rule(n):
    """Conical-product (Duffy) rule on the reference tet from an n^3 Gauss
    product on the unit cube: xi = u, eta = v (1-u), zeta = w (1-u)(1-v)."""
    x, w = gauss_legendre01(n)
    U, V, W = np.meshgrid(x, x, x, indexing="ij")
    WU, WV, WW = np.meshgrid(w, w, w, indexing="ij")
    xi = np.stack([U, V * (1 - U), W * (1 - U) * (1 - V)], -1).reshape(-1, 3)
    wt = (WU * WV * WW * (1 - U) ** 2 * (1 - V)).reshape(-1)
    return xi, wt


def collapsed_prism_rule(n_tri, n_line):
    """Duffy rule on the unit triangle times Gauss-Legendre on [-1, 1]."""
    x, w = gauss_legendre01(n_tri)
    U, V = np.meshgrid(x, x, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    tx = np.stack([U, V * (1 - U)], -1).reshape(-1, 2)
    tw = (WU * WV * (1 - U)).reshape(-1)
    z, zw = np.polynomial.legendre.leggauss(n_line)
    xi = np.array([[a, b, c] for (a, b) in tx for c in z])
    wt = np.array([p * q for p in tw for q in zw])
    return xi, wt


def prism_shape_np(P):
    """Prism shape functions at points P (m, 3): values (m, 6) and reference
    derivatives (m, 6, 3), written independently of the oracle."""
    xi, eta, z = P[:, 0], P[:, 1], P[:, 2]
    N = np.stack([1 - xi - eta, xi, eta], 1)
    dN = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    lo, hi = (1 - z) / 2, (1 + z) / 2
    phi = np.concatenate([N * lo[:, None], N * hi[:, None]], 1)
    d = np.zeros((P.shape[0], 6, 3))
    for v in range(3):
        d[:, v, 0] = dN[v, 0] * lo
        d[:, v, 1] = dN[v, 1] * lo
        d[:, v, 2] = -N[:, v] / 2
        d[:, v + 3, 0] = dN[v, 0] * hi
        d[:, v + 3, 1] = dN[v, 1] * hi
        d[:, v + 3, 2] = N[:, v] / 2
    return phi, d


def prism_brute_scalar(X, slots, xi, wt):
    """Scalar weak-form integrals over one prism (vertex rows X (6, 3)) with
    constant coefficients, by an arbitrary rule, with NumPy linear algebra
    (np.linalg.solve per point)."""
    phi, dphi = prism_shape_np(xi)
    J = np.einsum("ri,mrk->mik", X, dphi)             # (m, 3, 3) dx_i/dxi_k
    det = np.linalg.det(J)
    # physical gradients: J^T g = dphi_ref  ->  g = solve(J^T, dphi_ref)
    g = np.linalg.solve(np.transpose(J, (0, 2, 1))[:, None, :, :],
                        dphi[:, :, :, None])[..., 0]  # (m, 6, 3)
    Phi = np.concatenate([phi[:, :, None], g], 2)      # (m, 6, 4)
    c = np.asarray(slots[:16]).reshape(4, 4)
    d = np.asarray(slots[16:20])
    vol = det * wt
    K = np.einsum("m,mra,ab,msb->rs", vol, Phi, c, Phi)
    F = np.einsum("m,mra,a->r", vol, Phi, d)
    return K, F, det


def prism_extended(X, coeffs_q, xi, w):
    """Scalar weak-form quadrature sum on one prism in long double (x87
    extended precision), per-point coefficient slots coeffs_q (n_q, 20):
    an accuracy reference for thin (sliver) elements."""
    ld = np.longdouble
    X = np.asarray(X, dtype=ld)
    E = X - X[0]
    K = np.zeros((6, 6), ld)
    F = np.zeros(6, ld)
    for q in range(len(w)):
        phi, dphi = prism_shape_np(np.asarray(xi[q:q + 1], dtype=np.float64))
        phi, dphi = phi[0].astype(ld), dphi[0].astype(ld)
        J = np.einsum("ri,rk->ik", E, dphi)
        c0 = J[1, 1] * J[2, 2] - J[1, 2] * J[2, 1]
        c1 = J[1, 2] * J[2, 0] - J[1, 0] * J[2, 2]
        c2 = J[1, 0] * J[2, 1] - J[1, 1] * J[2, 0]
        det = J[0, 0] * c0 + J[0, 1] * c1 + J[0, 2] * c2
        adj = np.empty((3, 3), ld)
        adj[0, 0], adj[1, 0], adj[2, 0] = c0, c1, c2
        adj[0, 1] = J[0, 2] * J[2, 1] - J[0, 1] * J[2, 2]
        adj[1, 1] = J[0, 0] * J[2, 2] - J[0, 2] * J[2, 0]
        adj[2, 1] = J[0, 1] * J[2, 0] - J[0, 0] * J[2, 1]
        adj[0, 2] = J[0, 1] * J[1, 2] - J[0, 2] * J[1, 1]
        adj[1, 2] = J[0, 2] * J[1, 0] - J[0, 0] * J[1, 2]
        adj[2, 2] = J[0, 0] * J[1, 1] - J[0, 1] * J[1, 0]
        g = dphi @ (adj / det)
        Phi = np.concatenate([phi[:, None], g], 1)
        c = np.asarray(coeffs_q[q], dtype=ld)
        vol = det * ld(w[q])
        K += vol * Phi @ c[:16].reshape(4, 4) @ Phi.T
        F += vol * Phi @ c[16:20]
    return K, F
