"""Python access to the plain FP64 CPU oracle (fe_oracle.c).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the
benchmark's CPU-baseline leg import this package. It never touches the GPU and
shares nothing with the GPU library; the inputs it is given come from the
seeded generators.

The element integrals are in fe_oracle.c (the quadrature sums that define
K and F, eqs. "sm_local" and "lv_local" with the rule of eq. "quadrature",
written out term by term); the functions here marshal their arguments. Two small pieces
are plain NumPy beside it: the scatter of element matrices into the
assembled operator (apply_assembled, assemble_dense) and det J at the rule points
(jacobian_dets, count_inverted).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fe_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TET4, PRISM6 = 0, 1
SCALAR, ELASTICITY, VECTOR = 0, 1, 2
UNIFORM, PER_ELEMENT, PER_QP, FUNCTION = 0, 1, 2, 3

_ELEM = {"tet4": TET4, "prism6": PRISM6}
_KIND = {"scalar": SCALAR, "elasticity": ELASTICITY, "vector": VECTOR}
_MODE = {"uniform": UNIFORM, "element": PER_ELEMENT, "qp": PER_QP, "function": FUNCTION}


def build(force: bool = True) -> str:
    """Compile fe_oracle.c into liboracle.so with gcc (strict IEEE FP64)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", _LIB + ".tmp", _SRC, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_quad_rule.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.oracle_quad_rule.restype = ctypes.c_int
        L.oracle_shape.argtypes = [ctypes.c_int, dp, dp, dp]
        L.oracle_shape.restype = ctypes.c_int
        L.oracle_integrate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint, dp,
                                       ctypes.c_int64, dp, ctypes.c_int64, dp, ctypes.c_int64,
                                       ctypes.c_int, dp, dp, dp, dp, ctypes.c_int]
        L.oracle_integrate.restype = ctypes.c_int
        L.oracle_elasticity_voigt.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint, dp,
                                              ctypes.c_int64, dp, ctypes.c_int64, dp,
                                              ctypes.c_int64, ctypes.c_int, dp, dp, dp, dp]
        L.oracle_elasticity_voigt.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def quad_rule(elem: str, n_q: int):
    """The oracle's own copy of the built-in rules: (xi (n_q,3), w (n_q,))."""
    xi = np.zeros((n_q, 3))
    w = np.zeros(n_q)
    rc = lib().oracle_quad_rule(_ELEM[elem], n_q, _p(xi), _p(w))
    if rc != 0:
        raise ValueError(f"no built-in oracle rule for {elem} with {n_q} points")
    return xi, w


def shape(elem: str, xi):
    """Reference shape functions and their reference derivatives at one point."""
    ns = 4 if elem == "tet4" else 6
    x = np.ascontiguousarray(xi, dtype=np.float64)
    phi = np.zeros(ns)
    dphi = np.zeros((ns, 3))
    lib().oracle_shape(_ELEM[elem], _p(x), _p(phi), _p(dphi))
    return phi, dphi


def n_dof(elem: str, kind: str) -> int:
    return (4 if elem == "tet4" else 6) * (1 if kind == "scalar" else 3)


def integrate(elem: str, kind: str, coords, rule, coef_mode: str = "uniform", mask: int = 0,
              uniform=None, coeffs=None, threads: int = 1):
    """Full element matrices K (n, N, N) and vectors F (n, N), float64.

    ``coords`` is the SoA (n_vert*3, n) array; ``coeffs`` the compact
    coefficient array (float64, or float32 promoted exactly); ``rule`` a pair
    (xi (n_q,3), w (n_q,)). For kind "vector" (156 slots) ``mask`` has one
    bit per block (bits 0..15: the 3x3 blocks c^{a;b}, bits 16..19: the
    3-vectors d^a) and absent blocks are zero."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    n = coords.shape[1]
    N = n_dof(elem, kind)
    xi = np.ascontiguousarray(rule[0], dtype=np.float64).reshape(-1, 3)
    w = np.ascontiguousarray(rule[1], dtype=np.float64).reshape(-1)
    n_slots = {"scalar": 20, "elasticity": 5, "vector": 20}[kind]
    u = np.zeros(20)
    if uniform is not None:
        u[: len(uniform)] = np.asarray(uniform, dtype=np.float64)
    c = None
    ldc = n
    if coef_mode == "function":
        c = np.ascontiguousarray(coeffs, dtype=np.float64).reshape(-1)
        if c.size != 122:
            raise ValueError("a coefficient function takes 122 parameters")
    elif coef_mode != "uniform" and mask:
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        ldc = c.shape[1]
    K = np.empty((n, N, N))
    F = np.empty((n, N))
    rc = lib().oracle_integrate(_ELEM[elem], _KIND[kind], _MODE[coef_mode],
                                mask & ((1 << n_slots) - 1), _p(u), n, _p(coords), n, _p(c),
                                ldc, xi.shape[0], _p(xi), _p(w), _p(K), _p(F), int(threads))
    if rc != 0:
        raise RuntimeError(f"oracle_integrate failed with status {rc}")
    return K, F


def elasticity_voigt(elem: str, coords, rule, coef_mode: str = "uniform", mask: int = 0,
                     uniform=None, coeffs=None):
    """Second, independent elasticity route (B^T D B in Voigt form)."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    n = coords.shape[1]
    N = n_dof(elem, "elasticity")
    xi = np.ascontiguousarray(rule[0], dtype=np.float64).reshape(-1, 3)
    w = np.ascontiguousarray(rule[1], dtype=np.float64).reshape(-1)
    u = np.zeros(20)
    if uniform is not None:
        u[: len(uniform)] = np.asarray(uniform, dtype=np.float64)
    c = None
    ldc = n
    if coef_mode != "uniform" and mask:
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        ldc = c.shape[1]
    K = np.empty((n, N, N))
    F = np.empty((n, N))
    rc = lib().oracle_elasticity_voigt(_ELEM[elem], _MODE[coef_mode], mask & 31, _p(u), n,
                                       _p(coords), n, _p(c), ldc, xi.shape[0], _p(xi), _p(w),
                                       _p(K), _p(F))
    if rc != 0:
        raise RuntimeError(f"oracle_elasticity_voigt failed with status {rc}")
    return K, F


def integrate_workload(wl, threads: int = 1, elements=None):
    """Run the oracle on a generated workload (optionally on a subset of
    element indices), with the oracle's own copy of the workload's rule."""
    coords = wl.mesh.coords
    coeffs = wl.coeffs
    if elements is not None:
        idx = np.asarray(elements)
        coords = coords[:, idx]
        if coeffs is not None and wl.coef_mode != "function":
            coeffs = coeffs[:, idx]
    return integrate(wl.elem, wl.kind, coords, quad_rule(wl.elem, wl.n_q), wl.coef_mode, wl.mask,
                     wl.uniform, coeffs, threads)


def apply_assembled(elem: str, kind: str, nodes, conn, rule, coef_mode: str = "uniform",
                    mask: int = 0, uniform=None, coeffs=None, x=None, threads: int = 1):
    """The assembled operator applied to a nodal vector, and the assembled
    load vector, from the element matrices (Sec. 3.2: the global system is
    the sum of the element contributions at their nodes):

        y = sum_e P_e^T K^e P_e x,    b = sum_e P_e^T F^e

    ``nodes`` (n_nodes, 3), ``conn`` (n_elem, n_vert) node ids; ``x`` (n_nodes *
    n_comp,) node-major (node * n_comp + component). K^e, F^e come from
    ``integrate`` on the gathered coordinates; the scatter is numpy's add.at.
    Returns (y, b), float64."""
    nodes = np.asarray(nodes, dtype=np.float64)
    conn = np.asarray(conn, dtype=np.int64)
    n, nv = conn.shape
    nc = 1 if kind == "scalar" else 3
    coords = np.ascontiguousarray(nodes[conn].transpose(1, 2, 0).reshape(nv * 3, n))
    K, F = integrate(elem, kind, coords, rule, coef_mode, mask, uniform, coeffs, threads)
    dof = (conn[:, :, None] * nc + np.arange(nc)[None, None, :]).reshape(n, nv * nc)
    x = np.asarray(x, dtype=np.float64)
    ye = np.einsum("ers,es->er", K, x[dof])
    y = np.zeros(nodes.shape[0] * nc)
    b = np.zeros(nodes.shape[0] * nc)
    np.add.at(y, dof.ravel(), ye.ravel())
    np.add.at(b, dof.ravel(), F.ravel())
    return y, b


def assemble_dense(elem: str, kind: str, nodes, conn, rule, coef_mode: str = "uniform",
                   mask: int = 0, uniform=None, coeffs=None, threads: int = 1):
    """The assembled global matrix and load vector, dense (small meshes
    only), from the element matrices (Sec. 3.2: the sum of the element
    contributions at their nodes):

        A = sum_e P_e^T K^e P_e,    b = sum_e P_e^T F^e

    with unknowns node-major (node * n_comp + component); the scatter is
    numpy's add.at. Returns (A (n_dof, n_dof), b (n_dof,)), float64."""
    nodes = np.asarray(nodes, dtype=np.float64)
    conn = np.asarray(conn, dtype=np.int64)
    n, nv = conn.shape
    nc = 1 if kind == "scalar" else 3
    coords = np.ascontiguousarray(nodes[conn].transpose(1, 2, 0).reshape(nv * 3, n))
    K, F = integrate(elem, kind, coords, rule, coef_mode, mask, uniform, coeffs, threads)
    dof = (conn[:, :, None] * nc + np.arange(nc)[None, None, :]).reshape(n, nv * nc)
    nd = nodes.shape[0] * nc
    A = np.zeros((nd, nd))
    b = np.zeros(nd)
    np.add.at(A, (dof[:, :, None], dof[:, None, :]), K)
    np.add.at(b, dof, F)
    return A, b


def jacobian_dets(elem: str, coords, rule):
    """det J of the reference-to-physical map at every rule point, (n, n_q).

    J_ik = sum_r X_{r,i} dphi_r/dxi_k (Sec. 2.2, the change of variables of
    the reference element); the determinant is numpy's."""
    coords = np.asarray(coords, dtype=np.float64)
    nv = 4 if elem == "tet4" else 6
    n = coords.shape[1]
    X = coords.reshape(nv, 3, n).transpose(2, 0, 1)          # (n, vertex, i)
    xi = np.asarray(rule[0], dtype=np.float64).reshape(-1, 3)
    dets = np.empty((n, xi.shape[0]))
    for q in range(xi.shape[0]):
        _, dphi = shape(elem, xi[q])
        J = np.einsum("eri,rk->eik", X, dphi)
        dets[:, q] = np.linalg.det(J)
    return dets


def count_inverted(elem: str, coords, rule) -> int:
    """Number of elements whose det J is not positive at some rule point
    (the signed-determinant convention integrates them as written)."""
    d = jacobian_dets(elem, coords, rule)
    return int(np.count_nonzero((~(d > 0.0)).any(axis=1)))
