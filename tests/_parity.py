"""Helpers for the GPU-vs-oracle parity tests: run a generated workload
through the C ABI and through the oracle, and compare per element."""
from __future__ import annotations

import dataclasses
import functools
import os

import numpy as np

import oracle
from paper_1504_01023_amd import fe, inputs

# Relative Frobenius error bounds per element: FP64 path against the FP64
# oracle, and the FP32 bulk tier against the FP64 oracle run on the FP32
# coefficients promoted exactly (so only the arithmetic differs).
TOL = {"fp64": 1e-12, "fp32": 2e-5}
ORACLE_THREADS = max(1, min(16, os.cpu_count() or 1))


def n_dof(wl) -> int:
    return oracle.n_dof(wl.elem, wl.kind)


def oracle_coeffs(wl, precision):
    if wl.coeffs is None:
        return None
    if wl.coef_mode == "function":
        return wl.coeffs  # FP64 parameters in both tiers
    if precision == "fp32":
        return wl.coeffs.astype(np.float32).astype(np.float64)
    return wl.coeffs


def oracle_run(wl, precision="fp64", elements=None, rule=None):
    coords, coeffs = wl.mesh.coords, oracle_coeffs(wl, precision)
    if elements is not None:
        coords = np.ascontiguousarray(coords[:, elements])
        if coeffs is not None and wl.coef_mode != "function":
            coeffs = np.ascontiguousarray(coeffs[:, elements])
    r = rule if rule is not None else oracle.quad_rule(wl.elem, wl.n_q)
    return oracle.integrate(wl.elem, wl.kind, coords, r, wl.coef_mode, wl.mask, wl.uniform,
                            coeffs, ORACLE_THREADS)


def gpu_raw(wl, precision="fp64", variant=None, rule=None, device="cuda"):
    import torch
    dw = fe.to_device(wl, precision, device=device, rule=rule)
    K, F = fe.integrate(dw.problem, wl.elem, dw.coords, dw.coeffs, dw.rule, variant=variant)
    torch.cuda.synchronize()
    return K.cpu().numpy(), F.cpu().numpy()


def to_full(Kraw, Fraw, wl):
    N = n_dof(wl)
    K = fe.unpack_full(Kraw.astype(np.float64), N, wl.k_format == "packed")
    return K, np.ascontiguousarray(Fraw.astype(np.float64).T)


def rel_errors(Kg, Fg, Ko, Fo):
    """Per-element relative Frobenius errors of K and F (an all-zero
    reference F is compared in absolute terms against the scale of K)."""
    dk = np.sqrt(((Kg - Ko) ** 2).sum(axis=(1, 2)))
    nk = np.sqrt((Ko ** 2).sum(axis=(1, 2)))
    df = np.sqrt(((Fg - Fo) ** 2).sum(axis=1))
    nf = np.sqrt((Fo ** 2).sum(axis=1))
    ek = dk / np.where(nk > 0, nk, 1.0)
    ef = df / np.where(nf > 0, nf, np.where(nk > 0, nk, 1.0))
    return ek, ef


def assert_parity(wl, precision, Kraw, Fraw, elements=None, tol=None):
    tol = TOL[precision] if tol is None else tol
    Kg, Fg = to_full(Kraw, Fraw, wl)
    if elements is not None:
        Kg, Fg = Kg[elements], Fg[elements]
    Ko, Fo = oracle_run(wl, precision, elements)
    assert np.all(np.isfinite(Kg)) and np.all(np.isfinite(Fg))
    ek, ef = rel_errors(Kg, Fg, Ko, Fo)
    assert ek.max() <= tol, f"K rel err {ek.max():.3e} at element {int(ek.argmax())}"
    assert ef.max() <= tol, f"F rel err {ef.max():.3e} at element {int(ef.argmax())}"
    return float(ek.max()), float(ef.max())


# Small workloads spanning several workgroups and a ragged tail.
SMALL = {
    "tet_poisson": lambda: inputs.tet_poisson(8, seed=1),
    "tet_poisson_qp": lambda: inputs.tet_poisson_qp_rhs(7, seed=11),
    "tet_cdr": lambda: inputs.tet_cdr(7, seed=2),
    "prism_cdr_qp": lambda: inputs.prism_cdr_qp(9, 8, seed=3),
    "prism_cdr": lambda: inputs.prism_cdr_element(9, 7, seed=13),
    "tet_elasticity": lambda: inputs.tet_elasticity(7, seed=4),
    "prism_elasticity": lambda: inputs.prism_elasticity(6, 6, seed=14),
    "tet_cdr_fn": lambda: inputs.tet_cdr_fn(6, seed=15),
    "prism_cdr_fn": lambda: inputs.prism_cdr_fn(8, 6, seed=16),
    "prism_poisson_qp": lambda: inputs.prism_poisson_qp_rhs(8, 5, seed=19),
    "tet_vector": lambda: inputs.tet_vector(6, seed=17),
    "prism_vector": lambda: inputs.prism_vector(7, 5, seed=18),
    "prism_elasticity_qp": lambda: _elasticity_per_point(inputs.prism_elasticity(5, 4, seed=20)),
}


def _elasticity_per_point(wl):
    """The same mesh with E, nu, f varying over the points of the rule
    (rows j * n_q + q): the element values scaled by 1 + 0.1 (q / n_q) per
    point, nu kept below 0.45 + 0.045."""
    n_q = 6
    c = wl.coeffs
    rows = []
    for j in range(c.shape[0]):
        for q in range(n_q):
            rows.append(c[j] * (1.0 + 0.1 * q / n_q))
    return dataclasses.replace(wl, name="prism_elasticity_qp", n_q=n_q, coef_mode="qp",
                               coeffs=np.ascontiguousarray(np.array(rows)))


@functools.lru_cache(maxsize=None)
def small(name):
    return SMALL[name]()


def apply_reference(wl, precision, x):
    """Oracle side of the matrix-free tests: the assembled y = A x and load b
    (from the oracle's element matrices), and the row-wise magnitudes
    |A| |x| and sum |F| that scale their rounding errors."""
    coeffs = oracle_coeffs(wl, precision)
    r = oracle.quad_rule(wl.elem, wl.n_q)
    y, b = oracle.apply_assembled(wl.elem, wl.kind, wl.mesh.nodes, wl.mesh.conn, r, wl.coef_mode,
                                  wl.mask, wl.uniform, coeffs, x)
    K, F = oracle.integrate(wl.elem, wl.kind, wl.mesh.coords, r, wl.coef_mode, wl.mask,
                            wl.uniform, coeffs, ORACLE_THREADS)
    nc = 1 if wl.kind == "scalar" else 3
    conn = wl.mesh.conn
    n, nv = conn.shape
    dof = (conn[:, :, None] * nc + np.arange(nc)[None, None, :]).reshape(n, nv * nc)
    yabs = np.zeros_like(y)
    babs = np.zeros_like(b)
    np.add.at(yabs, dof.ravel(), np.einsum("ers,es->er", np.abs(K), np.abs(x[dof])).ravel())
    np.add.at(babs, dof.ravel(), np.abs(F).ravel())
    return y, b, yabs, babs


def assembly_reference(wl, precision):
    """Oracle side of the CSR assembly tests: the dense assembled matrix and
    load vector, and the entry-wise sums of |K^e| and |F^e| that scale their
    rounding errors."""
    coeffs = oracle_coeffs(wl, precision)
    r = oracle.quad_rule(wl.elem, wl.n_q)
    A, b = oracle.assemble_dense(wl.elem, wl.kind, wl.mesh.nodes, wl.mesh.conn, r, wl.coef_mode,
                                 wl.mask, wl.uniform, coeffs)
    K, F = oracle.integrate(wl.elem, wl.kind, wl.mesh.coords, r, wl.coef_mode, wl.mask,
                            wl.uniform, coeffs, ORACLE_THREADS)
    nc = 1 if wl.kind == "scalar" else 3
    conn = wl.mesh.conn
    n, nv = conn.shape
    dof = (conn[:, :, None] * nc + np.arange(nc)[None, None, :]).reshape(n, nv * nc)
    Aabs = np.zeros_like(A)
    babs = np.zeros_like(b)
    np.add.at(Aabs, (dof[:, :, None], dof[:, None, :]), np.abs(K))
    np.add.at(babs, dof, np.abs(F))
    return A, b, Aabs, babs
