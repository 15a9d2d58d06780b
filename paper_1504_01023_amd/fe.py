"""Thin Python binding of libfe.so (the C ABI declared in include/fe.h).

Argument marshalling only: every step of the integration runs in the HIP
kernels of libfe. Device memory and streams come from PyTorch (ROCm build):
tensors are passed by ``data_ptr()`` and work is enqueued on
``torch.cuda.current_stream()`` unless a stream is given. There is no CPU
fallback: if libfe.so is missing or the device is not a GPU, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfe.so")

TET4, PRISM6 = 0, 1
SCALAR_CDR, ELASTICITY, VECTOR_CDR = 0, 1, 2
FP64, FP32_BULK = 0, 1
COEF_UNIFORM, COEF_PER_ELEMENT, COEF_PER_QP, COEF_FUNCTION = 0, 1, 2, 3
FN_PARAMS = 122
K_FULL, K_SYM_PACKED = 0, 1
MAX_QP = 8

ELEM = {"tet4": TET4, "prism6": PRISM6}
KIND = {"scalar": SCALAR_CDR, "elasticity": ELASTICITY, "vector": VECTOR_CDR}
MODE = {"uniform": COEF_UNIFORM, "element": COEF_PER_ELEMENT, "qp": COEF_PER_QP,
        "function": COEF_FUNCTION}
KFMT = {"full": K_FULL, "packed": K_SYM_PACKED}
PREC = {"fp64": FP64, "fp32": FP32_BULK}

STATUS = {0: "FE_OK", 1: "FE_ERR_INVALID_ARG", 2: "FE_ERR_UNSUPPORTED", 3: "FE_ERR_NOT_SYMMETRIC",
          4: "FE_ERR_HIP", 5: "FE_ERR_CAPACITY"}


class Problem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("coef_mode", ctypes.c_int32), ("coef_mask", ctypes.c_uint32),
                ("k_format", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("uniform", ctypes.c_double * 20)]


class QuadRule(ctypes.Structure):
    _fields_ = [("n_q", ctypes.c_int32), ("xi", ctypes.POINTER(ctypes.c_double)),
                ("w", ctypes.POINTER(ctypes.c_double))]


class Variant(ctypes.Structure):
    _fields_ = [("wg_size", ctypes.c_int32), ("elems_per_thread", ctypes.c_int32),
                ("ref_in_lds", ctypes.c_int32), ("nontemporal", ctypes.c_int32),
                ("blocks", ctypes.c_int32), ("row_split", ctypes.c_int32),
                ("loop_order", ctypes.c_int32), ("lanes", ctypes.c_int32)]

    def as_tuple(self):
        return (self.wg_size, self.elems_per_thread, self.ref_in_lds, self.nontemporal, self.blocks,
                self.row_split, self.loop_order, self.lanes)


class FeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libfe.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                               "`python -m paper_1504_01023_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, R, V = ctypes.POINTER(Problem), ctypes.POINTER(QuadRule), ctypes.POINTER(Variant)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.fe_integrate.argtypes = [P, i32, i64, vp, vp, R, vp, vp, vp]
        L.fe_integrate_ex.argtypes = [P, i32, i64, vp, vp, i64, R, vp, vp, i64, V, vp]
        for f in ("fe_k_entries", "fe_f_entries"):
            getattr(L, f).argtypes = [P, i32]
            getattr(L, f).restype = i64
        for f in ("fe_coeff_entries", "fe_bytes_per_element"):
            getattr(L, f).argtypes = [P, i32, i32]
            getattr(L, f).restype = i64
        L.fe_k_index.argtypes = [P, i32, i32, i32]
        L.fe_k_index.restype = i64
        L.fe_quad_rule_builtin.argtypes = [i32, i32, R]
        L.fe_status_string.argtypes = [i32]
        L.fe_status_string.restype = ctypes.c_char_p
        L.fe_last_error.restype = ctypes.c_char_p
        L.fe_autotune.argtypes = [P, i32, i64, vp, vp, i64, R, vp, vp, i64, i32, V,
                                  ctypes.POINTER(ctypes.c_double), vp]
        L.fe_tuning_get.argtypes = [P, i32, i32, V]
        L.fe_tuning_set.argtypes = [P, i32, i32, V]
        L.fe_tuning_save.argtypes = [ctypes.c_char_p]
        L.fe_tuning_load.argtypes = [ctypes.c_char_p]
        L.fe_stream_copy.argtypes = [vp, vp, i64, vp]
        L.fe_integrate_indexed.argtypes = [P, i32, i64, vp, i64, vp, i64, vp, i64, R, vp, vp, i64,
                                           V, vp]
        L.fe_apply_indexed.argtypes = [P, i32, i64, vp, i64, vp, i64, vp, i64, R, vp, vp, vp,
                                       ctypes.POINTER(ctypes.c_int64), i32, vp]
        L.fe_color_elements.argtypes = [i32, i64, vp, i64, i64, vp, vp, i32]
        L.fe_integrate_natural.argtypes = [P, i32, i64, vp, vp, R, vp, vp, vp]
        L.fe_count_inverted.argtypes = [i32, i64, vp, i64, R, vp, vp]
        L.fe_csr_pattern.argtypes = [i32, i64, vp, i64, i64, i32, vp, vp, i64]
        L.fe_csr_pattern.restype = i64
        L.fe_assemble_csr.argtypes = [P, i32, i64, vp, i64, vp, i64, vp, i64, R, vp, vp, i64, vp,
                                      vp, ctypes.POINTER(ctypes.c_int64), i32, vp]
        L.fe_assemble_csr_stored.argtypes = [P, i32, i64, vp, i64, i64, vp, vp, i64, i32, vp, vp,
                                             i64, vp, vp, vp, vp, vp]
        L.fe_node_incidence.argtypes = [i32, i64, vp, i64, i64, vp, vp]
        L.fe_node_incidence.restype = i64
        L.fe_assemble_csr_rows.argtypes = [P, i32, i64, vp, i64, vp, i64, vp, i64, R, vp, vp, i64,
                                           vp, vp, vp, vp, vp]
        L.fe_csr_blocks.argtypes = [i32, i64, vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                    vp]
        L.fe_csr_blocks.restype = i64
        L.fe_assemble_csr_blocks.argtypes = [P, i32, i64, vp, i64, vp, i64, R, vp, vp, i64, vp,
                                             vp, vp, i64, vp, vp, vp, vp, vp, vp]
        L.fe_stream_pattern.argtypes = [vp, i32, vp, i32, i32, i64, i64, vp]
        L.fe_ld_for.argtypes = [i64]
        L.fe_ld_for.restype = i64
        L.fe_tuning_builtin.argtypes = [ctypes.c_char_p, i32, ctypes.POINTER(ctypes.c_int)]
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != 0:
        raise FeError(status, lib().fe_last_error().decode())


# ------------------------------------------------------------------ descriptors
def problem(kind="scalar", precision="fp64", coef_mode="uniform", mask=0, uniform=None,
            k_format="full") -> Problem:
    p = Problem()
    p.kind = KIND.get(kind, kind)
    p.precision = PREC.get(precision, precision)
    p.coef_mode = MODE.get(coef_mode, coef_mode)
    p.coef_mask = int(mask)
    p.k_format = KFMT.get(k_format, k_format)
    p.reserved = 0
    if uniform is not None:
        u = np.asarray(uniform, dtype=np.float64).ravel()
        for i, x in enumerate(u[:20]):
            p.uniform[i] = float(x)
    return p


def problem_for(wl, precision="fp64") -> Problem:
    """Descriptor for a generated workload (paper_1504_01023_amd.inputs)."""
    return problem(wl.kind, precision, wl.coef_mode, wl.mask, wl.uniform, wl.k_format)


class Rule:
    """A quadrature rule held in host memory for the duration of the calls."""

    def __init__(self, xi, w):
        self.xi = np.ascontiguousarray(np.asarray(xi, dtype=np.float64).reshape(-1, 3))
        self.w = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(-1))
        self.c = QuadRule(len(self.w), self.xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          self.w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))

    @property
    def n_q(self) -> int:
        return len(self.w)


def builtin_rule(elem, n_q: int) -> Rule:
    r = QuadRule()
    _check(lib().fe_quad_rule_builtin(ELEM.get(elem, elem), n_q, ctypes.byref(r)))
    xi = np.ctypeslib.as_array(r.xi, shape=(n_q * 3,)).copy()
    w = np.ctypeslib.as_array(r.w, shape=(n_q,)).copy()
    return Rule(xi, w)


def k_entries(p: Problem, elem) -> int:
    return int(lib().fe_k_entries(ctypes.byref(p), ELEM.get(elem, elem)))


def f_entries(p: Problem, elem) -> int:
    return int(lib().fe_f_entries(ctypes.byref(p), ELEM.get(elem, elem)))


def coeff_entries(p: Problem, elem, n_q: int) -> int:
    return int(lib().fe_coeff_entries(ctypes.byref(p), ELEM.get(elem, elem), n_q))


def bytes_per_element(p: Problem, elem, n_q: int) -> int:
    return int(lib().fe_bytes_per_element(ctypes.byref(p), ELEM.get(elem, elem), n_q))


def k_index(p: Problem, elem, row: int, col: int) -> int:
    return int(lib().fe_k_index(ctypes.byref(p), ELEM.get(elem, elem), row, col))


def variant(wg_size=0, elems_per_thread=0, ref_in_lds=0, nontemporal=0, blocks=0,
            row_split=0, loop_order=0, lanes=0) -> Variant:
    return Variant(wg_size, elems_per_thread, ref_in_lds, nontemporal, blocks, row_split,
                   loop_order, lanes)


# ------------------------------------------------------------------- execution
def _dtype(p: Problem):
    import torch
    return torch.float64 if p.precision == FP64 else torch.float32


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def ld_for(n_elem: int) -> int:
    """fe_ld_for: the leading dimension to allocate for rows of n_elem
    elements (n_elem rounded up to whole cache lines of every row)."""
    return int(lib().fe_ld_for(int(n_elem)))


def _ld(t, name="tensor"):
    """Leading dimension of a row-major (rows, n) tensor: its row stride, so
    a view t[:, :n] of a padded (rows, ld) buffer passes ld."""
    if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1):
        raise ValueError(f"{name} must be a 2-D tensor with unit column stride")
    return t.stride(0) if t.shape[0] > 1 else max(t.stride(0), t.shape[1])


def _check_tensor(t, name, dtype, rows, ld):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 2 or _ld(t, name) != ld or t.shape[0] < rows:
        raise ValueError(f"{name} must be a ({rows}, n) tensor with leading dimension {ld}, got "
                         f"shape {tuple(t.shape)} and strides {tuple(t.stride())}")


def _padded_out(rows, n, dt, device):
    """A (rows, n) view of a (rows, ld_for(n)) buffer: line-aligned rows."""
    import torch
    return torch.empty((rows, max(1, ld_for(n))), dtype=dt, device=device)[:, :n]


def _check_coeffs(p: Problem, coeffs, dt, nc, ld_in):
    import torch
    if p.coef_mode == COEF_FUNCTION:
        if not (coeffs.is_cuda and coeffs.dtype == torch.float64 and coeffs.is_contiguous()
                and coeffs.numel() == FN_PARAMS):
            raise ValueError(f"function parameters must be {FN_PARAMS} contiguous float64 GPU values")
        return
    _check_tensor(coeffs, "coeffs", dt, nc, ld_in)


def integrate(p: Problem, elem, coords, coeffs, rule: Rule, out_K=None, out_F=None,
              n_elem: int | None = None, variant: Variant | None = None, stream=None):
    """Enqueue the integration of n_elem elements (default: all columns of
    coords) and return (out_K, out_F). Arrays are (rows, n) tensors whose
    row stride is the leading dimension (views of padded buffers pass their
    padding). Outputs not given are allocated with line-aligned rows
    (ld_for(n)) and returned as (k_entries, n) and (f_entries, n) views."""
    import torch
    e = ELEM.get(elem, elem)
    ld_in = _ld(coords, "coords")
    n = coords.shape[1] if n_elem is None else int(n_elem)
    dt = _dtype(p)
    nk, nf = k_entries(p, e), f_entries(p, e)
    if out_K is None and out_F is None:
        out_K = _padded_out(nk, n, dt, coords.device)
        out_F = _padded_out(nf, n, dt, coords.device)
    elif out_K is None or out_F is None:
        raise ValueError("give both out_K and out_F, or neither")
    ld_out = _ld(out_K, "out_K")
    _check_tensor(coords, "coords", torch.float64, 3 * (4 if e == TET4 else 6), ld_in)
    nc = coeff_entries(p, e, rule.n_q)
    if nc > 0:
        if coeffs is None:
            raise ValueError("this problem reads coefficients from memory; coeffs is None")
        _check_coeffs(p, coeffs, dt, nc, ld_in)
    _check_tensor(out_K, "out_K", dt, nk, ld_out)
    _check_tensor(out_F, "out_F", dt, nf, ld_out)
    cptr = ctypes.c_void_p(coeffs.data_ptr()) if (coeffs is not None and nc > 0) else None
    vptr = ctypes.byref(variant) if variant is not None else None
    _check(lib().fe_integrate_ex(ctypes.byref(p), e, n, ctypes.c_void_p(coords.data_ptr()), cptr,
                                 ld_in, ctypes.byref(rule.c), ctypes.c_void_p(out_K.data_ptr()),
                                 ctypes.c_void_p(out_F.data_ptr()), ld_out, vptr,
                                 _stream_handle(stream)))
    return out_K, out_F


def integrate_indexed(p: Problem, elem, nodes, conn, coeffs, rule: Rule, out_K=None, out_F=None,
                      n_elem: int | None = None, variant: Variant | None = None, stream=None):
    """Indexed geometry: nodes (n_nodes, 3) FP64 and conn (n_vert, ld) int32
    device tensors. Returns (out_K, out_F)."""
    import torch
    e = ELEM.get(elem, elem)
    nv = 4 if e == TET4 else 6
    ld_conn = _ld(conn, "conn")
    n = conn.shape[1] if n_elem is None else int(n_elem)
    dt = _dtype(p)
    nk, nf = k_entries(p, e), f_entries(p, e)
    if out_K is None and out_F is None:
        out_K = _padded_out(nk, n, dt, conn.device)
        out_F = _padded_out(nf, n, dt, conn.device)
    elif out_K is None or out_F is None:
        raise ValueError("give both out_K and out_F, or neither")
    if not (nodes.is_cuda and nodes.dtype == torch.float64 and nodes.is_contiguous()
            and nodes.dim() == 2 and nodes.shape[1] == 3):
        raise ValueError("nodes must be a contiguous (n_nodes, 3) float64 GPU tensor")
    _check_tensor(conn, "conn", torch.int32, nv, ld_conn)
    nc = coeff_entries(p, e, rule.n_q)
    ld_in = _ld(coeffs, "coeffs") if (coeffs is not None and nc > 0 and coeffs.dim() == 2) else n
    if nc > 0:
        _check_coeffs(p, coeffs, dt, nc, ld_in)
    ld_out = _ld(out_K, "out_K")
    _check_tensor(out_K, "out_K", dt, nk, ld_out)
    _check_tensor(out_F, "out_F", dt, nf, ld_out)
    cptr = ctypes.c_void_p(coeffs.data_ptr()) if (coeffs is not None and nc > 0) else None
    vptr = ctypes.byref(variant) if variant is not None else None
    _check(lib().fe_integrate_indexed(ctypes.byref(p), e, n, ctypes.c_void_p(nodes.data_ptr()),
                                      nodes.shape[0], ctypes.c_void_p(conn.data_ptr()), ld_conn,
                                      cptr, ld_in, ctypes.byref(rule.c),
                                      ctypes.c_void_p(out_K.data_ptr()),
                                      ctypes.c_void_p(out_F.data_ptr()), ld_out, vptr,
                                      _stream_handle(stream)))
    return out_K, out_F


def integrate_natural(p: Problem, elem, coords, coeffs, rule: Rule, out_K=None, out_F=None,
                      stream=None):
    """Natural (element-contiguous) order: coords (n, 3 n_vert) FP64, coeffs
    (n, coeff_entries) or the function parameters, outputs (n, k_entries) and
    (n, f_entries), all contiguous device tensors. Returns (out_K, out_F)."""
    import torch
    e = ELEM.get(elem, elem)
    nv = 4 if e == TET4 else 6
    n = coords.shape[0]
    dt = _dtype(p)
    nk, nf = k_entries(p, e), f_entries(p, e)
    if not (coords.is_cuda and coords.dtype == torch.float64 and coords.is_contiguous()
            and coords.dim() == 2 and coords.shape[1] == 3 * nv):
        raise ValueError(f"coords must be a contiguous (n, {3 * nv}) float64 GPU tensor")
    if out_K is None:
        out_K = torch.empty((n, nk), dtype=dt, device=coords.device)
    if out_F is None:
        out_F = torch.empty((n, nf), dtype=dt, device=coords.device)
    for name, t, c in (("out_K", out_K, nk), ("out_F", out_F, nf)):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous() and tuple(t.shape) == (n, c)):
            raise ValueError(f"{name} must be a contiguous ({n}, {c}) {dt} GPU tensor")
    nc = coeff_entries(p, e, rule.n_q)
    cptr = None
    if nc > 0:
        if coeffs is None:
            raise ValueError("this problem reads coefficients from memory; coeffs is None")
        if p.coef_mode == COEF_FUNCTION:
            _check_coeffs(p, coeffs, dt, nc, n)
        elif not (coeffs.is_cuda and coeffs.dtype == dt and coeffs.is_contiguous()
                  and tuple(coeffs.shape) == (n, nc)):
            raise ValueError(f"coeffs must be a contiguous ({n}, {nc}) {dt} GPU tensor")
        cptr = ctypes.c_void_p(coeffs.data_ptr())
    _check(lib().fe_integrate_natural(ctypes.byref(p), e, n, ctypes.c_void_p(coords.data_ptr()), cptr,
                                      ctypes.byref(rule.c), ctypes.c_void_p(out_K.data_ptr()),
                                      ctypes.c_void_p(out_F.data_ptr()), _stream_handle(stream)))
    return out_K, out_F


def color_elements(elem, conn, n_nodes: int, max_colors: int = 256):
    """Greedy colouring on the host (elements of one colour share no node).
    conn: (n_elem, n_vert) integer array of node ids. Returns (perm, color_ptr):
    the original element ids colour by colour, and the n_colors + 1 offsets."""
    e = ELEM.get(elem, elem)
    c = np.ascontiguousarray(np.asarray(conn).T.astype(np.int32))
    n = c.shape[1]
    perm = np.empty(n, dtype=np.int32)
    ptr = np.empty(max_colors + 1, dtype=np.int64)
    k = lib().fe_color_elements(e, n, c.ctypes.data_as(ctypes.c_void_p), n, int(n_nodes),
                                perm.ctypes.data_as(ctypes.c_void_p),
                                ptr.ctypes.data_as(ctypes.c_void_p), max_colors)
    if k < 0:
        _check(-k)
    return perm, ptr[: k + 1].copy()


def apply_indexed(p: Problem, elem, nodes, conn, coeffs, rule: Rule, x, y=None, b=None,
                  color_ptr=None, n_elem: int | None = None, stream=None):
    """Matrix-free y += A x (and b += assembled F when b is given) over the
    elements of conn (n_vert, ld) int32; x, y, b device vectors of n_nodes *
    components values in the tier's precision. color_ptr: host offsets of the
    colours (None: one launch with atomic adds). Returns (y, b)."""
    import torch
    e = ELEM.get(elem, elem)
    nv = 4 if e == TET4 else 6
    ld_conn = _ld(conn, "conn")
    n = conn.shape[1] if n_elem is None else int(n_elem)
    dt = _dtype(p)
    ncomp = 1 if p.kind == SCALAR_CDR else 3
    ndof = nodes.shape[0] * ncomp
    if not (nodes.is_cuda and nodes.dtype == torch.float64 and nodes.is_contiguous()
            and nodes.dim() == 2 and nodes.shape[1] == 3):
        raise ValueError("nodes must be a contiguous (n_nodes, 3) float64 GPU tensor")
    _check_tensor(conn, "conn", torch.int32, nv, ld_conn)
    for name, t in (("x", x), ("y", y), ("b", b)):
        if t is not None and not (t.is_cuda and t.dtype == dt and t.is_contiguous()
                                  and t.numel() == ndof):
            raise ValueError(f"{name} must be a contiguous {dt} GPU vector of {ndof} values")
    if y is None:
        y = torch.zeros(ndof, dtype=dt, device=nodes.device)
    nc = coeff_entries(p, e, rule.n_q)
    ld_in = _ld(coeffs, "coeffs") if (coeffs is not None and nc > 0 and coeffs.dim() == 2) else n
    if nc > 0:
        _check_coeffs(p, coeffs, dt, nc, ld_in)
    cptr = ctypes.c_void_p(coeffs.data_ptr()) if (coeffs is not None and nc > 0) else None
    if color_ptr is None:
        cp, ncol = None, 0
    else:
        cpa = np.ascontiguousarray(color_ptr, dtype=np.int64)
        cp, ncol = cpa.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(cpa) - 1
    _check(lib().fe_apply_indexed(ctypes.byref(p), e, n, ctypes.c_void_p(nodes.data_ptr()),
                                  nodes.shape[0], ctypes.c_void_p(conn.data_ptr()), ld_conn, cptr,
                                  ld_in, ctypes.byref(rule.c), ctypes.c_void_p(x.data_ptr()),
                                  ctypes.c_void_p(y.data_ptr()),
                                  ctypes.c_void_p(b.data_ptr()) if b is not None else None,
                                  cp, ncol, _stream_handle(stream)))
    return y, b


def csr_pattern(elem, conn, n_nodes: int, n_comp: int = 1):
    """Sparsity pattern of the assembled matrix, built on the host. conn:
    (n_elem, n_vert) integer array of node ids. Returns (row_ptr int64
    (n_nodes * n_comp + 1,), col_idx int32 (nnz,)) numpy arrays."""
    e = ELEM.get(elem, elem)
    c = np.ascontiguousarray(np.asarray(conn).T.astype(np.int32))
    n = c.shape[1]
    row_ptr = np.empty(int(n_nodes) * n_comp + 1, dtype=np.int64)
    args = (e, n, c.ctypes.data_as(ctypes.c_void_p), n, int(n_nodes), int(n_comp),
            row_ptr.ctypes.data_as(ctypes.c_void_p))
    nnz = lib().fe_csr_pattern(*args, None, 0)
    if nnz < 0:
        _check(-nnz)
    col_idx = np.empty(nnz, dtype=np.int32)
    got = lib().fe_csr_pattern(*args, col_idx.ctypes.data_as(ctypes.c_void_p), nnz)
    if got < 0:
        _check(-got)
    return row_ptr, col_idx


def node_incidence(elem, conn, n_nodes: int):
    """Elements at each node, built on the host. conn: (n_elem, n_vert)
    integer array of node ids. Returns (inc_ptr int64 (n_nodes + 1,), inc
    int32 (n_elem * n_vert,)) numpy arrays, inc coded element * n_vert +
    local vertex."""
    e = ELEM.get(elem, elem)
    c = np.ascontiguousarray(np.asarray(conn).T.astype(np.int32))
    n = c.shape[1]
    inc_ptr = np.empty(int(n_nodes) + 1, dtype=np.int64)
    inc = np.empty(n * c.shape[0], dtype=np.int32)
    got = lib().fe_node_incidence(e, n, c.ctypes.data_as(ctypes.c_void_p), n, int(n_nodes),
                                  inc_ptr.ctypes.data_as(ctypes.c_void_p),
                                  inc.ctypes.data_as(ctypes.c_void_p))
    if got < 0:
        _check(-got)
    return inc_ptr, inc


def _csr_args(p: Problem, elem, nodes, conn, coeffs, rule: Rule, row_ptr, col_idx, values, b,
              n_elem, with_b):
    import torch
    e = ELEM.get(elem, elem)
    nv = 4 if e == TET4 else 6
    ld_conn = _ld(conn, "conn")
    n = conn.shape[1] if n_elem is None else int(n_elem)
    dt = _dtype(p)
    ncomp = 1 if p.kind == SCALAR_CDR else 3
    ndof = nodes.shape[0] * ncomp
    if not (nodes.is_cuda and nodes.dtype == torch.float64 and nodes.is_contiguous()
            and nodes.dim() == 2 and nodes.shape[1] == 3):
        raise ValueError("nodes must be a contiguous (n_nodes, 3) float64 GPU tensor")
    _check_tensor(conn, "conn", torch.int32, nv, ld_conn)
    if not (row_ptr.is_cuda and row_ptr.dtype == torch.int64 and row_ptr.is_contiguous()
            and row_ptr.numel() == ndof + 1):
        raise ValueError(f"row_ptr must be a contiguous int64 GPU vector of {ndof + 1} values")
    if not (col_idx.is_cuda and col_idx.dtype == torch.int32 and col_idx.is_contiguous()):
        raise ValueError("col_idx must be a contiguous int32 GPU vector")
    nnz = col_idx.numel()
    if values is None:
        values = torch.zeros(nnz, dtype=dt, device=nodes.device)
    if b is None and with_b:
        b = torch.zeros(ndof, dtype=dt, device=nodes.device)
    for name, t, size in (("values", values, nnz), ("b", b, ndof)):
        if t is not None and not (t.is_cuda and t.dtype == dt and t.is_contiguous()
                                  and t.numel() == size):
            raise ValueError(f"{name} must be a contiguous {dt} GPU vector of {size} values")
    nc = coeff_entries(p, e, rule.n_q)
    ld_in = _ld(coeffs, "coeffs") if (coeffs is not None and nc > 0 and coeffs.dim() == 2) else n
    if nc > 0:
        _check_coeffs(p, coeffs, dt, nc, ld_in)
    cptr = ctypes.c_void_p(coeffs.data_ptr()) if (coeffs is not None and nc > 0) else None
    head = (ctypes.byref(p), e, n, ctypes.c_void_p(nodes.data_ptr()), nodes.shape[0],
            ctypes.c_void_p(conn.data_ptr()), ld_conn, cptr, ld_in, ctypes.byref(rule.c),
            ctypes.c_void_p(row_ptr.data_ptr()), ctypes.c_void_p(col_idx.data_ptr()), nnz,
            ctypes.c_void_p(values.data_ptr()),
            ctypes.c_void_p(b.data_ptr()) if b is not None else None)
    return head, values, b


def assemble_csr(p: Problem, elem, nodes, conn, coeffs, rule: Rule, row_ptr, col_idx,
                 values=None, b=None, color_ptr=None, n_elem: int | None = None, stream=None,
                 with_b: bool = False):
    """Assemble the global matrix into CSR values (values += sum of the
    element matrices at their couplings) and, when b is given or with_b,
    the load vector. row_ptr (int64) and col_idx (int32) are device tensors
    of the pattern csr_pattern builds; values (nnz,) and b (n_nodes *
    components,) device vectors in the tier's precision, zeroed here when not
    given. color_ptr as for apply_indexed. Returns (values, b)."""
    head, values, b = _csr_args(p, elem, nodes, conn, coeffs, rule, row_ptr, col_idx, values, b,
                                n_elem, with_b)
    if color_ptr is None:
        cp, ncol = None, 0
    else:
        cpa = np.ascontiguousarray(color_ptr, dtype=np.int64)
        cp, ncol = cpa.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(cpa) - 1
    _check(lib().fe_assemble_csr(*head, cp, ncol, _stream_handle(stream)))
    return values, b


def assemble_csr_rows(p: Problem, elem, nodes, conn, coeffs, rule: Rule, row_ptr, col_idx,
                      inc_ptr, inc, values=None, b=None, n_elem: int | None = None, stream=None,
                      with_b: bool = False):
    """The same assembly by row ownership (one lane per node, no colours, no
    atomics). inc_ptr (int64, n_nodes + 1) and inc (int32) are device copies
    of node_incidence's arrays. Returns (values, b)."""
    import torch
    head, values, b = _csr_args(p, elem, nodes, conn, coeffs, rule, row_ptr, col_idx, values, b,
                                n_elem, with_b)
    if not (inc_ptr.is_cuda and inc_ptr.dtype == torch.int64 and inc_ptr.is_contiguous()
            and inc_ptr.numel() == nodes.shape[0] + 1):
        raise ValueError("inc_ptr must be a contiguous int64 GPU vector of n_nodes + 1 values")
    if not (inc.is_cuda and inc.dtype == torch.int32 and inc.is_contiguous()):
        raise ValueError("inc must be a contiguous int32 GPU vector")
    _check(lib().fe_assemble_csr_rows(*head, ctypes.c_void_p(inc_ptr.data_ptr()),
                                      ctypes.c_void_p(inc.data_ptr()), _stream_handle(stream)))
    return values, b


@dataclass
class CsrBlocks:
    """Node blocks for assemble_csr_blocks (fe_csr_blocks): numpy arrays on
    the host, or device tensors after .to(device) (lconn and linc then hold
    their unsigned codes as int16 / int32 bits)."""
    n_blocks: int
    blk: object     # int64, 3 * (n_blocks + 1)
    elems: object   # int32, element slots
    verts: object   # int32, vertex slots
    lconn: object   # uint16, element slots * 4
    linc: object    # uint32, n_elem * 4: slot, local vertex and row positions

    def to(self, device):
        import torch

        def dev(a):
            a = np.ascontiguousarray(a)
            if a.dtype == np.uint16:
                a = a.view(np.int16)
            elif a.dtype == np.uint32:
                a = a.view(np.int32)
            return torch.from_numpy(a).to(device)
        return CsrBlocks(self.n_blocks, dev(self.blk), dev(self.elems), dev(self.verts),
                         dev(self.lconn), dev(self.linc))


def csr_blocks(elem, conn, n_nodes: int, inc_ptr, inc, row_ptr, col_idx) -> CsrBlocks:
    """Node blocks built on the host from conn ((n_elem, 4) node ids),
    node_incidence's (inc_ptr, inc) and csr_pattern's scalar (row_ptr,
    col_idx): consecutive nodes whose elements and vertices fit one
    workgroup's LDS (FE_CSR_BLOCK_* limits), with every incidence coded with
    the row positions of its element's vertices."""
    e = ELEM.get(elem, elem)
    c = np.ascontiguousarray(np.asarray(conn).T.astype(np.int32))
    nv, n = c.shape
    ip = np.ascontiguousarray(inc_ptr, dtype=np.int64)
    ic = np.ascontiguousarray(inc, dtype=np.int32)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    if ip.shape[0] != int(n_nodes) + 1 or ic.shape[0] != n * nv:
        raise ValueError("inc_ptr / inc do not match conn and n_nodes")
    if rp.shape[0] != int(n_nodes) + 1 or ci.shape[0] != rp[-1]:
        raise ValueError("row_ptr / col_idx are not a scalar pattern of n_nodes rows")
    vp = ctypes.c_void_p
    sizes = np.zeros(3, dtype=np.int64)
    args = (e, n, c.ctypes.data_as(vp), n, int(n_nodes), ip.ctypes.data_as(vp),
            ic.ctypes.data_as(vp), rp.ctypes.data_as(vp), ci.ctypes.data_as(vp),
            sizes.ctypes.data_as(vp))
    got = lib().fe_csr_blocks(*args, None, None, None, None, None)
    if got < 0:
        _check(-got)
    nb, ne, nvx = (int(x) for x in sizes)
    blk = np.empty(3 * (nb + 1), dtype=np.int64)
    elems = np.empty(max(ne, 1), dtype=np.int32)
    verts = np.empty(max(nvx, 1), dtype=np.int32)
    lconn = np.empty(max(ne * nv, 1), dtype=np.uint16)
    linc = np.empty(max(n * nv, 1), dtype=np.uint32)
    got = lib().fe_csr_blocks(*args, blk.ctypes.data_as(vp), elems.ctypes.data_as(vp),
                              verts.ctypes.data_as(vp), lconn.ctypes.data_as(vp),
                              linc.ctypes.data_as(vp))
    if got < 0:
        _check(-got)
    return CsrBlocks(nb, blk, elems[:ne], verts[:nvx], lconn[:ne * nv], linc[:n * nv])


def assemble_csr_blocks(p: Problem, elem, nodes, coeffs, rule: Rule, row_ptr, col_idx, inc_ptr,
                        blocks: CsrBlocks, values=None, b=None, stream=None,
                        with_b: bool = False):
    """The row-ownership assembly over node blocks (blocks: device
    CsrBlocks, inc_ptr the device copy of node_incidence's inc_ptr): each
    workgroup stages its block's elements and vertices in LDS once. Values
    and b equal assemble_csr_rows' bit for bit. Returns (values, b)."""
    import torch
    e = ELEM.get(elem, elem)
    nv = 4 if e == TET4 else 6
    dt = _dtype(p)
    n = blocks.linc.numel() // nv
    ndof = nodes.shape[0]
    if not (nodes.is_cuda and nodes.dtype == torch.float64 and nodes.is_contiguous()
            and nodes.dim() == 2 and nodes.shape[1] == 3):
        raise ValueError("nodes must be a contiguous (n_nodes, 3) float64 GPU tensor")
    if not (row_ptr.is_cuda and row_ptr.dtype == torch.int64 and row_ptr.is_contiguous()
            and row_ptr.numel() == ndof + 1):
        raise ValueError(f"row_ptr must be a contiguous int64 GPU vector of {ndof + 1} values")
    if not (col_idx.is_cuda and col_idx.dtype == torch.int32 and col_idx.is_contiguous()):
        raise ValueError("col_idx must be a contiguous int32 GPU vector")
    if not (inc_ptr.is_cuda and inc_ptr.dtype == torch.int64 and inc_ptr.is_contiguous()
            and inc_ptr.numel() == ndof + 1):
        raise ValueError("inc_ptr must be a contiguous int64 GPU vector of n_nodes + 1 values")
    for name, t, want in (("blk", blocks.blk, torch.int64), ("elems", blocks.elems, torch.int32),
                          ("verts", blocks.verts, torch.int32), ("lconn", blocks.lconn, torch.int16),
                          ("linc", blocks.linc, torch.int32)):
        if not (t.is_cuda and t.dtype == want and t.is_contiguous()):
            raise ValueError(f"blocks.{name} must be a contiguous {want} GPU tensor")
    if blocks.blk.numel() != 3 * (blocks.n_blocks + 1):
        raise ValueError("blocks.blk must hold 3 * (n_blocks + 1) values")
    nnz = col_idx.numel()
    if values is None:
        values = torch.zeros(nnz, dtype=dt, device=nodes.device)
    if b is None and with_b:
        b = torch.zeros(ndof, dtype=dt, device=nodes.device)
    for name, t, size in (("values", values, nnz), ("b", b, ndof)):
        if t is not None and not (t.is_cuda and t.dtype == dt and t.is_contiguous()
                                  and t.numel() == size):
            raise ValueError(f"{name} must be a contiguous {dt} GPU vector of {size} values")
    nc = coeff_entries(p, e, rule.n_q)
    ld_in = _ld(coeffs, "coeffs") if (coeffs is not None and nc > 0 and coeffs.dim() == 2) else n
    if nc > 0:
        _check_coeffs(p, coeffs, dt, nc, ld_in)
    cptr = ctypes.c_void_p(coeffs.data_ptr()) if (coeffs is not None and nc > 0) else None
    vp = ctypes.c_void_p
    _check(lib().fe_assemble_csr_blocks(
        ctypes.byref(p), e, n, vp(nodes.data_ptr()), ndof, cptr, ld_in, ctypes.byref(rule.c),
        vp(row_ptr.data_ptr()), vp(col_idx.data_ptr()), nnz, vp(values.data_ptr()),
        vp(b.data_ptr()) if b is not None else None, vp(inc_ptr.data_ptr()), blocks.n_blocks,
        vp(blocks.blk.data_ptr()), vp(blocks.elems.data_ptr()), vp(blocks.verts.data_ptr()),
        vp(blocks.lconn.data_ptr()), vp(blocks.linc.data_ptr()), _stream_handle(stream)))
    return values, b


def assemble_csr_stored(p: Problem, elem, conn, n_nodes: int, K, F, row_ptr, col_idx, inc_ptr, inc,
                        values=None, b=None, n_elem: int | None = None, stream=None,
                        with_b: bool = False, elem_major: bool = False):
    """Assemble stored element matrices into CSR values, one lane per node.
    K, F: (k_entries, ld) and (f_entries, ld) device tensors as fe.integrate
    returns them, or with elem_major (n_elem, k_entries) and (n_elem,
    f_entries) as fe.integrate_natural returns them. conn (n_vert, ld_conn)
    int32; row_ptr, col_idx, inc_ptr, inc device tensors as for
    assemble_csr_rows. Returns (values, b)."""
    import torch
    e = ELEM.get(elem, elem)
    nv = 4 if e == TET4 else 6
    ld_conn = _ld(conn, "conn")
    n = conn.shape[1] if n_elem is None else int(n_elem)
    dt = _dtype(p)
    ncomp = 1 if p.kind == SCALAR_CDR else 3
    ndof = int(n_nodes) * ncomp
    _check_tensor(conn, "conn", torch.int32, nv, ld_conn)
    if elem_major:
        ld = 0
        _check_tensor(K, "K", dt, n, k_entries(p, e))
        if F is not None:
            _check_tensor(F, "F", dt, n, f_entries(p, e))
    else:
        ld = _ld(K, "K")
        _check_tensor(K, "K", dt, k_entries(p, e), ld)
        if F is not None:
            _check_tensor(F, "F", dt, f_entries(p, e), ld)
    nnz = col_idx.numel()
    if values is None:
        values = torch.zeros(nnz, dtype=dt, device=K.device)
    if b is None and with_b:
        b = torch.zeros(ndof, dtype=dt, device=K.device)
    for name, t, size in (("values", values, nnz), ("b", b, ndof)):
        if t is not None and not (t.is_cuda and t.dtype == dt and t.is_contiguous()
                                  and t.numel() == size):
            raise ValueError(f"{name} must be a contiguous {dt} GPU vector of {size} values")
    for name, t, d in (("row_ptr", row_ptr, torch.int64), ("col_idx", col_idx, torch.int32),
                       ("inc_ptr", inc_ptr, torch.int64), ("inc", inc, torch.int32)):
        if not (t.is_cuda and t.dtype == d and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {d} GPU vector")
    vp = ctypes.c_void_p
    _check(lib().fe_assemble_csr_stored(ctypes.byref(p), e, n, vp(conn.data_ptr()), ld_conn,
                                        int(n_nodes), vp(K.data_ptr()),
                                        vp(F.data_ptr()) if F is not None else None, ld,
                                        int(bool(elem_major)), vp(row_ptr.data_ptr()), vp(col_idx.data_ptr()), nnz,
                                        vp(values.data_ptr()),
                                        vp(b.data_ptr()) if b is not None else None,
                                        vp(inc_ptr.data_ptr()), vp(inc.data_ptr()),
                                        _stream_handle(stream)))
    return values, b


def count_inverted(elem, coords, rule: Rule, n_elem: int | None = None, count=None,
                   stream=None):
    """Enqueue the count of elements whose det J is not positive at some rule
    point. coords: (3 n_vert, ld) FP64 device tensor. Adds to ``count`` (a
    one-element int64 device tensor, zeroed here when not given) and returns
    it."""
    import torch
    e = ELEM.get(elem, elem)
    ld_in = _ld(coords, "coords")
    n = coords.shape[1] if n_elem is None else int(n_elem)
    _check_tensor(coords, "coords", torch.float64, 3 * (4 if e == TET4 else 6), ld_in)
    if count is None:
        count = torch.zeros(1, dtype=torch.int64, device=coords.device)
    if not (count.is_cuda and count.dtype == torch.int64 and count.numel() == 1):
        raise ValueError("count must be a one-element int64 GPU tensor")
    _check(lib().fe_count_inverted(e, n, ctypes.c_void_p(coords.data_ptr()), ld_in,
                                   ctypes.byref(rule.c), ctypes.c_void_p(count.data_ptr()),
                                   _stream_handle(stream)))
    return count


def autotune(p: Problem, elem, coords, coeffs, rule: Rule, out_K, out_F, reps: int = 5,
             stream=None, n_elem: int | None = None):
    """Exhaustive search over the compiled variants (synchronises the stream)
    on n_elem elements (default: all columns of coords), with the leading
    dimensions of the given tensors. Returns (variant tuple, mean ms)."""
    e = ELEM.get(elem, elem)
    best = Variant()
    ms = ctypes.c_double(0.0)
    ld_in = _ld(coords, "coords")
    n = coords.shape[1] if n_elem is None else int(n_elem)
    cptr = ctypes.c_void_p(coeffs.data_ptr()) if coeffs is not None else None
    _check(lib().fe_autotune(ctypes.byref(p), e, n, ctypes.c_void_p(coords.data_ptr()), cptr, ld_in,
                             ctypes.byref(rule.c), ctypes.c_void_p(out_K.data_ptr()),
                             ctypes.c_void_p(out_F.data_ptr()), _ld(out_K, "out_K"), reps,
                             ctypes.byref(best), ctypes.byref(ms), _stream_handle(stream)))
    return best.as_tuple(), ms.value


def tuning_get(p: Problem, elem, n_q: int):
    v = Variant()
    st = lib().fe_tuning_get(ctypes.byref(p), ELEM.get(elem, elem), n_q, ctypes.byref(v))
    return v.as_tuple() if st == 0 else None


def tuning_set(p: Problem, elem, n_q: int, v: Variant) -> None:
    _check(lib().fe_tuning_set(ctypes.byref(p), ELEM.get(elem, elem), n_q, ctypes.byref(v)))


def tuning_save(path: str) -> None:
    _check(lib().fe_tuning_save(path.encode()))


def tuning_load(path: str) -> None:
    _check(lib().fe_tuning_load(path.encode()))


def tuning_clear() -> None:
    """Empty the caller's tuning table (the built-in entries stay in effect)."""
    lib().fe_tuning_clear()


def tuning_builtin():
    """(in effect, table architecture, entries in effect) of the built-in
    tuning table."""
    arch = ctypes.create_string_buffer(64)
    n = ctypes.c_int(0)
    on = lib().fe_tuning_builtin(arch, 64, ctypes.byref(n))
    return bool(on), arch.value.decode(), n.value


def stream_pattern(inp, out, n: int, stream=None) -> None:
    """The bare access pattern of an integration kernel: inp (rows_in, ld)
    float64 and out (rows_out, ld) float64 or float32 device tensors (row
    views of ld >= n columns); reads the first n columns of every input row
    and writes those of every output row."""
    import torch
    ld = inp.stride(0) if inp.dim() == 2 and inp.shape[0] > 0 else out.stride(0)
    if not (out.is_cuda and out.dim() == 2 and out.stride(1) == 1 and out.stride(0) == ld
            and out.dtype in (torch.float64, torch.float32)):
        raise ValueError("out must be a (rows_out, ld) float64 / float32 GPU row view")
    if not (inp.is_cuda and inp.dim() == 2 and inp.dtype == torch.float64
            and (inp.shape[0] == 0 or (inp.stride(1) == 1 and inp.stride(0) == ld))):
        raise ValueError("inp must be a (rows_in, ld) float64 GPU row view with out's ld")
    _check(lib().fe_stream_pattern(ctypes.c_void_p(inp.data_ptr()) if inp.shape[0] else None,
                                   inp.shape[0], ctypes.c_void_p(out.data_ptr()), out.shape[0],
                                   out.element_size(), int(n), int(ld), _stream_handle(stream)))


def stream_copy(dst, src, stream=None) -> None:
    """Plain streaming copy of src into dst (same byte size, multiple of 16)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("dst and src sizes differ")
    _check(lib().fe_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                nb, _stream_handle(stream)))


@dataclass
class DeviceWorkload:
    """A generated workload resident in device memory."""
    wl: object
    precision: str
    problem: Problem
    rule: Rule
    coords: object
    coeffs: object

    @property
    def n_elem(self) -> int:
        return self.wl.n_elem


def to_device(wl, precision="fp64", device="cuda", rule: Rule | None = None) -> DeviceWorkload:
    """Upload a generated workload (coordinates FP64; coefficients in the
    precision of the tier) into buffers with line-aligned rows (ld_for(n));
    the arrays are (rows, n) views of them."""
    import torch
    p = problem_for(wl, precision)
    r = rule if rule is not None else builtin_rule(wl.elem, wl.n_q)
    n = wl.n_elem

    def upload(a, dt):
        # rows padded to ld_for(n): the (rows, n) view keeps line-aligned rows
        buf = torch.zeros((a.shape[0], max(1, ld_for(n))), dtype=dt, device=device)
        buf[:, :n] = torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        return buf[:, :n]

    coords = upload(wl.mesh.coords, torch.float64)
    coeffs = None
    if wl.coeffs is not None and wl.coef_mode == "function":
        coeffs = torch.from_numpy(np.ascontiguousarray(wl.coeffs, dtype=np.float64)).to(device)
    elif wl.coeffs is not None and wl.coef_mode != "uniform":
        coeffs = upload(wl.coeffs, torch.float64 if precision == "fp64" else torch.float32)
    return DeviceWorkload(wl, precision, p, r, coords, coeffs)


def unpack_full(K: np.ndarray, N: int, packed: bool) -> np.ndarray:
    """(k_entries, n) SoA output -> (n, N, N) full matrices (host arrays)."""
    n = K.shape[1]
    out = np.empty((n, N, N), dtype=K.dtype)
    if not packed:
        return np.ascontiguousarray(K[: N * N].T.reshape(n, N, N))
    k = 0
    for r in range(N):
        for s in range(r, N):
            out[:, r, s] = K[k]
            out[:, s, r] = K[k]
            k += 1
    return out


# ------------------------------------------------------------ batched launches
class BatchKind(ctypes.Structure):
    _fields_ = [("problem", Problem), ("elem_type", ctypes.c_int32), ("n_q", ctypes.c_int32),
                ("xi", ctypes.POINTER(ctypes.c_double)), ("w", ctypes.POINTER(ctypes.c_double))]


class BatchRequest(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("n_elem", ctypes.c_int64),
                ("coords", ctypes.c_void_p), ("coeffs", ctypes.c_void_p), ("ld_in", ctypes.c_int64),
                ("out_K", ctypes.c_void_p), ("out_F", ctypes.c_void_p), ("ld_out", ctypes.c_int64)]


BATCH_STATIC_MAX_CHUNKS = 1024


def _batch_sigs(L):
    if getattr(L, "_batch_sigs", False):
        return
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.fe_batch_integrate_static.argtypes = [ctypes.POINTER(BatchKind), i32,
                                            ctypes.POINTER(BatchRequest), i32, i64, i32, vp]
    L.fe_batch_create.argtypes = [ctypes.POINTER(BatchKind), i32, i32, i64, i32,
                                  ctypes.POINTER(vp)]
    L.fe_batch_add.argtypes = [vp, i32, i64, vp, vp, i64, vp, vp, i64]
    L.fe_batch_pending.argtypes = [vp]
    L.fe_batch_launch.argtypes = [vp, vp]
    L.fe_batch_destroy.argtypes = [vp]
    L._batch_sigs = True


def _batch_kinds(kinds):
    arr = (BatchKind * len(kinds))()
    for i, (p, elem, rule) in enumerate(kinds):
        arr[i].problem = p
        arr[i].elem_type = ELEM.get(elem, elem)
        arr[i].n_q = rule.n_q
        arr[i].xi = rule.c.xi
        arr[i].w = rule.c.w
    return arr


def batch_integrate_static(kinds, requests, chunk_elems=16384, blocks_per_kind=0,
                           stream=None) -> None:
    """fe_batch_integrate_static: integrate a list of requests with the
    persistent batched kernels, allocating nothing (the chunk table lives in
    the library's own device array). kinds: list of (Problem, elem, Rule);
    requests: list of (kind, coords, coeffs, out_K, out_F[, n_elem]) with
    (rows, ld) tensors."""
    L = lib()
    _batch_sigs(L)
    arr = _batch_kinds(kinds)
    reqs = (BatchRequest * max(1, len(requests)))()
    for i, r in enumerate(requests):
        kind, coords, coeffs, out_K, out_F = r[:5]
        reqs[i].kind = kind
        reqs[i].n_elem = coords.shape[1] if len(r) < 6 or r[5] is None else int(r[5])
        reqs[i].coords = coords.data_ptr()
        reqs[i].coeffs = coeffs.data_ptr() if coeffs is not None else None
        reqs[i].ld_in = _ld(coords, "coords")
        reqs[i].out_K = out_K.data_ptr()
        reqs[i].out_F = out_F.data_ptr()
        reqs[i].ld_out = _ld(out_K, "out_K")
    _check(L.fe_batch_integrate_static(arr, len(kinds), reqs, len(requests), chunk_elems,
                                       blocks_per_kind, _stream_handle(stream)))


class Batch:
    """Persistent batched launches over a fixed set of kinds
    (fe_batch_create / fe_batch_add / fe_batch_launch)."""

    def __init__(self, kinds, max_chunks=1024, chunk_elems=16384, blocks_per_kind=0):
        """kinds: list of (Problem, elem, Rule)."""
        L = lib()
        _batch_sigs(L)
        self._rules = [k[2] for k in kinds]
        arr = _batch_kinds(kinds)
        self.kinds = list(kinds)
        self._h = ctypes.c_void_p()
        _check(L.fe_batch_create(arr, len(kinds), max_chunks, chunk_elems, blocks_per_kind,
                                 ctypes.byref(self._h)))

    def add(self, kind: int, coords, coeffs, out_K, out_F, n_elem=None) -> None:
        n = coords.shape[1] if n_elem is None else int(n_elem)
        _check(lib().fe_batch_add(self._h, kind, n, ctypes.c_void_p(coords.data_ptr()),
                                  ctypes.c_void_p(coeffs.data_ptr()) if coeffs is not None else None,
                                  _ld(coords, "coords"), ctypes.c_void_p(out_K.data_ptr()),
                                  ctypes.c_void_p(out_F.data_ptr()), _ld(out_K, "out_K")))

    def pending(self) -> int:
        return int(lib().fe_batch_pending(self._h))

    def launch(self, stream=None) -> None:
        _check(lib().fe_batch_launch(self._h, _stream_handle(stream)))

    def close(self) -> None:
        if self._h:
            lib().fe_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
