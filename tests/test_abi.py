"""CPU-only checks of the C ABI: the library loads and exports every symbol
include/fe.h declares, argument validation returns the documented status
codes before anything is enqueued, and the host-side helpers (sizes,
accounting, packed index map, built-in rules) are right. No GPU compute."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1504_01023_amd import fe, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "fe.h")).read()
    return sorted(set(re.findall(r"FE_API\s+[\w\s\*]+?\b(fe_\w+)\s*\(", src)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for must in ("fe_integrate", "fe_integrate_ex", "fe_k_entries", "fe_f_entries",
                 "fe_coeff_entries", "fe_quad_rule_builtin", "fe_status_string", "fe_last_error",
                 "fe_autotune", "fe_tuning_save", "fe_tuning_load", "fe_stream_copy"):
        assert must in syms


def test_library_exports_every_declared_symbol():
    L = fe.lib()
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing


def test_library_exports_nothing_undeclared():
    # only the documented C ABI is visible (everything else is hidden)
    out = os.popen(f"nm -D --defined-only {fe.LIB_PATH}").read()
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    fe_syms = {s for s in exported if s.startswith("fe_")}
    assert fe_syms == set(declared_symbols())


def test_status_strings():
    L = fe.lib()
    for st in range(6):
        assert L.fe_status_string(st)
    assert L.fe_status_string(99) == b"unknown status"


@pytest.mark.parametrize("elem,n_q", [("tet4", 1), ("tet4", 4), ("prism6", 6)])
def test_builtin_rules_match_oracle_rules(elem, n_q):
    r = fe.builtin_rule(elem, n_q)
    xi, w = oracle.quad_rule(elem, n_q)
    np.testing.assert_allclose(r.xi, xi, rtol=0, atol=1e-16)
    np.testing.assert_allclose(r.w, w, rtol=0, atol=1e-17)


def test_builtin_rule_unknown():
    with pytest.raises(fe.FeError) as ei:
        fe.builtin_rule("tet4", 5)
    assert ei.value.status == 2


def test_accounting_matches_paper_word_counts():
    # Sec. 4.4, table "accesses_and_operations": global accesses per element
    # 36 / 66 / 52 / 80 double words for tet Poisson, prism Poisson, tet
    # conv-diff, prism conv-diff (4 / 6 Gauss points, full K, Poisson with one
    # right-hand-side value per point, conv-diff with 20 element constants).
    poisson = fe.problem("scalar", "fp64", "qp", 1 << 16, np.r_[np.zeros(5), 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, np.zeros(4)], "full")
    cdr = fe.problem("scalar", "fp64", "element", (1 << 20) - 1, None, "full")
    assert fe.bytes_per_element(poisson, "tet4", 4) == 8 * 36
    assert fe.bytes_per_element(poisson, "prism6", 6) == 8 * 66
    assert fe.bytes_per_element(cdr, "tet4", 4) == 8 * 52
    assert fe.bytes_per_element(cdr, "prism6", 6) == 8 * 80
    # the headline workload: uniform Poisson, packed K: 96 + 80 + 32 bytes
    p1 = fe.problem("scalar", "fp64", "uniform", 0, None, "packed")
    assert fe.bytes_per_element(p1, "tet4", 1) == 208
    # FP32 tier: coordinates stay FP64
    c32 = fe.problem("scalar", "fp32", "element", (1 << 20) - 1, None, "full")
    assert fe.bytes_per_element(c32, "tet4", 4) == 96 + 4 * (20 + 16 + 4)
    el = fe.problem("elasticity", "fp64", "element", 31, None, "packed")
    assert fe.bytes_per_element(el, "tet4", 1) == 96 + 8 * (5 + 78 + 12)
    assert fe.bytes_per_element(el, "prism6", 6) == 144 + 8 * (5 + 171 + 18)


def test_entry_counts_and_packed_index():
    for kind, nc in (("scalar", 1), ("elasticity", 3)):
        for elem, ns in (("tet4", 4), ("prism6", 6)):
            N = ns * nc
            pf = fe.problem(kind, "fp64", "uniform", 0, None, "full")
            pp = fe.problem(kind, "fp64", "uniform", 0, None, "packed")
            assert fe.k_entries(pf, elem) == N * N
            assert fe.k_entries(pp, elem) == N * (N + 1) // 2
            assert fe.f_entries(pf, elem) == N
            seen = []
            for r in range(N):
                for s in range(N):
                    assert fe.k_index(pf, elem, r, s) == r * N + s
                    k = fe.k_index(pp, elem, r, s)
                    if s < r:
                        assert k == -1
                    else:
                        seen.append(k)
            assert seen == list(range(N * (N + 1) // 2))
            assert fe.k_index(pf, elem, N, 0) == -1


def test_coeff_entries():
    p = fe.problem("scalar", "fp64", "qp", (1 << 20) - 1, None, "full")
    assert fe.coeff_entries(p, "prism6", 6) == 120
    p = fe.problem("scalar", "fp64", "element", 0b101, None, "full")
    assert fe.coeff_entries(p, "tet4", 4) == 2
    p = fe.problem("scalar", "fp64", "uniform", 0b101, None, "full")
    assert fe.coeff_entries(p, "tet4", 4) == 0


def _call(p, elem=0, n=10, coords=0x1000, coeffs=None, ld_in=None, rule=None, K=0x2000, F=0x3000,
          ld_out=None, variant=None):
    L = fe.lib()
    rule = rule if rule is not None else fe.builtin_rule("tet4", 1)
    ld_in = n if ld_in is None else ld_in
    ld_out = n if ld_out is None else ld_out
    v = ctypes.byref(variant) if variant is not None else None
    return L.fe_integrate_ex(ctypes.byref(p) if p is not None else None, elem, n, coords, coeffs,
                             ld_in, ctypes.byref(rule.c), K, F, ld_out, v, None)


# Every case below fails validation, so nothing is launched and the fake
# addresses are never dereferenced.
def test_validation_status_codes():
    ok = fe.problem("scalar", "fp64", "uniform", 0, np.r_[np.zeros(5), 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 1, 0, 0, 0], "packed")
    assert _call(None) == 1
    assert _call(ok, elem=7) == 1
    assert _call(ok, n=-1) == 1
    assert _call(ok, coords=None) == 1
    assert _call(ok, K=None) == 1
    assert _call(ok, ld_in=5) == 1
    assert _call(ok, ld_out=9) == 1
    bad = fe.problem("scalar", "fp64", "uniform", 0, None, "packed")
    bad.kind = 5
    assert _call(bad) == 1
    bad = fe.problem("scalar", "fp64", "uniform", 0, None, "packed")
    bad.precision = 9
    assert _call(bad) == 1
    bad = fe.problem("scalar", "fp64", "uniform", 0, None, "packed")
    bad.reserved = 1
    assert _call(bad) == 1
    # per-element data without a coefficient pointer
    pe = fe.problem("scalar", "fp64", "element", 1 << 16, None, "full")
    assert _call(pe, coeffs=None) == 1
    # mask bits beyond the elasticity slots
    el = fe.problem("elasticity", "fp64", "element", 1 << 7, None, "packed")
    assert _call(el, coeffs=0x4000) == 1
    # unsupported point counts
    assert _call(ok, rule=fe.Rule(np.zeros((9, 3)), np.ones(9))) == 2
    # weights must be finite
    assert _call(ok, rule=fe.Rule(np.zeros((1, 3)), [np.nan])) == 1
    # misaligned pointer
    assert _call(ok, coords=0x1004) == 2
    # packed K with convection read from memory, or non-symmetric uniform data
    conv = fe.problem("scalar", "fp64", "element", 1 << 4, None, "packed")
    assert _call(conv, coeffs=0x4000) == 3
    u = np.zeros(20)
    u[4] = 1.0
    assert _call(fe.problem("scalar", "fp64", "uniform", 0, u, "packed")) == 3
    u = np.zeros(20)
    u[6] = 1.0
    assert _call(fe.problem("scalar", "fp64", "uniform", 0, u, "packed")) == 3
    # symmetric convection pair is fine for packed: validation passes (n = 0)
    u = np.zeros(20)
    u[4] = u[1] = 0.5
    assert _call(fe.problem("scalar", "fp64", "uniform", 0, u, "packed"), n=0) == 0
    # forced variants that do not exist
    assert _call(ok, variant=fe.variant(wg_size=96)) == 2
    # two elements per lane need even leading dimensions
    assert _call(ok, n=9, variant=fe.variant(elems_per_thread=2)) == 2
    assert fe.lib().fe_last_error()


def test_empty_batch_enqueues_nothing():
    # n_elem == 0 is FE_OK without any pointer or device
    p = fe.problem("scalar", "fp64", "uniform", 0, None, "full")
    assert _call(p, n=0, coords=None, K=None, F=None) == 0


def test_tuning_table_roundtrip(tmp_path):
    fe.tuning_clear()
    p = fe.problem("scalar", "fp64", "uniform", 0, None, "packed")
    # a 2-point rule: a family the built-in table has no entry for
    assert fe.tuning_get(p, "tet4", 2) is None
    fe.tuning_set(p, "tet4", 2, fe.variant(128, 2, 2, 1, 0, 1, 1, 3))
    assert fe.tuning_get(p, "tet4", 2) == (128, 2, 2, 1, 0, 1, 1, 3)
    path = str(tmp_path / "tune.txt")
    fe.tuning_save(path)
    fe.tuning_clear()
    assert fe.tuning_get(p, "tet4", 2) is None
    fe.tuning_load(path)
    assert fe.tuning_get(p, "tet4", 2) == (128, 2, 2, 1, 0, 1, 1, 3)
    fe.tuning_clear()
    # tables written before the lanes field (and before split / order) still load
    old = tmp_path / "old.txt"
    old.write_text("0 0 0 33 0 1 1 | 256 2 2 2 0 1 1\n0 0 0 63 1 0 4 | 64 1 1 1 0\n")
    fe.tuning_load(str(old))
    assert fe.tuning_get(p, "tet4", 1) == (256, 2, 2, 2, 0, 1, 1, 1)
    q = fe.problem("scalar", "fp64", "element", (1 << 20) - 1, None, "full")
    assert fe.tuning_get(q, "tet4", 4) == (64, 1, 1, 1, 0, 1, 1, 1)
    fe.tuning_clear()


def test_function_mode_sizes_and_validation():
    p = fe.problem("scalar", "fp64", "function", (1 << 20) - 1, None, "full")
    assert fe.coeff_entries(p, "prism6", 6) == 122
    # parameters are not per-element traffic
    assert fe.bytes_per_element(p, "prism6", 6) == 144 + 8 * (36 + 6)
    el = fe.problem("elasticity", "fp64", "function", 31, None, "packed")
    assert _call(el, coeffs=0x4000) == 2
    assert _call(p, coeffs=None) == 1


def test_vector_problem_sizes_and_validation():
    full = inputs.ALL_VECTOR_MASK
    p = fe.problem("vector", "fp64", "element", full, None, "full")
    assert fe.k_entries(p, "tet4") == 144 and fe.f_entries(p, "tet4") == 12
    assert fe.k_entries(p, "prism6") == 324 and fe.f_entries(p, "prism6") == 18
    assert fe.coeff_entries(p, "tet4", 4) == 156
    assert fe.bytes_per_element(p, "tet4", 4) == 96 + 8 * (156 + 144 + 12)
    q = fe.problem("vector", "fp32", "qp", (1 << 5) | (1 << 16), None, "full")
    assert fe.coeff_entries(q, "prism6", 6) == (9 + 3) * 6
    assert fe.bytes_per_element(q, "prism6", 6) == 144 + 4 * (72 + 324 + 18)
    assert fe.k_index(p, "tet4", 11, 0) == 132
    # per element or per point only, full K only
    for mode, fmt, mask in (("uniform", "full", 0), ("function", "full", full),
                            ("element", "packed", full)):
        bad = fe.problem("vector", "fp64", mode, mask, None, fmt)
        assert fe.k_entries(bad, "tet4") == -1
        assert _call(bad, coeffs=0x4000) == 2
    assert _call(p, coeffs=None) == 1


@pytest.mark.parametrize("elem", ["tet4", "prism6"])
def test_element_colouring(elem):
    mesh = inputs.tet_cube(4, 1) if elem == "tet4" else inputs.prism_layers(5, 3, 2)
    n = mesh.conn.shape[0]
    perm, ptr = fe.color_elements(elem, mesh.conn, mesh.nodes.shape[0])
    assert sorted(perm.tolist()) == list(range(n))
    assert ptr[0] == 0 and ptr[-1] == n and np.all(np.diff(ptr) > 0)
    for c in range(len(ptr) - 1):
        ids = perm[ptr[c]:ptr[c + 1]]
        assert np.all(np.diff(ids) > 0)                      # original order within a colour
        nodes = mesh.conn[ids].ravel()
        assert len(np.unique(nodes)) == len(nodes)           # no shared node
    # a node touches at most 24 Kuhn tets / 12 prisms: greedy needs few colours
    assert len(ptr) - 1 <= (32 if elem == "tet4" else 16)


def test_colouring_errors():
    mesh = inputs.tet_cube(2, 1)
    with pytest.raises(fe.FeError) as e:
        fe.color_elements("tet4", mesh.conn, mesh.nodes.shape[0], max_colors=3)
    assert e.value.status == 5
    bad = mesh.conn.copy()
    bad[3, 1] = mesh.nodes.shape[0]
    with pytest.raises(fe.FeError) as e:
        fe.color_elements("tet4", bad, mesh.nodes.shape[0])
    assert e.value.status == 1


def _apply_call(p, color_ptr=None, n_colors=0, x=0x5000, y=0x6000, nodes=0x7000, n_nodes=10,
                coeffs=None, elem=0):
    L = fe.lib()
    rule = fe.builtin_rule("tet4", 1) if elem == 0 else fe.builtin_rule("prism6", 6)
    cp = None
    if color_ptr is not None:
        arr = np.asarray(color_ptr, dtype=np.int64)
        cp = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        _apply_call.keep = arr
    return L.fe_apply_indexed(ctypes.byref(p), elem, 10, ctypes.c_void_p(nodes), n_nodes,
                              ctypes.c_void_p(0x1000), 10,
                              ctypes.c_void_p(coeffs) if coeffs else None, 10, ctypes.byref(rule.c),
                              ctypes.c_void_p(x) if x else None, ctypes.c_void_p(y) if y else None,
                              None, cp, n_colors, None)


def test_apply_validation_before_launch():
    p = fe.problem("scalar", "fp64", "uniform", 0, inputs.identity_diffusion_uniform(), "packed")
    assert _apply_call(p, x=0) == 1                               # x missing
    assert _apply_call(p, n_nodes=0) == 1                         # no nodes
    assert _apply_call(p, color_ptr=[0, 4], n_colors=1) == 1      # does not reach n_elem
    assert _apply_call(p, color_ptr=[0, 6, 4, 10], n_colors=3) == 1
    assert _apply_call(p, n_colors=2) == 1                        # colours without offsets
    # coefficient functions exist for scalar problems only
    vf = fe.problem("vector", "fp64", "function", inputs.ALL_VECTOR_MASK, None, "full")
    assert _apply_call(vf, coeffs=0x8000) == 2
    e = fe.problem("elasticity", "fp64", "uniform", 0, [1.0, 0.3, 0, 0, 0], "packed")
    assert _apply_call(e, y=0x6004) == 2                          # misaligned y


def test_count_inverted_validation_before_launch():
    L = fe.lib()
    r = fe.builtin_rule("prism6", 6)
    vp = ctypes.c_void_p
    call = lambda elem=1, n=10, coords=0x4000, ld=16, rule=r, count=0x8000: \
        L.fe_count_inverted(elem, n, vp(coords) if coords else None, ld,
                            ctypes.byref(rule.c) if rule is not None else None,
                            vp(count) if count else None, None)
    assert call(elem=3) == 1
    assert call(n=-1) == 1
    assert call(coords=0) == 1
    assert call(count=0) == 1
    assert call(ld=9) == 1
    assert call(rule=None) == 1
    assert call(rule=fe.Rule(np.zeros((9, 3)), np.ones(9))) == 2
    assert call(rule=fe.Rule(np.full((1, 3), np.inf), [1.0])) == 1
    assert call(coords=0x4004) == 2
    # nothing to count: no pointer is touched
    assert call(n=0, coords=0, count=0) == 0


@pytest.mark.parametrize("elem,n_comp", [("tet4", 1), ("tet4", 3), ("prism6", 1), ("prism6", 3)])
def test_csr_pattern_matches_brute_force(elem, n_comp):
    mesh = inputs.tet_cube(3, 2) if elem == "tet4" else inputs.prism_layers(3, 3, 2)
    nn = mesh.nodes.shape[0]
    row_ptr, col_idx = fe.csr_pattern(elem, mesh.conn, nn, n_comp)
    share = [set() for _ in range(nn)]
    for el in mesh.conn:
        for i in el:
            share[i].update(int(j) for j in el)
    want_ptr = [0]
    want_cols = []
    for i in range(nn):
        cols = [n_comp * j + b for j in sorted(share[i]) for b in range(n_comp)]
        for _ in range(n_comp):
            want_cols += cols
            want_ptr.append(len(want_cols))
    assert np.array_equal(row_ptr, np.array(want_ptr, dtype=np.int64))
    assert np.array_equal(col_idx, np.array(want_cols, dtype=np.int32))


def test_csr_pattern_errors_and_isolated_nodes():
    L = fe.lib()
    conn = np.ascontiguousarray(np.array([[0, 1, 2, 3]], dtype=np.int32).T)   # one tet, SoA
    vp = ctypes.c_void_p
    rp = np.zeros(6 * 3 + 1, dtype=np.int64)
    ci = np.zeros(200, dtype=np.int32)
    call = lambda n_nodes=6, n_comp=1, cap=200, c=conn, cols=True: L.fe_csr_pattern(
        0, 1, c.ctypes.data_as(vp), 1, n_nodes, n_comp, rp.ctypes.data_as(vp),
        ci.ctypes.data_as(vp) if cols else None, cap)
    # nodes 4 and 5 touch no element: empty rows
    assert call(cols=False) == 16
    assert call() == 16
    assert list(rp[:7]) == [0, 4, 8, 12, 16, 16, 16]
    assert call(n_comp=3) == 144
    assert call(n_comp=2) == -1
    assert call(n_nodes=3) == -1            # node id 3 outside [0, 3)
    assert call(cap=15) == -5               # col_idx too small
    assert fe.lib().fe_last_error()


def _csr_call(p, rows=0x5000, cols=0x6000, nnz=100, vals=0x7000, b=None, n=10, coeffs=None,
              elem=0):
    L = fe.lib()
    rule = fe.builtin_rule("tet4", 1) if elem == 0 else fe.builtin_rule("prism6", 6)
    v = lambda a: ctypes.c_void_p(a) if a else None
    return L.fe_assemble_csr(ctypes.byref(p), elem, n, ctypes.c_void_p(0x8000), 10,
                             ctypes.c_void_p(0x1000), 10, v(coeffs), 10, ctypes.byref(rule.c),
                             v(rows), v(cols), nnz, v(vals), v(b), None, 0, None)


def test_assemble_csr_validation_before_launch():
    p = fe.problem("scalar", "fp64", "uniform", 0, inputs.identity_diffusion_uniform(), "packed")
    assert _csr_call(p, rows=0) == 1
    assert _csr_call(p, cols=0) == 1
    assert _csr_call(p, vals=0) == 1
    assert _csr_call(p, nnz=-1) == 1
    assert _csr_call(p, rows=0x5004) == 2                          # misaligned row_ptr
    assert _csr_call(p, vals=0x7004) == 2                          # misaligned values
    vf = fe.problem("vector", "fp64", "function", inputs.ALL_VECTOR_MASK, None, "full")
    assert _csr_call(vf, coeffs=0x9000) == 2                       # not built
    assert _csr_call(p, rows=0, cols=0, vals=0, n=0) == 0          # nothing to do


@pytest.mark.parametrize("elem", ["tet4", "prism6"])
def test_node_incidence_matches_brute_force(elem):
    mesh = inputs.tet_cube(3, 3) if elem == "tet4" else inputs.prism_layers(3, 3, 3)
    nn = mesh.nodes.shape[0]
    ip, inc = fe.node_incidence(elem, mesh.conn, nn)
    nv = mesh.conn.shape[1]
    want_ptr = [0]
    want = []
    for i in range(nn):
        for e in range(mesh.n_elem):
            for v in range(nv):
                if mesh.conn[e, v] == i:
                    want.append(e * nv + v)
        want_ptr.append(len(want))
    assert np.array_equal(ip, np.array(want_ptr, dtype=np.int64))
    assert np.array_equal(inc, np.array(want, dtype=np.int32))


def test_assemble_csr_rows_validation_before_launch():
    L = fe.lib()
    p = fe.problem("scalar", "fp64", "uniform", 0, inputs.identity_diffusion_uniform(), "packed")
    rule = fe.builtin_rule("tet4", 1)
    v = lambda a: ctypes.c_void_p(a) if a else None
    call = lambda inc=0x9000, incp=0xa000, vals=0x7000, n=10: L.fe_assemble_csr_rows(
        ctypes.byref(p), 0, n, v(0x8000), 10, v(0x1000), 10, None, 10, ctypes.byref(rule.c),
        v(0x5000), v(0x6000), 100, v(vals), None, v(incp), v(inc), None)
    assert call(inc=0) == 1
    assert call(incp=0) == 1
    assert call(vals=0) == 1
    assert call(inc=0x9002) == 2
    assert call(vals=0x7004) == 2
    assert call(inc=0, incp=0, vals=0, n=0) == 0
    conn = np.zeros((1, 4), dtype=np.int32)
    assert L.fe_node_incidence(0, 1, conn.ctypes.data_as(ctypes.c_void_p), 1, 0,
                               np.zeros(2, dtype=np.int64).ctypes.data_as(ctypes.c_void_p),
                               None) == -1


def test_assemble_csr_stored_validation_before_launch():
    L = fe.lib()
    p = fe.problem("scalar", "fp64", "uniform", 0, inputs.identity_diffusion_uniform(), "packed")
    v = lambda a: ctypes.c_void_p(a) if a else None
    call = lambda K=0x2000, F=0x3000, b=0x4000, ld=10, n=10, inc=0x9000, nn=10: \
        L.fe_assemble_csr_stored(ctypes.byref(p), 0, n, v(0x1000), 10, nn, v(K), v(F), ld, 0,
                                 v(0x5000), v(0x6000), 100, v(0x7000), v(b), v(0xa000), v(inc), None)
    assert call(K=0) == 1
    assert call(F=0) == 1              # F needed with b
    assert call(inc=0) == 1
    assert call(ld=9) == 1
    assert call(nn=0) == 1
    assert call(K=0x2004) == 2         # misaligned
    assert call(n=0, K=0, F=0, inc=0) == 0


def test_assemble_csr_blocks_validation_before_launch():
    L = fe.lib()
    p = fe.problem("scalar", "fp64", "uniform", 0, inputs.identity_diffusion_uniform(), "packed")
    rule = fe.builtin_rule("tet4", 1)
    v = lambda a: ctypes.c_void_p(a) if a else None
    call = lambda elem=0, n=10, nb=2, blk=0x2000, linc=0x3000, vals=0x7000, prob=p: \
        L.fe_assemble_csr_blocks(ctypes.byref(prob), elem, n, v(0x8000), 10, None, 10,
                                 ctypes.byref(rule.c), v(0x5000), v(0x6000), 100, v(vals), None,
                                 v(0xa000), nb, v(blk), v(0x4000), v(0x4800), v(0x5800),
                                 v(linc), None)
    assert call(elem=1) == 2           # prisms: not built
    pe = fe.problem("elasticity", "fp64", "element", (1 << 5) - 1, np.zeros(20), "packed")
    assert call(prob=pe) == 2          # vector problems: not built
    assert call(blk=0) == 1
    assert call(linc=0) == 1
    assert call(vals=0) == 1
    assert call(nb=0) == 1
    assert call(nb=-1) == 1
    assert call(linc=0x3002) == 2      # misaligned codes
    assert call(n=0, nb=0, blk=0, linc=0, vals=0) == 0


def test_stream_pattern_validation():
    L = fe.lib()
    v = lambda a: ctypes.c_void_p(a) if a else None
    call = lambda rin=2, rout=3, ob=8, n=10, ld=10, inp=0x1000, out=0x2000: L.fe_stream_pattern(
        v(inp), rin, v(out), rout, ob, n, ld, None)
    assert call(rin=-1) == 1
    assert call(rout=0) == 1
    assert call(ob=2) == 1
    assert call(ld=9) == 1
    assert call(out=0) == 1
    assert call(inp=0) == 1            # rows to read but no input
    assert call(out=0x2004) == 1       # misaligned for FP64 output
    assert call(n=0) == 0


def test_product_path_fails_loudly_without_the_library(tmp_path):
    # with libfe.so absent the binding raises; nothing falls back to the oracle
    import subprocess
    import sys
    code = (
        "import paper_1504_01023_amd.fe as fe\n"
        f"fe.LIB_PATH = {str(tmp_path / 'libfe.so')!r}\n"
        "fe._lib = None\n"
        "try:\n"
        "    fe.lib()\n"
        "except RuntimeError as e:\n"
        "    print('raised', 'missing' in str(e))\n"
        "import sys\n"
        "print('oracle imported', 'oracle' in sys.modules)\n"
    )
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                         timeout=120)
    assert "raised True" in out.stdout, out.stdout + out.stderr
    assert "oracle imported False" in out.stdout, out.stdout


def test_ld_for_rounds_to_whole_lines():
    assert fe.ld_for(0) == 0
    assert fe.ld_for(1) == 256
    assert fe.ld_for(256) == 256
    assert fe.ld_for(257) == 512
    assert fe.ld_for(10_110_954) == 10_110_976
    assert fe.lib().fe_ld_for(-1) == -1


def test_builtin_tuning_table_is_the_committed_one():
    """The table compiled into the library is tuning_mi355x.txt; it is in
    effect only on its own architecture (never without a device)."""
    import re
    path = os.path.join(ROOT, "paper_1504_01023_amd", "tuning_mi355x.txt")
    text = open(path).read()
    arch = re.search(r"^# arch (\S+)", text, re.M).group(1)
    assert re.search(r"^# rocm (\d+)\.(\d+)", text, re.M)
    on, tab_arch, n = fe.tuning_builtin()
    assert tab_arch == arch == "gfx950"
    if not on:
        assert n == 0
    else:
        assert n == sum(1 for line in text.splitlines() if line and not line.startswith("#"))
