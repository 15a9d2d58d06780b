"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element
by element, on seeded inputs; plus indexing, ordering and determinism checks.
"""
import numpy as np
import pytest

from paper_1504_01023_amd import fe, inputs
from tests import _parity as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fe.lib()
    yield


@pytest.mark.parametrize("name", sorted(P.SMALL))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_small_parity(name, precision):
    wl = P.small(name)
    print(f"[parity] {name} {precision} n={wl.n_elem}", flush=True)
    K, F = P.gpu_raw(wl, precision)
    P.assert_parity(wl, precision, K, F)


VARIANTS = [
    dict(wg_size=wg, elems_per_thread=v, nontemporal=nt, ref_in_lds=ref, blocks=b, row_split=sp)
    for wg in (64, 128, 256) for v in (1, 2, 4) for nt in (1, 2, 3) for ref in (1, 2) for b in (0, 7)
    for sp in (1, 2, 3)
]
# the SQS / SSQ loop orders and the lane-split point loop sum in a different
# order: parity, not bitwise
ORDER_VARIANTS = [dict(wg_size=wg, nontemporal=nt, loop_order=o)
                  for wg in (64, 256) for nt in (1, 2) for o in (2, 3)]
ORDER_VARIANTS += [dict(wg_size=wg, lanes=g, blocks=b) for wg in (64, 256) for g in (2, 3, 6)
                   for b in (0, 3)]


@pytest.mark.parametrize("name", ["tet_poisson", "tet_cdr", "prism_cdr_qp", "tet_elasticity",
                                  "prism_elasticity", "tet_poisson_qp", "tet_vector",
                                  "prism_vector"])
def test_every_compiled_variant(name):
    """Force every launch variant the library accepts and compare each with
    the oracle; variants not compiled for this family are refused (status 2)
    without launching."""
    wl = P.small(name)
    dw = fe.to_device(wl, "fp64")
    Ko, Fo = P.oracle_run(wl, "fp64")
    ran = 0
    for kw in VARIANTS + ORDER_VARIANTS:
        v = fe.variant(**kw)
        try:
            K, F = fe.integrate(dw.problem, wl.elem, dw.coords, dw.coeffs, dw.rule, variant=v)
        except fe.FeError as e:
            assert e.status == 2
            continue
        torch.cuda.synchronize()
        Kg, Fg = P.to_full(K.cpu().numpy(), F.cpu().numpy(), wl)
        ek, ef = P.rel_errors(Kg, Fg, Ko, Fo)
        assert ek.max() <= 1e-12 and ef.max() <= 1e-12, (kw, ek.max(), ef.max())
        ran += 1
    assert ran >= 4


@pytest.mark.parametrize("n", [1, 2, 3, 5, 11, 21, 22, 63, 64, 65, 255, 257, 1001])
@pytest.mark.parametrize("lanes", [0, 2, 3, 6])
def test_lane_split_ragged_sizes(lanes, n):
    """Lane-split prism kernels on sizes that end inside a wavefront's group
    of 64 / G elements, with one and several wavefronts per workgroup."""
    wl = P.small("prism_cdr")
    idx = np.arange(n)
    sub = inputs.Workload(wl.name, wl.elem, wl.kind, wl.n_q, wl.coef_mode, wl.mask, wl.uniform,
                          wl.k_format,
                          inputs.Mesh(wl.elem, np.ascontiguousarray(wl.mesh.coords[:, idx]),
                                      wl.mesh.nodes, wl.mesh.conn[idx], wl.mesh.boundary),
                          np.ascontiguousarray(wl.coeffs[:, idx]))
    for wg, blocks in ((64, 0), (256, 0), (128, 1)):
        K, F = P.gpu_raw(sub, "fp64", variant=fe.variant(wg_size=wg, lanes=lanes, blocks=blocks))
        P.assert_parity(sub, "fp64", K, F)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 63, 64, 65, 255, 257, 1001])
@pytest.mark.parametrize("name", ["tet_cdr", "tet_poisson", "prism_cdr_qp", "tet_vector"])
def test_ragged_sizes(name, n):
    wl = P.small(name)
    idx = np.arange(n)
    sub = inputs.Workload(wl.name, wl.elem, wl.kind, wl.n_q, wl.coef_mode, wl.mask, wl.uniform,
                          wl.k_format,
                          inputs.Mesh(wl.elem, np.ascontiguousarray(wl.mesh.coords[:, idx]),
                                      wl.mesh.nodes, wl.mesh.conn[idx], wl.mesh.boundary),
                          None if wl.coeffs is None else np.ascontiguousarray(wl.coeffs[:, idx]))
    for v in (None, fe.variant(elems_per_thread=1), fe.variant(elems_per_thread=2, wg_size=64),
              fe.variant(elems_per_thread=4, blocks=3)):
        try:
            K, F = P.gpu_raw(sub, "fp64", variant=v)
        except fe.FeError as e:
            assert e.status == 2
            continue
        P.assert_parity(sub, "fp64", K, F)


def test_strided_slice_in_place():
    """fe_integrate_ex on a sub-range of a larger batch (pointer offset, ld of
    the whole batch): only the slice's columns of the outputs change."""
    wl = P.small("tet_cdr")
    dw = fe.to_device(wl, "fp64")
    n = wl.n_elem
    p = dw.problem
    nk, nf = fe.k_entries(p, "tet4"), fe.f_entries(p, "tet4")
    K = torch.full((nk, n), -7.0, dtype=torch.float64, device="cuda")
    F = torch.full((nf, n), -7.0, dtype=torch.float64, device="cuda")
    e0, m = 130, 517
    import ctypes
    L = fe.lib()
    ld_in = dw.coords.stride(0)
    st = L.fe_integrate_ex(ctypes.byref(p), 0, m, ctypes.c_void_p(dw.coords.data_ptr() + 8 * e0),
                           ctypes.c_void_p(dw.coeffs.data_ptr() + 8 * e0), ld_in,
                           ctypes.byref(dw.rule.c), ctypes.c_void_p(K.data_ptr() + 8 * e0),
                           ctypes.c_void_p(F.data_ptr() + 8 * e0), n, None,
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, L.fe_last_error()
    torch.cuda.synchronize()
    Kn, Fn = K.cpu().numpy(), F.cpu().numpy()
    assert np.all(Kn[:, :e0] == -7.0) and np.all(Kn[:, e0 + m:] == -7.0)
    assert np.all(Fn[:, :e0] == -7.0) and np.all(Fn[:, e0 + m:] == -7.0)
    sel = np.arange(e0, e0 + m)
    P.assert_parity(wl, "fp64", Kn, Fn, elements=sel)


def test_empty_batch_with_tensors():
    wl = P.small("tet_poisson")
    dw = fe.to_device(wl, "fp64")
    K = torch.full((10, 4), 3.0, dtype=torch.float64, device="cuda")
    F = torch.full((4, 4), 3.0, dtype=torch.float64, device="cuda")
    fe.integrate(dw.problem, "tet4", dw.coords, None, dw.rule, out_K=K, out_F=F, n_elem=0)
    torch.cuda.synchronize()
    assert torch.all(K == 3.0) and torch.all(F == 3.0)


def test_sentinel_element_id_indexing():
    """d^0 = element id per element: F_r(e) = e * V_e / 4 (1-point rule on
    tets); any indexing slip shows up as a wrong element's value."""
    mesh = inputs.tet_cube(6, 21)
    n = mesh.n_elem
    wl = inputs.Workload("sentinel", "tet4", "scalar", 1, "element", 1 << 16, np.zeros(20),
                         "full", mesh, np.arange(n, dtype=np.float64)[None, :])
    K, F = P.gpu_raw(wl, "fp64")
    P.assert_parity(wl, "fp64", K, F)
    Fo = P.oracle_run(wl)[1]
    # the element id is recovered exactly (to rounding) from every element
    vol4 = P.oracle_run(inputs.Workload("v", "tet4", "scalar", 1, "uniform", 0,
                                        np.eye(1, 20, 16)[0], "full", mesh, None))[1]
    ids = (F.T / vol4).mean(axis=1)
    assert np.all(np.abs(ids - np.arange(n)) < 1e-6 * (1 + np.arange(n)))
    assert np.allclose(F.T, Fo, rtol=1e-12, atol=0)


@pytest.mark.parametrize("name", ["tet_cdr", "prism_cdr_qp", "tet_elasticity", "prism_vector"])
def test_permutation_equivariance_bit_exact(name):
    wl = P.small(name)
    K0, F0 = P.gpu_raw(wl, "fp64", variant=fe.variant(elems_per_thread=1))
    p = np.random.default_rng(5).permutation(wl.n_elem)
    sub = inputs.Workload(wl.name, wl.elem, wl.kind, wl.n_q, wl.coef_mode, wl.mask, wl.uniform,
                          wl.k_format,
                          inputs.Mesh(wl.elem, np.ascontiguousarray(wl.mesh.coords[:, p]),
                                      wl.mesh.nodes, wl.mesh.conn[p], wl.mesh.boundary),
                          None if wl.coeffs is None else np.ascontiguousarray(wl.coeffs[:, p]))
    K1, F1 = P.gpu_raw(sub, "fp64", variant=fe.variant(elems_per_thread=1))
    assert np.array_equal(K1, K0[:, p]) and np.array_equal(F1, F0[:, p])


@pytest.mark.parametrize("name", ["tet_poisson", "prism_cdr_qp"])
def test_run_to_run_bitwise_determinism(name):
    wl = P.small(name)
    a = P.gpu_raw(wl, "fp64")
    b = P.gpu_raw(wl, "fp64")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_caller_supplied_rules():
    """Rules are caller arguments: a non-built-in 8-point prism rule (2x2
    Gauss in the triangle's collapsed square times 2-point Gauss) and a
    2-point tet rule run through the runtime point loop."""
    from tests import _witness as W
    xi, w = W.collapsed_prism_rule(2, 2)
    wl = P.small("prism_cdr")
    rule = fe.Rule(xi, w)
    K, F = P.gpu_raw(wl, "fp64", rule=rule)
    Kg, Fg = P.to_full(K, F, wl)
    import oracle
    Ko, Fo = oracle.integrate(wl.elem, wl.kind, wl.mesh.coords, (xi, w), wl.coef_mode, wl.mask,
                              wl.uniform, wl.coeffs, P.ORACLE_THREADS)
    ek, ef = P.rel_errors(Kg, Fg, Ko, Fo)
    assert ek.max() <= 1e-12 and ef.max() <= 1e-12


def test_autotune_then_parity():
    wl = P.small("tet_cdr")
    dw = fe.to_device(wl, "fp64")
    nk, nf = fe.k_entries(dw.problem, "tet4"), fe.f_entries(dw.problem, "tet4")
    K = torch.empty((nk, wl.n_elem), dtype=torch.float64, device="cuda")
    F = torch.empty((nf, wl.n_elem), dtype=torch.float64, device="cuda")
    fe.tuning_clear()
    best, ms = fe.autotune(dw.problem, "tet4", dw.coords, dw.coeffs, dw.rule, K, F, reps=2)
    assert ms > 0 and best[0] in (64, 128, 256)
    assert fe.tuning_get(dw.problem, "tet4", 4) == best
    P.assert_parity(wl, "fp64", K.cpu().numpy(), F.cpu().numpy())
    K2, F2 = fe.integrate(dw.problem, "tet4", dw.coords, dw.coeffs, dw.rule)
    torch.cuda.synchronize()
    P.assert_parity(wl, "fp64", K2.cpu().numpy(), F2.cpu().numpy())
    fe.tuning_clear()


def test_stream_copy():
    x = torch.arange(1 << 20, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    fe.stream_copy(y, x)
    torch.cuda.synchronize()
    assert torch.equal(x, y)


@pytest.mark.parametrize("name", ["tet_poisson", "tet_cdr", "tet_elasticity", "prism_cdr_qp",
                                  "prism_elasticity", "tet_vector", "prism_vector"])
def test_variants_are_bitwise_identical(name):
    """Every compiled variant of a family (elements per lane, cache policy,
    reference-table placement, workgroup and grid shape, row split) performs
    the same per-element rounding sequence, so all outputs agree bit for bit
    (on an odd element count, which also exercises the partial last group)."""
    wl = P.small(name)
    n = wl.n_elem - (1 - wl.n_elem % 2)
    dw = fe.to_device(wl, "fp64")
    ld = (wl.n_elem + 3) // 4 * 4
    c = torch.zeros((dw.coords.shape[0], ld), dtype=torch.float64, device="cuda")
    c[:, :wl.n_elem] = dw.coords
    k = None
    if dw.coeffs is not None:
        k = torch.zeros((dw.coeffs.shape[0], ld), dtype=dw.coeffs.dtype, device="cuda")
        k[:, :wl.n_elem] = dw.coeffs
    nk, nf = fe.k_entries(dw.problem, wl.elem), fe.f_entries(dw.problem, wl.elem)
    ref = None
    for kw in VARIANTS:
        K = torch.full((nk, ld), 7.0, dtype=torch.float64, device="cuda")
        F = torch.full((nf, ld), 7.0, dtype=torch.float64, device="cuda")
        try:
            fe.integrate(dw.problem, wl.elem, c, k, dw.rule, out_K=K, out_F=F, n_elem=n,
                         variant=fe.variant(**kw))
        except fe.FeError as e:
            assert e.status == 2
            continue
        torch.cuda.synchronize()
        assert torch.all(K[:, n:] == 7.0) and torch.all(F[:, n:] == 7.0)
        if ref is None:
            ref = (K, F)
        else:
            assert torch.equal(K, ref[0]) and torch.equal(F, ref[1]), kw


@pytest.mark.parametrize("name", ["tet_poisson", "tet_cdr", "tet_elasticity", "prism_cdr_qp",
                                  "prism_elasticity", "tet_vector", "prism_vector"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_indexed_geometry(name, precision):
    """Coordinates gathered from the node array through the connectivity give
    bit for bit the results of per-element coordinates (same arithmetic on
    the same values), and so match the oracle."""
    wl = P.small(name)
    dw = fe.to_device(wl, precision)
    nodes = torch.from_numpy(wl.mesh.nodes).cuda().contiguous()
    conn = torch.from_numpy(np.ascontiguousarray(wl.mesh.conn.T.astype(np.int32))).cuda()
    for v in (None, fe.variant(elems_per_thread=1), fe.variant(elems_per_thread=2, nontemporal=2)):
        try:
            K0, F0 = fe.integrate(dw.problem, wl.elem, dw.coords, dw.coeffs, dw.rule, variant=v)
            K1, F1 = fe.integrate_indexed(dw.problem, wl.elem, nodes, conn, dw.coeffs, dw.rule,
                                          variant=v)
        except fe.FeError as e:
            assert e.status == 2
            continue
        torch.cuda.synchronize()
        assert torch.equal(K0, K1) and torch.equal(F0, F1)
    P.assert_parity(wl, precision, K1.cpu().numpy(), F1.cpu().numpy())


def test_indexed_geometry_clamps_bad_ids():
    wl = P.small("tet_poisson")
    dw = fe.to_device(wl, "fp64")
    nodes = torch.from_numpy(wl.mesh.nodes).cuda().contiguous()
    c = wl.mesh.conn.T.astype(np.int32).copy()
    c[0, 5] = -3
    c[2, 7] = 10 ** 9
    conn = torch.from_numpy(c).cuda()
    K, F = fe.integrate_indexed(dw.problem, wl.elem, nodes, conn, None, dw.rule)
    torch.cuda.synchronize()
    good = np.setdiff1d(np.arange(wl.n_elem), [5, 7])
    P.assert_parity(wl, "fp64", K.cpu().numpy(), F.cpu().numpy(), elements=good)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_symmetric_full_storage(precision):
    """A symmetric prism problem asked for full K accumulates the upper
    triangle and stores both halves: the stored matrix is exactly symmetric,
    and matches the oracle and the plain full-K (SQS order) kernel."""
    wl = P.small("prism_poisson_qp")
    K, F = P.gpu_raw(wl, precision)
    Kf, _ = P.to_full(K, F, wl)
    assert np.array_equal(Kf, np.transpose(Kf, (0, 2, 1)))
    P.assert_parity(wl, precision, K, F)
    K2, F2 = P.gpu_raw(wl, precision, variant=fe.variant(loop_order=2))
    tol = P.TOL[precision]
    assert np.abs(K2 - K).max() <= tol * np.abs(K).max() * 10
