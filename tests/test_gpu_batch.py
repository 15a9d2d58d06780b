"""Persistent batched launches (captured HIP graphs over a chunk table):
results of many uneven requests in one launch are bitwise identical to
plain launches of the same kernel variant, and match the oracle."""
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
    fe.tuning_clear()
    yield


def _requests(seed):
    rng = np.random.default_rng(seed)
    reqs = []
    makers = [
        lambda s: inputs.tet_cdr(int(rng.integers(2, 7)), seed=s),
        lambda s: inputs.tet_elasticity(int(rng.integers(2, 6)), seed=s),
        lambda s: inputs.prism_cdr_element(int(rng.integers(2, 8)), int(rng.integers(2, 6)), seed=s),
        lambda s: inputs.prism_elasticity(int(rng.integers(2, 6)), int(rng.integers(2, 5)), seed=s),
        lambda s: inputs.tet_vector(int(rng.integers(2, 5)), seed=s),
        lambda s: inputs.prism_vector(int(rng.integers(2, 5)), int(rng.integers(2, 4)), seed=s),
    ]
    for i in range(18):
        k = int(rng.integers(0, len(makers)))
        prec = "fp64" if rng.random() < 0.5 else "fp32"
        wl = makers[k](100 + i)
        if wl.elem == "tet4" and i % 2 == 0:
            # an odd element count: rows that do not suit two elements per lane
            wl = _prefix(wl, wl.n_elem - 1)
        reqs.append((k, prec, wl))
    return reqs


def _prefix(wl, n):
    """The first n elements of a workload, as a workload of its own."""
    mesh = inputs.Mesh(wl.elem, np.ascontiguousarray(wl.mesh.coords[:, :n]), wl.mesh.nodes,
                       wl.mesh.conn[:n], wl.mesh.boundary)
    return inputs.Workload(wl.name, wl.elem, wl.kind, wl.n_q, wl.coef_mode, wl.mask, wl.uniform,
                           wl.k_format, mesh, np.ascontiguousarray(wl.coeffs[:, :n]))


def _kind_list():
    ks = []
    for prec in ("fp64", "fp32"):
        for wl in (P.small("tet_cdr"), P.small("tet_elasticity"), P.small("prism_cdr"),
                   P.small("prism_elasticity"), P.small("tet_vector"), P.small("prism_vector")):
            ks.append((fe.problem_for(wl, prec), wl.elem, fe.builtin_rule(wl.elem, wl.n_q)))
    return ks


def test_batch_matches_plain_bitwise_and_oracle():
    kinds = _kind_list()
    b = fe.Batch(kinds, max_chunks=256, chunk_elems=256, blocks_per_kind=64)
    reqs = _requests(7)
    outs, plain = [], []
    for k, prec, wl in reqs:
        kind = k + (0 if prec == "fp64" else 6)
        dw = fe.to_device(wl, prec)
        p = kinds[kind][0]
        nk, nf = fe.k_entries(p, wl.elem), fe.f_entries(p, wl.elem)
        dt = torch.float64 if prec == "fp64" else torch.float32
        K = torch.full((nk, wl.n_elem), float("nan"), dtype=dt, device="cuda")
        F = torch.full((nf, wl.n_elem), float("nan"), dtype=dt, device="cuda")
        # odd leading dimensions do not suit two elements per lane: such
        # requests are processed element by element, with the same results
        b.add(kind, dw.coords, dw.coeffs, K, F)
        outs.append((wl, prec, dw, K, F))
    assert len(outs) == len(reqs)
    assert any(wl.n_elem % 2 == 1 and wl.elem == "tet4" for wl, *_ in outs)
    assert b.pending() > 0
    b.launch()
    torch.cuda.synchronize()
    assert b.pending() == 0
    for wl, prec, dw, K, F in outs:
        K2, F2 = fe.integrate(dw.problem, wl.elem, dw.coords, dw.coeffs, dw.rule)
        torch.cuda.synchronize()
        assert torch.equal(K, K2) and torch.equal(F, F2), (wl.name, prec, wl.n_elem)
        P.assert_parity(wl, prec, K.cpu().numpy(), F.cpu().numpy())
    b.close()


def test_batch_replay_and_capacity():
    kinds = _kind_list()[:1]
    b = fe.Batch(kinds, max_chunks=8, chunk_elems=64, blocks_per_kind=16)
    wl = inputs.tet_cdr(4, seed=3)  # 384 elements = 6 chunks
    dw = fe.to_device(wl, "fp64")
    ref = fe.integrate(dw.problem, "tet4", dw.coords, dw.coeffs, dw.rule)
    for rep in range(5):
        K = torch.zeros_like(ref[0])
        F = torch.zeros_like(ref[1])
        b.add(0, dw.coords, dw.coeffs, K, F)
        with pytest.raises(fe.FeError) as ei:   # 6 + 6 chunks > 8
            b.add(0, dw.coords, dw.coeffs, K, F)
        assert ei.value.status == 5
        b.launch()
        torch.cuda.synchronize()
        assert torch.equal(K, ref[0]) and torch.equal(F, ref[1])
    b.launch()  # nothing pending: no-op
    b.close()


def test_batch_rejects_unbatched_kind():
    wl = P.small("prism_cdr_qp")
    k = [(fe.problem_for(wl, "fp64"), wl.elem, fe.builtin_rule(wl.elem, wl.n_q))]
    b = fe.Batch(k, max_chunks=16, chunk_elems=64)   # per-point kinds have batched forms too
    b.close()
    with pytest.raises(fe.FeError):
        fe.Batch(k, max_chunks=16, chunk_elems=63)


def test_batch_falls_back_when_tuned_variant_has_no_batched_form():
    wl = P.small("tet_cdr")
    p = fe.problem_for(wl, "fp64")
    rule = fe.builtin_rule("tet4", 4)
    fe.tuning_clear()
    # one element per lane with caching stores: compiled without a batched form
    fe.tuning_set(p, "tet4", 4, fe.variant(256, 1, 2, 2, 0, 1, 1))
    try:
        b = fe.Batch([(p, "tet4", rule)], max_chunks=16, chunk_elems=256)
        dw = fe.to_device(wl, "fp64")
        K = torch.empty((16, wl.n_elem), dtype=torch.float64, device="cuda")
        F = torch.empty((4, wl.n_elem), dtype=torch.float64, device="cuda")
        b.add(0, dw.coords, dw.coeffs, K, F)
        b.launch()
        torch.cuda.synchronize()
        P.assert_parity(wl, "fp64", K.cpu().numpy(), F.cpu().numpy())
        b.close()
    finally:
        fe.tuning_clear()
