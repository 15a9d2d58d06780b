"""fe_batch_integrate_static, the batched entry point that allocates
nothing (its chunk table lives in the library's own device array), called
through the C ABI: two calls in a row, the second with a smaller input, each
bitwise equal to the same requests through fe_batch_create / fe_batch_add /
fe_batch_launch (the existing entry point, same kernels), and the first also
against the oracle."""
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
    yield


def _kinds():
    out = []
    for wl, prec in ((P.small("tet_cdr"), "fp64"), (P.small("tet_elasticity"), "fp32"),
                     (P.small("prism_cdr"), "fp64"), (P.small("prism_vector"), "fp32")):
        out.append((fe.problem_for(wl, prec), wl.elem, fe.builtin_rule(wl.elem, wl.n_q)))
    return out


PRECS = ("fp64", "fp32", "fp64", "fp32")


def _make(kind, wl, odd):
    """Device inputs and NaN-filled outputs of one request; `odd` gives its
    rows an odd leading dimension (element-by-element processing)."""
    prec = PRECS[kind]
    dw = fe.to_device(wl, prec)
    n = wl.n_elem
    ld = n + 1 if odd and n % 2 == 0 else n
    dt = torch.float64 if prec == "fp64" else torch.float32

    def pad(t):
        if t is None:
            return None
        out = torch.zeros((t.shape[0], ld), dtype=t.dtype, device="cuda")
        out[:, :n] = t
        return out

    c, k = pad(dw.coords), pad(dw.coeffs)
    p = dw.problem
    K = torch.full((fe.k_entries(p, wl.elem), ld), float("nan"), dtype=dt, device="cuda")
    F = torch.full((fe.f_entries(p, wl.elem), ld), float("nan"), dtype=dt, device="cuda")
    return {"kind": kind, "wl": wl, "prec": prec, "c": c, "k": k, "K": K, "F": F, "n": n}


def _requests(sizes):
    makers = [
        lambda s, m: inputs.tet_cdr(m, seed=s),
        lambda s, m: inputs.tet_elasticity(m, seed=s),
        lambda s, m: inputs.prism_cdr_element(m + 1, m, seed=s),
        lambda s, m: inputs.prism_vector(m, m, seed=s),
    ]
    return [_make(kind, makers[kind](300 + i, m), odd)
            for i, (kind, m, odd) in enumerate(sizes)]


def _via_batch(kinds, reqs, chunk_elems, blocks):
    """The same requests through the existing batched entry point."""
    b = fe.Batch(kinds, max_chunks=fe.BATCH_STATIC_MAX_CHUNKS, chunk_elems=chunk_elems,
                 blocks_per_kind=blocks)
    outs = []
    for r in reqs:
        K = torch.full_like(r["K"], float("nan"))
        F = torch.full_like(r["F"], float("nan"))
        b.add(r["kind"], r["c"], r["k"], K, F, n_elem=r["n"])
        outs.append((K, F))
    b.launch()
    torch.cuda.synchronize()
    b.close()
    return outs


def _check_call(kinds, reqs, chunk_elems, blocks, oracle):
    n_chunks = sum((r["n"] + chunk_elems - 1) // chunk_elems for r in reqs)
    print(f"[no-alloc] {len(reqs)} requests, {n_chunks} chunks of {chunk_elems}", flush=True)
    fe.batch_integrate_static(kinds, [(r["kind"], r["c"], r["k"], r["K"], r["F"], r["n"])
                                      for r in reqs], chunk_elems=chunk_elems,
                              blocks_per_kind=blocks)
    torch.cuda.synchronize()
    ref = _via_batch(kinds, reqs, chunk_elems, blocks)
    for r, (K2, F2) in zip(reqs, ref):
        n = r["n"]
        assert torch.equal(r["K"][:, :n], K2[:, :n]) and torch.equal(r["F"][:, :n], F2[:, :n]), \
            (r["wl"].name, r["prec"], n, r["K"].shape)
        # columns beyond n are never written
        assert torch.isnan(r["K"][:, n:]).all() and torch.isnan(r["F"][:, n:]).all()
        if oracle:
            P.assert_parity(r["wl"], r["prec"], r["K"][:, :n].cpu().numpy(),
                            r["F"][:, :n].cpu().numpy())
    return n_chunks


def test_two_calls_in_a_row_match_the_batched_entry_point():
    kinds = _kinds()
    # first call: every kind, odd and even leading dimensions, more chunks
    # than one table-writing launch carries
    big = _requests([(0, 3, False), (1, 3, True), (2, 3, False), (3, 2, False), (0, 2, True),
                     (2, 2, True), (1, 2, False)])
    n1 = _check_call(kinds, big, chunk_elems=8, blocks=48, oracle=True)
    assert n1 > 60
    # second call right after, smaller: two kinds, fewer chunks, a table
    # shorter than the first call's (stale records must not be read)
    small = _requests([(2, 2, False), (0, 1, True)])
    n2 = _check_call(kinds, small, chunk_elems=8, blocks=48, oracle=False)
    assert n2 < n1


def test_capacity_and_validation_leave_outputs_untouched():
    kinds = _kinds()
    r = _requests([(0, 3, False)])[0]   # 162 elements
    # 162 elements in chunks of 4 -> 41 chunks; 26 copies exceed 1024
    reqs = [(0, r["c"], r["k"], r["K"], r["F"], r["n"])] * 26
    with pytest.raises(fe.FeError) as ei:
        fe.batch_integrate_static(kinds, reqs, chunk_elems=4)
    assert ei.value.status == 5
    with pytest.raises(fe.FeError) as ei:
        fe.batch_integrate_static(kinds, [(7, r["c"], r["k"], r["K"], r["F"], r["n"])])
    assert ei.value.status == 1
    with pytest.raises(fe.FeError) as ei:
        fe.batch_integrate_static(kinds, reqs[:1], chunk_elems=6)
    assert ei.value.status == 1
    torch.cuda.synchronize()
    assert torch.isnan(r["K"]).all() and torch.isnan(r["F"]).all()
    # no requests, or empty ones: nothing to do
    fe.batch_integrate_static(kinds, [])
    fe.batch_integrate_static(kinds, [(0, r["c"], r["k"], r["K"], r["F"], 0)])
    torch.cuda.synchronize()
    assert torch.isnan(r["K"]).all()
    # and a valid call afterwards still matches
    _check_call(kinds, [r], chunk_elems=16, blocks=8, oracle=True)
