"""The continuous-batching server on the GPU: every served result matches the
oracle, and is bitwise the same alone and in the mix (and the same as a
plain launch of the same kernel variant)."""
import ctypes
import time

import numpy as np
import pytest

from paper_1504_01023_amd import fe, inputs, serve
from tests import _parity as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fe.tuning_clear()
    yield


KIND_WL = [("tet_cdr", "fp64"), ("tet_elasticity", "fp64"), ("prism_cdr", "fp64"),
           ("prism_elasticity", "fp64"), ("tet_cdr", "fp32"), ("tet_elasticity", "fp32"),
           ("prism_cdr", "fp32"), ("prism_elasticity", "fp32")]


def server_kinds():
    out = []
    for name, prec in KIND_WL:
        wl = P.small(name)
        out.append((fe.problem_for(wl, prec), wl.elem, fe.builtin_rule(wl.elem, wl.n_q)))
    return out


def make_request(kind, seed):
    rng = np.random.default_rng(seed)
    name, prec = KIND_WL[kind]
    if name == "tet_cdr":
        wl = inputs.tet_cdr(int(rng.integers(2, 9)), seed=seed)
    elif name == "tet_elasticity":
        wl = inputs.tet_elasticity(int(rng.integers(2, 9)), seed=seed)
    elif name == "prism_cdr":
        wl = inputs.prism_cdr_element(int(rng.integers(2, 12)), int(rng.integers(2, 8)), seed=seed)
    else:
        wl = inputs.prism_elasticity(int(rng.integers(2, 9)), int(rng.integers(2, 6)), seed=seed)
    # a random prefix of the mesh, so sizes are ragged
    n = int(rng.integers(1, wl.n_elem + 1))
    mesh = inputs.Mesh(wl.elem, np.ascontiguousarray(wl.mesh.coords[:, :n]), wl.mesh.nodes,
                       wl.mesh.conn[:n], wl.mesh.boundary)
    coeffs = np.ascontiguousarray(wl.coeffs[:, :n])
    wl = inputs.Workload(wl.name, wl.elem, wl.kind, wl.n_q, wl.coef_mode, wl.mask, wl.uniform,
                         wl.k_format, mesh, coeffs)
    hc = torch.from_numpy(wl.mesh.coords).pin_memory()
    dt = torch.float64 if prec == "fp64" else torch.float32
    hk = torch.from_numpy(wl.coeffs).to(dt).pin_memory()
    return wl, prec, hc, hk


def fetch(ptr, rows, ld, dt):
    """Copy a server-owned device array into a torch tensor."""
    out = torch.empty((rows, ld), dtype=dt, device="cuda")
    nbytes = out.numel() * out.element_size()
    st = fe.lib().fe_stream_copy(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ptr), nbytes,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    torch.cuda.synchronize()
    return out


def run_and_collect(srv, reqs):
    ids = {}
    for kind, (wl, prec, hc, hk) in reqs:
        rid = srv.submit(kind, wl.n_elem, hc.data_ptr(), hk.data_ptr(), keep=(hc, hk))
        ids[rid] = (kind, wl, prec)
    res = {}
    t0 = time.time()
    while len(res) < len(ids) and time.time() - t0 < 60:
        for c in srv.poll(64, 0.05):
            kind, wl, prec = ids[c.id]
            assert c.status == 0, c.status
            p = srv.kinds[kind][0]
            dt = torch.float64 if prec == "fp64" else torch.float32
            K = fetch(c.out_K, fe.k_entries(p, wl.elem), c.ld_out, dt)
            F = fetch(c.out_F, fe.f_entries(p, wl.elem), c.ld_out, dt)
            res[c.id] = (kind, wl, prec, K, F, c.ld_out)
            srv.release(c.id)
    assert len(res) == len(ids)
    return res


def test_served_mix_matches_oracle_and_is_identical_alone():
    kinds = server_kinds()
    reqs = [(k, make_request(k, 500 + i)) for i, k in
            enumerate(np.random.default_rng(3).integers(0, len(KIND_WL), 24))]
    with serve.Server(kinds, max_slots=8, hbm_budget_bytes=1 << 30, max_chunks=64,
                      chunk_elems=512, blocks_per_kind=64) as srv:
        mix = run_and_collect(srv, reqs)
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0 and st["bytes_in_use"] == 0
        # the same requests one at a time
        alone = {}
        for item in reqs[:10]:
            alone.update(run_and_collect(srv, [item]))
    by_tag = {}
    for _, (kind, wl, prec, K, F, ld) in mix.items():
        n = wl.n_elem
        Kn, Fn = K[:, :n].cpu().numpy(), F[:, :n].cpu().numpy()
        P.assert_parity(wl, prec, Kn, Fn)
        by_tag[id(wl)] = (K[:, :n], F[:, :n])
        # plain launch of the same variant on the same layout: bitwise equal
        dw = fe.to_device(wl, prec)
        ci = torch.zeros((dw.coords.shape[0], ld), dtype=torch.float64, device="cuda")
        ci[:, :n] = dw.coords
        ki = torch.zeros((dw.coeffs.shape[0], ld), dtype=dw.coeffs.dtype, device="cuda")
        ki[:, :n] = dw.coeffs
        K2 = torch.empty_like(K)
        F2 = torch.empty_like(F)
        fe.integrate(dw.problem, wl.elem, ci, ki, dw.rule, out_K=K2, out_F=F2, n_elem=n)
        torch.cuda.synchronize()
        assert torch.equal(K2[:, :n], K[:, :n]) and torch.equal(F2[:, :n], F[:, :n])
    for _, (kind, wl, prec, K, F, ld) in alone.items():
        Km, Fm = by_tag[id(wl)]
        n = wl.n_elem
        assert torch.equal(K[:, :n], Km) and torch.equal(F[:, :n], Fm)


def test_device_inputs_in_place():
    kinds = server_kinds()
    wl, prec, hc, hk = make_request(0, 77)
    n = wl.n_elem
    ld = (n + 3) // 4 * 4
    dc = torch.zeros((hc.shape[0], ld), dtype=torch.float64, device="cuda")
    dc[:, :n] = hc.cuda()
    dk = torch.zeros((hk.shape[0], ld), dtype=hk.dtype, device="cuda")
    dk[:, :n] = hk.cuda()
    torch.cuda.synchronize()
    with serve.Server(kinds, max_slots=2, hbm_budget_bytes=1 << 28, max_chunks=16,
                      chunk_elems=256) as srv:
        rid = srv.submit(0, n, dc.data_ptr(), dk.data_ptr(), on_device=True, ld_in=ld)
        got = []
        t0 = time.time()
        while not got and time.time() - t0 < 30:
            got = srv.poll(4, 0.05)
        c = got[0]
        assert c.id == rid and c.status == 0
        p = kinds[0][0]
        K = fetch(c.out_K, fe.k_entries(p, "tet4"), c.ld_out, torch.float64)[:, :n]
        F = fetch(c.out_F, fe.f_entries(p, "tet4"), c.ld_out, torch.float64)[:, :n]
        P.assert_parity(wl, prec, K.cpu().numpy(), F.cpu().numpy())
        srv.release(rid)
        # device inputs whose leading dimension does not suit two elements per
        # lane are processed element by element: the same results
        if n > 2:
            dc2 = torch.zeros((hc.shape[0], ld - 1), dtype=torch.float64, device="cuda")
            dc2[:, :n - 1] = dc[:, :n - 1]
            dk2 = torch.zeros((hk.shape[0], ld - 1), dtype=hk.dtype, device="cuda")
            dk2[:, :n - 1] = dk[:, :n - 1]
            torch.cuda.synchronize()
            rid2 = srv.submit(0, n - 1, dc2.data_ptr(), dk2.data_ptr(), on_device=True,
                              ld_in=ld - 1)
            got = []
            t0 = time.time()
            while not got and time.time() - t0 < 30:
                got = srv.poll(4, 0.05)
            c2 = got[0]
            assert c2.id == rid2 and c2.status == 0
            K2 = fetch(c2.out_K, fe.k_entries(p, "tet4"), c2.ld_out, torch.float64)[:, :n - 1]
            F2 = fetch(c2.out_F, fe.f_entries(p, "tet4"), c2.ld_out, torch.float64)[:, :n - 1]
            assert torch.equal(K2, K[:, :n - 1]) and torch.equal(F2, F[:, :n - 1])
            srv.release(rid2)
