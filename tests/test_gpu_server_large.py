"""The continuous-batching server at the mixed stream's scale: requests of
1e3 to 4e5 elements, each its own jittered mesh (tet cube with N =
round((n/6)^(1/3)), prism layers with n = L = round((n/2)^(1/3))), all eight
kinds of the mix, 4096-element chunks, the default persistent grid and a
multi-GiB budget. Every result matches the oracle on sampled elements and is
bitwise the result of a plain launch of the same kernel on the same layout."""
import time

import numpy as np
import pytest

from paper_1504_01023_amd import fe, inputs, serve
from tests import _parity as P
from tests.test_gpu_server import KIND_WL, fetch, server_kinds

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fe.tuning_clear()
    yield


def request(kind, n_target, seed):
    name, prec = KIND_WL[kind]
    if name.startswith("tet"):
        N = max(1, round((n_target / 6) ** (1 / 3)))
        wl = (inputs.tet_cdr(N, seed=seed) if name == "tet_cdr"
              else inputs.tet_elasticity(N, seed=seed))
    else:
        m = max(1, round((n_target / 2) ** (1 / 3)))
        wl = (inputs.prism_cdr_element(m, m, seed=seed) if name == "prism_cdr"
              else inputs.prism_elasticity(m, m, seed=seed))
    hc = torch.from_numpy(wl.mesh.coords).pin_memory()
    dt = torch.float64 if prec == "fp64" else torch.float32
    hk = torch.from_numpy(wl.coeffs).to(dt).pin_memory()
    return wl, prec, hc, hk


def test_served_at_scale():
    rng = np.random.default_rng(7)
    kinds = server_kinds()
    reqs = []
    for i in range(12):
        kind = i % len(KIND_WL)
        n_target = float(np.exp(rng.uniform(np.log(1e3), np.log(4e5))))
        reqs.append((kind, request(kind, n_target, 900 + i)))
    sizes = [wl.n_elem for _, (wl, _, _, _) in reqs]
    print(f"[served at scale] {len(reqs)} requests, {sum(sizes)} elements, "
          f"largest {max(sizes)}", flush=True)
    assert max(sizes) > 4096 * 8  # many chunks per request
    with serve.Server(kinds, max_slots=16, hbm_budget_bytes=8 << 30, max_chunks=2048,
                      chunk_elems=4096) as srv:
        ids = {}
        for kind, (wl, prec, hc, hk) in reqs:
            ids[srv.submit(kind, wl.n_elem, hc.data_ptr(), hk.data_ptr(), keep=(hc, hk))] = (
                kind, wl, prec)
        got = {}
        t0 = time.time()
        while len(got) < len(ids) and time.time() - t0 < 90:
            for c in srv.poll(64, 0.05):
                kind, wl, prec = ids[c.id]
                assert c.status == 0, c.status
                p = srv.kinds[kind][0]
                dt = torch.float64 if prec == "fp64" else torch.float32
                K = fetch(c.out_K, fe.k_entries(p, wl.elem), c.ld_out, dt)
                F = fetch(c.out_F, fe.f_entries(p, wl.elem), c.ld_out, dt)
                got[c.id] = (wl, prec, K, F, c.ld_out)
                srv.release(c.id)
        assert len(got) == len(ids)
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0 and st["bytes_in_use"] == 0
    srng = np.random.default_rng(11)
    for wl, prec, K, F, ld in got.values():
        n = wl.n_elem
        sample = np.sort(srng.choice(n, size=min(n, 400), replace=False))
        Kn, Fn = K[:, :n].cpu().numpy(), F[:, :n].cpu().numpy()
        Ks = Kn[:, sample]
        Fs = Fn[:, sample]
        # the oracle on the sampled elements
        P.assert_parity(_subset(wl, sample), prec, Ks, Fs)
        # a plain launch of the same kernel on the same layout: the same bits
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


def _subset(wl, idx):
    mesh = inputs.Mesh(wl.elem, np.ascontiguousarray(wl.mesh.coords[:, idx]), wl.mesh.nodes,
                       wl.mesh.conn[idx], wl.mesh.boundary)
    coeffs = np.ascontiguousarray(wl.coeffs[:, idx])
    return inputs.Workload(wl.name, wl.elem, wl.kind, wl.n_q, wl.coef_mode, wl.mask, wl.uniform,
                           wl.k_format, mesh, coeffs)
