"""GPU parity of CSR assembly on rows longer than the entries a lane holds in
registers: a small tetrahedral mesh plus hubs of extra tetrahedra (positively
oriented, their other three nodes drawn at random) at three nodes, so one row
has far more than 32 entries, another just over 32, and rows of every length
in between occur in the same waves as the 15-entry rows of the mesh. Row
ownership and the stored-matrix gather are checked against the oracle's
assembled matrix, against each other bit for bit, and when adding into values
that already hold a first assembly. FP64 and FP32."""
import numpy as np
import pytest
import torch

from paper_1504_01023_amd import fe, inputs
from tests import _parity as P

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-5}


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fe.lib()
    yield


def _with_hubs(wl, seed):
    rng = np.random.default_rng(seed)
    nodes = wl.mesh.nodes
    nn = nodes.shape[0]
    add = []
    for hub, count in ((0, 60), (nn // 2, 10), (nn - 1, 6)):
        others = np.setdiff1d(np.arange(nn), [hub])
        done = 0
        while done < count:
            a, b, c = (int(x) for x in rng.choice(others, 3, replace=False))
            det = np.linalg.det(nodes[[a, b, c]] - nodes[hub])
            if abs(det) < 1e-3:
                continue
            add.append([hub, a, b, c] if det > 0 else [hub, b, a, c])
            done += 1
    extra = len(add)
    conn = np.concatenate([wl.mesh.conn, np.array(add, dtype=wl.mesh.conn.dtype)])
    n = conn.shape[0]
    coords = np.empty((12, n))
    for v in range(4):
        for d in range(3):
            coords[3 * v + d] = nodes[conn[:, v], d]
    coeffs = wl.coeffs
    if coeffs is not None:
        coeffs = np.ascontiguousarray(
            np.concatenate([coeffs, coeffs[:, rng.integers(0, wl.n_elem, extra)]], axis=1))
    mesh = inputs.Mesh(wl.elem, coords, nodes, conn, wl.mesh.boundary)
    return inputs.Workload(wl.name, wl.elem, wl.kind, wl.n_q, wl.coef_mode, wl.mask, wl.uniform,
                           wl.k_format, mesh, coeffs)


def _dense(rp, ci, vals):
    n = len(rp) - 1
    A = np.zeros((n, n))
    A[np.repeat(np.arange(n), np.diff(rp)), ci] = vals.double().cpu().numpy()
    return A


def _check(A, b, ref, tol, scale_by=1.0):
    Ar, br, Aabs, babs = ref
    Ar, br, Aabs, babs = Ar * scale_by, br * scale_by, Aabs * scale_by, babs * scale_by
    scale = np.maximum(Aabs, Aabs.max(axis=1, keepdims=True))
    inside = Aabs > 0
    e = np.abs(A - Ar)[inside] / scale[inside]
    assert e.max() <= tol, f"A rel err {e.max():.3e}"
    eb = np.abs(b.double().cpu().numpy() - br) / np.maximum(babs, 1e-300)
    assert eb.max() <= tol, f"b rel err {eb.max():.3e}"


@pytest.mark.parametrize("name", ["tet_poisson", "tet_cdr"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_long_rows(name, precision):
    wl = _with_hubs(P.small(name), 5)
    nn = wl.mesh.nodes.shape[0]
    rp, ci = fe.csr_pattern(wl.elem, wl.mesh.conn, nn, 1)
    lens = np.diff(rp)
    print(f"[csr-long] {name} {precision} n={wl.n_elem} nnz={len(ci)} longest row={lens.max()} "
          f"rows over 32={int((lens > 32).sum())}", flush=True)
    assert lens[0] > 64 and (lens > 32).sum() >= 2 and ((lens > 16) & (lens <= 32)).any()
    ref = P.assembly_reference(wl, precision)
    dw = fe.to_device(wl, precision)
    conn = torch.from_numpy(np.ascontiguousarray(wl.mesh.conn.T.astype(np.int32))).cuda()
    nodes = torch.from_numpy(wl.mesh.nodes).cuda().contiguous()
    ip, inc = fe.node_incidence(wl.elem, wl.mesh.conn, nn)
    rows = (torch.from_numpy(ip).cuda(), torch.from_numpy(inc).cuda())
    rpd = torch.from_numpy(rp).cuda()
    cid = torch.from_numpy(ci).cuda()
    v_own, b_own = fe.assemble_csr_rows(dw.problem, wl.elem, nodes, conn, dw.coeffs, dw.rule, rpd,
                                        cid, *rows, with_b=True)
    Ks, Fs = fe.integrate_indexed(dw.problem, wl.elem, nodes, conn, dw.coeffs, dw.rule)
    Kn, Fn = Ks.t().contiguous(), Fs.t().contiguous()
    v_st, b_st = fe.assemble_csr_stored(dw.problem, wl.elem, conn, nn, Ks, Fs, rpd, cid, *rows,
                                        with_b=True)
    v_nm, b_nm = fe.assemble_csr_stored(dw.problem, wl.elem, conn, nn, Kn, Fn, rpd, cid, *rows,
                                        with_b=True, elem_major=True)
    torch.cuda.synchronize()
    _check(_dense(rp, ci, v_own), b_own, ref, TOL[precision])
    _check(_dense(rp, ci, v_st), b_st, ref, TOL[precision])
    assert torch.equal(v_own, v_st) and torch.equal(b_own, b_st)
    assert torch.equal(v_st, v_nm) and torch.equal(b_st, b_nm)
    # a second assembly into the same values: both schedules add to what is
    # there, element by element in the same order
    fe.assemble_csr_rows(dw.problem, wl.elem, nodes, conn, dw.coeffs, dw.rule, rpd, cid, *rows,
                         values=v_own, b=b_own)
    fe.assemble_csr_stored(dw.problem, wl.elem, conn, nn, Kn, Fn, rpd, cid, *rows, values=v_st,
                           b=b_st, elem_major=True)
    torch.cuda.synchronize()
    _check(_dense(rp, ci, v_st), b_st, ref, TOL[precision], scale_by=2.0)
    assert torch.equal(v_own, v_st) and torch.equal(b_own, b_st)
