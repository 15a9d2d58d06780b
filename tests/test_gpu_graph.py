"""The entry points only enqueue kernels (no allocation, no memset, no
synchronisation), so a caller can capture them in a HIP graph: integration,
matrix-free application and CSR assembly captured once in a torch CUDA graph
(outputs cleared with fill kernels inside the graph), replayed several times
with eager work between the replays, give the eager results bit for bit on
every replay."""
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


def test_captured_graph_replays_match_eager():
    wl = P.small("tet_cdr")
    dw = fe.to_device(wl, "fp64")
    nn = wl.mesh.nodes.shape[0]
    perm, ptr = fe.color_elements(wl.elem, wl.mesh.conn, nn)
    conn = torch.from_numpy(np.ascontiguousarray(wl.mesh.conn[perm].T.astype(np.int32))).cuda()
    coeffs = dw.coeffs[:, torch.from_numpy(perm.astype(np.int64)).cuda()].contiguous()
    nodes = torch.from_numpy(wl.mesh.nodes).cuda().contiguous()
    x = torch.from_numpy(np.random.default_rng(5).standard_normal(nn)).cuda()
    rp, ci = fe.csr_pattern(wl.elem, wl.mesh.conn, nn, 1)
    ip, inc = fe.node_incidence(wl.elem, wl.mesh.conn[perm], nn)
    rpd, cid = torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()
    ipd, incd = torch.from_numpy(ip).cuda(), torch.from_numpy(inc).cuda()
    K = torch.empty((16, wl.n_elem), dtype=torch.float64, device="cuda")
    F = torch.empty((4, wl.n_elem), dtype=torch.float64, device="cuda")
    y = torch.empty(nn, dtype=torch.float64, device="cuda")
    vals = torch.empty(len(ci), dtype=torch.float64, device="cuda")

    def work():
        fe.integrate(dw.problem, wl.elem, dw.coords, dw.coeffs, dw.rule, out_K=K, out_F=F)
        y.zero_()
        fe.apply_indexed(dw.problem, wl.elem, nodes, conn, coeffs, dw.rule, x, y, None,
                         color_ptr=ptr)
        vals.zero_()
        fe.assemble_csr_rows(dw.problem, wl.elem, nodes, conn, coeffs, dw.rule, rpd, cid, ipd,
                             incd, values=vals)

    # eager reference (and a warm-up outside capture)
    work()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (K, F, y, vals)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        work()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        work()
    torch.cuda.synchronize()
    for rep in range(4):
        for t in (K, F, y, vals):
            t.fill_(float("nan"))
        # eager work of the program between replays
        scratch = torch.randn(1 << 20, device="cuda") * 2.0
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for t, r in zip((K, F, y, vals), ref):
            assert torch.equal(t, r), rep
        del scratch
    P.assert_parity(wl, "fp64", K.cpu().numpy(), F.cpu().numpy())
