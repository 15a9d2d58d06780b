"""GPU parity at leading dimensions whose row offsets row * ld + e pass 2^32
elements: a ragged number of elements in the first columns of very wide
inputs and outputs, against the oracle, with every output column past them
left as it was. This exercises the largest index arithmetic of the SoA
streams (tens of GB per array; uninitialised input columns are never read)."""
import numpy as np
import pytest

from paper_1504_01023_amd import fe
from tests import _parity as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SENTINEL = -7.25
# (workload, precision, leading dimension): the largest row offset is
# (rows - 1) * ld, beyond 2^32 in every case
CASES = [
    ("tet_poisson", "fp64", 2 ** 29 + 64),       # coordinates: 11 * ld = 5.9e9
    ("tet_cdr", "fp32", 2 ** 28 + 64),           # coefficients: 19 * ld = 5.1e9
    ("prism_cdr_qp", "fp64", 2 ** 26 + 64),      # per-point coefficients: 119 * ld = 8.0e9
    ("prism_elasticity", "fp32", 2 ** 25 + 64),  # packed K: 170 * ld = 5.7e9
]


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fe.lib()
    yield
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name,precision,ld", CASES)
def test_wide_rows_match_oracle(name, precision, ld):
    wl = P.small(name)
    n = wl.n_elem - 5
    assert (wl.n_elem and n > 0)
    dw = fe.to_device(wl, precision)
    print(f"[large] {name} {precision} n={n} ld={ld}", flush=True)
    coords = torch.empty((dw.coords.shape[0], ld), dtype=torch.float64, device="cuda")
    coords[:, :n] = dw.coords[:, :n]
    coeffs = None
    if dw.coeffs is not None:
        coeffs = torch.empty((dw.coeffs.shape[0], ld), dtype=dw.coeffs.dtype, device="cuda")
        coeffs[:, :n] = dw.coeffs[:, :n]
    dt = torch.float64 if precision == "fp64" else torch.float32
    nk = fe.k_entries(dw.problem, wl.elem)
    nf = fe.f_entries(dw.problem, wl.elem)
    K = torch.full((nk, ld), SENTINEL, dtype=dt, device="cuda")
    F = torch.full((nf, ld), SENTINEL, dtype=dt, device="cuda")
    fe.integrate(dw.problem, wl.elem, coords, coeffs, dw.rule, K, F, n_elem=n)
    torch.cuda.synchronize()
    Kh = K[:, :n].cpu().numpy()
    Fh = F[:, :n].cpu().numpy()
    untouched = all(bool(torch.all(t[:, lo:hi] == SENTINEL))
                    for t in (K, F) for lo, hi in ((n, n + 300), (ld - 300, ld)))
    del coords, coeffs, K, F
    torch.cuda.empty_cache()
    assert untouched
    P.assert_parity(wl, precision, Kh, Fh, elements=np.arange(n))


def test_indexed_geometry_high_node_ids_and_wide_connectivity():
    # node ids near 2^30 in a node array of 25.8 GB, connectivity rows of
    # 2^31 - 64 entries (largest offset 3 * ld = 6.4e9)
    wl = P.small("tet_cdr")
    n = wl.n_elem - 3
    nn = wl.mesh.nodes.shape[0]
    base = 2 ** 30 - nn // 2
    n_nodes = base + nn + 1000
    ld = 2 ** 31 - 64
    dw = fe.to_device(wl, "fp64")
    print(f"[large] indexed tet_cdr n={n} node ids from {base} ld_conn={ld}", flush=True)
    nodes = torch.empty((n_nodes, 3), dtype=torch.float64, device="cuda")
    nodes[base:base + nn] = torch.from_numpy(wl.mesh.nodes).cuda()
    conn = torch.empty((4, ld), dtype=torch.int32, device="cuda")
    conn[:, :n] = torch.from_numpy(np.ascontiguousarray(wl.mesh.conn[:n].T + base).astype(np.int32)).cuda()
    K, F = fe.integrate_indexed(dw.problem, wl.elem, nodes, conn, dw.coeffs[:, :n].contiguous(),
                                dw.rule, n_elem=n)
    torch.cuda.synchronize()
    Kh, Fh = K.cpu().numpy(), F.cpu().numpy()
    del nodes, conn, K, F
    torch.cuda.empty_cache()
    P.assert_parity(wl, "fp64", Kh, Fh, elements=np.arange(n))
