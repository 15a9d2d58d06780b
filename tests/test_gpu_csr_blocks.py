"""GPU: the row-ownership assembly over node blocks (fe_assemble_csr_blocks,
elements and vertices staged in LDS per workgroup) equals the plain
row-ownership assembly (fe_assemble_csr_rows) bit for bit, values and load
vector, for the scalar tetrahedral problems in both tiers, in generator and
Z order, with accumulation into nonzero values, on ragged element counts and
with hub nodes whose rows exceed the registers; and, through that equality,
the oracle's assembled matrix (tests/test_gpu_csr.py checks the plain form
against it); plus a direct oracle check on one case."""
import numpy as np
import pytest

from paper_1504_01023_amd import fe, inputs
from tests import _parity as P
from tests.test_gpu_csr_long_rows import _with_hubs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = ["tet_poisson", "tet_poisson_qp", "tet_cdr", "tet_cdr_fn", "tet_cdr_morton"]


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fe.lib()
    yield


def _small(name):
    if name.endswith("_morton"):
        return inputs.reordered(P.small(name[: -len("_morton")]))
    return P.small(name)


def _both(wl, precision, init=None):
    """(rows values, rows b, blocks values, blocks b) on the same inputs."""
    nn = wl.mesh.nodes.shape[0]
    dw = fe.to_device(wl, precision)
    conn = torch.from_numpy(np.ascontiguousarray(wl.mesh.conn.T.astype(np.int32))).cuda()
    nodes = torch.from_numpy(wl.mesh.nodes).cuda().contiguous()
    rp, ci = fe.csr_pattern(wl.elem, wl.mesh.conn, nn, 1)
    ip, inc = fe.node_incidence(wl.elem, wl.mesh.conn, nn)
    bl = fe.csr_blocks(wl.elem, wl.mesh.conn, nn, ip, inc, rp, ci)
    rpd, cid = torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()
    ipd, incd = torch.from_numpy(ip).cuda(), torch.from_numpy(inc).cuda()
    dt = torch.float64 if precision == "fp64" else torch.float32

    def start():
        v = torch.zeros(len(ci), dtype=dt, device="cuda")
        b = torch.zeros(nn, dtype=dt, device="cuda")
        if init is not None:
            g = torch.Generator(device="cpu").manual_seed(init)
            v.copy_(torch.rand(len(ci), generator=g, dtype=torch.float64).to(dt))
            b.copy_(torch.rand(nn, generator=g, dtype=torch.float64).to(dt))
        return v, b

    v1, b1 = start()
    fe.assemble_csr_rows(dw.problem, wl.elem, nodes, conn, dw.coeffs, dw.rule, rpd, cid, ipd,
                         incd, values=v1, b=b1)
    v2, b2 = start()
    print(f"[csr blocks] {wl.name} {precision} n={wl.n_elem} nodes={nn} blocks={bl.n_blocks}",
          flush=True)
    fe.assemble_csr_blocks(dw.problem, wl.elem, nodes, dw.coeffs, dw.rule, rpd, cid, ipd,
                           bl.to("cuda"), values=v2, b=b2)
    torch.cuda.synchronize()
    return v1, b1, v2, b2, (rp, ci)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_blocks_equal_rows_bitwise(name, precision):
    v1, b1, v2, b2, _ = _both(_small(name), precision)
    assert torch.equal(v1, v2) and torch.equal(b1, b2)


def test_blocks_accumulate_into_values():
    v1, b1, v2, b2, _ = _both(_small("tet_cdr"), "fp64", init=11)
    assert torch.equal(v1, v2) and torch.equal(b1, b2)


def test_blocks_many_blocks_morton():
    wl = inputs.reordered(inputs.tet_cdr(12, 2), "morton")
    v1, b1, v2, b2, _ = _both(wl, "fp64")
    assert torch.equal(v1, v2) and torch.equal(b1, b2)


def test_blocks_ragged_element_count():
    wl = P.small("tet_poisson")
    m = wl.n_elem - 37
    mesh = inputs.Mesh(wl.elem, wl.mesh.coords[:, :m], wl.mesh.nodes, wl.mesh.conn[:m],
                       wl.mesh.boundary)
    sub = inputs.Workload(wl.name, wl.elem, wl.kind, wl.n_q, wl.coef_mode, wl.mask, wl.uniform,
                          wl.k_format, mesh, wl.coeffs)
    v1, b1, v2, b2, _ = _both(sub, "fp64")
    assert torch.equal(v1, v2) and torch.equal(b1, b2)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_blocks_hub_rows(precision):
    # rows of 44 to 168 entries: past the 32 held in registers
    wl = _with_hubs(P.small("tet_cdr"), 5)
    v1, b1, v2, b2, (rp, _) = _both(wl, precision)
    assert np.diff(rp).max() > 32
    assert torch.equal(v1, v2) and torch.equal(b1, b2)


def test_blocks_match_oracle():
    wl = P.small("tet_cdr")
    v1, b1, v2, b2, (rp, ci) = _both(wl, "fp64")
    Ar, br, Aabs, babs = P.assembly_reference(wl, "fp64")
    n = len(rp) - 1
    A = np.zeros((n, n))
    A[np.repeat(np.arange(n), np.diff(rp)), ci] = v2.cpu().numpy()
    scale = np.maximum(Aabs, Aabs.max(axis=1, keepdims=True))
    inside = np.zeros(A.shape, dtype=bool)
    inside[np.repeat(np.arange(n), np.diff(rp)), ci] = True
    assert (np.abs(A - Ar)[inside] / scale[inside]).max() <= 1e-12
    assert (np.abs(b2.cpu().numpy() - br) / np.maximum(babs, 1e-300)).max() <= 1e-12


def test_blocks_unsupported_problem():
    # blocks of a tetrahedral mesh handed to an elasticity problem
    wl = P.small("tet_elasticity")
    nn = wl.mesh.nodes.shape[0]
    dw = fe.to_device(wl, "fp64")
    nodes = torch.from_numpy(wl.mesh.nodes).cuda().contiguous()
    rp, ci = fe.csr_pattern(wl.elem, wl.mesh.conn, nn, 1)
    ip, inc = fe.node_incidence(wl.elem, wl.mesh.conn, nn)
    bl = fe.csr_blocks(wl.elem, wl.mesh.conn, nn, ip, inc, rp, ci)
    with pytest.raises(fe.FeError) as ex:
        fe.assemble_csr_blocks(dw.problem, wl.elem, nodes, dw.coeffs, dw.rule,
                               torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(),
                               torch.from_numpy(ip).cuda(), bl.to("cuda"))
    assert ex.value.status == 2  # FE_ERR_UNSUPPORTED
