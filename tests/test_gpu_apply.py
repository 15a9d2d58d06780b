"""GPU parity of the matrix-free operator application (fe_apply_indexed)
against the oracle's assembled y = sum_e P_e^T K^e P_e x and load vector,
coloured (deterministic) and atomic."""
import numpy as np
import pytest

from paper_1504_01023_amd import fe, inputs
from tests import _parity as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# rounding of the assembled sums, relative to |A| |x| row by row
TOL = {"fp64": 1e-12, "fp32": 2e-5}
CASES = ["tet_poisson", "tet_poisson_qp", "tet_cdr", "tet_cdr_fn", "tet_elasticity", "prism_cdr_qp",
         "prism_cdr", "prism_cdr_fn", "prism_elasticity", "prism_elasticity_qp", "tet_vector", "prism_vector",
         "tet_cdr_morton",
         "prism_cdr_qp_morton"]


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fe.lib()
    yield


def _setup(name, precision):
    if name.endswith("_morton"):
        wl = inputs.reordered(P.small(name[: -len("_morton")]))
    else:
        wl = P.small(name)
    perm, ptr = fe.color_elements(wl.elem, wl.mesh.conn, wl.mesh.nodes.shape[0])
    dw = fe.to_device(wl, precision)
    conn = torch.from_numpy(np.ascontiguousarray(wl.mesh.conn[perm].T.astype(np.int32))).cuda()
    coeffs = dw.coeffs
    if coeffs is not None and wl.coef_mode not in ("uniform", "function"):
        coeffs = coeffs[:, torch.from_numpy(perm.astype(np.int64)).cuda()].contiguous()
    nodes = torch.from_numpy(wl.mesh.nodes).cuda().contiguous()
    nc = 1 if wl.kind == "scalar" else 3
    x64 = np.random.default_rng(71).standard_normal(wl.mesh.nodes.shape[0] * nc)
    dt = torch.float64 if precision == "fp64" else torch.float32
    x = torch.from_numpy(x64).to(device="cuda", dtype=dt)
    xo = x.double().cpu().numpy()  # the values the GPU sees
    return wl, dw, conn, coeffs, nodes, x, xo, ptr


def _check(y, b, ref, precision):
    yr, br, yabs, babs = ref
    tol = TOL[precision]
    y = y.double().cpu().numpy()
    b = b.double().cpu().numpy()
    scale_y = np.maximum(yabs, 1e-300)
    ey = np.abs(y - yr) / scale_y
    assert ey.max() <= tol, f"y rel err {ey.max():.3e} at dof {int(ey.argmax())}"
    eb = np.abs(b - br) / np.maximum(babs, 1e-300)
    assert eb.max() <= tol, f"b rel err {eb.max():.3e} at dof {int(eb.argmax())}"


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_coloured_and_atomic_match_oracle(name, precision):
    wl, dw, conn, coeffs, nodes, x, xo, ptr = _setup(name, precision)
    print(f"[apply] {name} {precision} n={wl.n_elem} colours={len(ptr) - 1}", flush=True)
    ref = P.apply_reference(wl, precision, xo)
    zeros = lambda: torch.zeros_like(x)
    y1, b1 = fe.apply_indexed(dw.problem, wl.elem, nodes, conn, coeffs, dw.rule, x, zeros(),
                              zeros(), color_ptr=ptr)
    y2, b2 = fe.apply_indexed(dw.problem, wl.elem, nodes, conn, coeffs, dw.rule, x, zeros(),
                              zeros(), color_ptr=ptr)
    y3, b3 = fe.apply_indexed(dw.problem, wl.elem, nodes, conn, coeffs, dw.rule, x, zeros(),
                              zeros())
    torch.cuda.synchronize()
    _check(y1, b1, ref, precision)
    _check(y3, b3, ref, precision)
    # colour by colour with plain updates: the same bits every run
    assert torch.equal(y1, y2) and torch.equal(b1, b2)


def test_accumulates_and_optional_load():
    wl, dw, conn, coeffs, nodes, x, xo, ptr = _setup("tet_cdr", "fp64")
    y0 = torch.full_like(x, 0.5)
    y, b = fe.apply_indexed(dw.problem, wl.elem, nodes, conn, coeffs, dw.rule, x, y0.clone(),
                            None, color_ptr=ptr)
    torch.cuda.synchronize()
    assert b is None
    yr, _, yabs, _ = P.apply_reference(wl, "fp64", xo)
    err = np.abs(y.cpu().numpy() - 0.5 - yr) / np.maximum(yabs, 1e-300)
    assert err.max() <= 1e-12


def test_empty_and_single_colour_subset():
    wl, dw, conn, coeffs, nodes, x, xo, ptr = _setup("tet_poisson", "fp64")
    y = torch.zeros_like(x)
    fe.apply_indexed(dw.problem, wl.elem, nodes, conn, coeffs, dw.rule, x, y, None,
                     color_ptr=np.array([0]), n_elem=0)
    torch.cuda.synchronize()
    assert not y.any()
    # the first colour alone equals the oracle on those elements
    c1 = int(ptr[1])
    fe.apply_indexed(dw.problem, wl.elem, nodes, conn, coeffs, dw.rule, x, y, None,
                     color_ptr=np.array([0, c1]), n_elem=c1)
    torch.cuda.synchronize()
    perm, _ = fe.color_elements(wl.elem, wl.mesh.conn, wl.mesh.nodes.shape[0])
    sub_conn = wl.mesh.conn[perm[:c1]]
    sub = inputs.Workload(wl.name, wl.elem, wl.kind, wl.n_q, wl.coef_mode, wl.mask, wl.uniform,
                          wl.k_format,
                          inputs.Mesh(wl.elem, np.ascontiguousarray(wl.mesh.coords[:, perm[:c1]]),
                                      wl.mesh.nodes, sub_conn, wl.mesh.boundary), None)
    yr, _, yabs, _ = P.apply_reference(sub, "fp64", xo)
    err = np.abs(y.cpu().numpy() - yr) / np.maximum(yabs, 1e-300)
    assert err.max() <= 1e-12
