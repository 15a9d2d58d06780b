"""GPU parity of natural-order (element-contiguous) inputs and outputs
(fe_integrate_natural): bit for bit the structure-of-arrays results of the
same per-element code, and the oracle within tolerance; ragged tiles."""
import numpy as np
import pytest

from paper_1504_01023_amd import fe, inputs
from tests import _parity as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = {
    "tet_poisson": lambda: P.small("tet_poisson"),
    "tet_poisson_qp": lambda: P.small("tet_poisson_qp"),
    "tet_cdr": lambda: P.small("tet_cdr"),
    "tet_cdr_fn": lambda: P.small("tet_cdr_fn"),
    "tet_elasticity": lambda: P.small("tet_elasticity"),
    "prism_cdr": lambda: P.small("prism_cdr"),
    "prism_cdr_fn": lambda: P.small("prism_cdr_fn"),
    "prism_poisson_qp": lambda: inputs.prism_poisson_qp_rhs(8, 5, seed=19),
    # records of more than 1 KiB per element: read and written in place
    # (no LDS tile) in FP64, tiles in FP32 for prism CDR and elasticity
    "prism_cdr_qp": lambda: P.small("prism_cdr_qp"),
    "prism_elasticity": lambda: P.small("prism_elasticity"),
    "tet_vector": lambda: P.small("tet_vector"),
    "prism_vector": lambda: P.small("prism_vector"),
}


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fe.lib()
    yield


def _natural(dw, wl, n):
    coords = dw.coords[:, :n].t().contiguous()
    coeffs = dw.coeffs
    if coeffs is not None and wl.coef_mode != "function":
        coeffs = coeffs[:, :n].t().contiguous()
    K, F = fe.integrate_natural(dw.problem, wl.elem, coords, coeffs, dw.rule)
    torch.cuda.synchronize()
    return K.t().contiguous(), F.t().contiguous()


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_natural_order_matches_soa_and_oracle(name, precision):
    wl = CASES[name]()
    print(f"[natural] {name} {precision} n={wl.n_elem}", flush=True)
    dw = fe.to_device(wl, precision)
    for n in (1, 63, 64, 65, 130, wl.n_elem):
        n = min(n, wl.n_elem)
        Kn, Fn = _natural(dw, wl, n)
        coeffs = dw.coeffs if (dw.coeffs is None or wl.coef_mode == "function") \
            else dw.coeffs[:, :n].contiguous()
        Ks, Fs = fe.integrate(dw.problem, wl.elem, dw.coords[:, :n].contiguous(), coeffs, dw.rule,
                              variant=fe.variant(elems_per_thread=1))
        torch.cuda.synchronize()
        assert torch.equal(Kn, Ks) and torch.equal(Fn, Fs), n
    P.assert_parity(wl, precision, Kn.cpu().numpy(), Fn.cpu().numpy())
