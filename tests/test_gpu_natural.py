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
    # tiles of more than 64 KiB of LDS (gfx950 allows 160 KiB per workgroup)
    "prism_cdr_qp": lambda: P.small("prism_cdr_qp"),
    "prism_elasticity": lambda: P.small("prism_elasticity"),
}
# 3-component problems: outputs in LDS bytes of their own; FP32 tiles fit
VECTOR_CASES = {
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


@pytest.mark.parametrize("name,precision",
                         [(n, p) for n in sorted(CASES) for p in ("fp64", "fp32")]
                         + [(n, "fp32") for n in sorted(VECTOR_CASES)])
def test_natural_order_matches_soa_and_oracle(name, precision):
    wl = {**CASES, **VECTOR_CASES}[name]()
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


def test_natural_order_limits():
    # FP64 3-component tiles need more than 160 KiB of LDS: refused
    for wl in (P.small("tet_vector"), P.small("prism_vector")):
        dw = fe.to_device(wl, "fp64")
        coeffs = dw.coeffs.t().contiguous() if dw.coeffs is not None else None
        with pytest.raises(fe.FeError) as e:
            fe.integrate_natural(dw.problem, wl.elem, dw.coords.t().contiguous(), coeffs, dw.rule)
        assert e.value.status == 2
