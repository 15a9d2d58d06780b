"""The library's defaults on the GPU: with an empty caller tuning table the
built-in table measured on MI355X is in effect (fe_integrate with variant =
NULL runs the tuned variants), and the binding's default buffers have
line-aligned rows (ld_for(n)) with (rows, n) views, matching the oracle."""
import os
import re

import numpy as np
import pytest

from paper_1504_01023_amd import fe
from tests import _parity as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_1504_01023_amd", "tuning_mi355x.txt")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fe.tuning_clear()
    yield


def _committed():
    out = {}
    for line in open(TABLE):
        if not line.strip() or line.startswith("#"):
            continue
        key, var = line.split("|")
        out[tuple(int(x) for x in key.split())] = tuple(int(x) for x in var.split())
    return out


def test_builtin_table_in_effect_on_gfx950():
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    on, tab_arch, n = fe.tuning_builtin()
    assert tab_arch == "gfx950"
    if arch != "gfx950":
        pytest.skip(f"device is {arch}")
    assert on and n == len(_committed())


@pytest.mark.parametrize("name,prec,key", [
    ("tet_poisson", "fp64", (0, 0, 0, 33, 0, 1, 1)),
    ("tet_poisson", "fp32", (0, 0, 1, 33, 0, 1, 1)),
    ("tet_cdr", "fp64", (0, 0, 0, 63, 1, 0, 4)),
    ("tet_elasticity", "fp32", (0, 1, 1, 64, 1, 1, 1)),
    ("prism_cdr", "fp64", (1, 0, 0, 63, 1, 0, 6)),
    ("prism_elasticity", "fp64", (1, 1, 0, 64, 1, 1, 6)),
])
def test_untuned_call_gets_the_table_variant_and_padded_layout(name, prec, key):
    fe.tuning_clear()
    if not fe.tuning_builtin()[0]:
        pytest.skip("built-in table not in effect on this device")
    wl = P.small(name)
    dw = fe.to_device(wl, prec)
    assert fe.tuning_get(dw.problem, wl.elem, wl.n_q) == _committed()[key]
    n = wl.n_elem
    ld = fe.ld_for(n)
    assert ld % 256 == 0 and ld >= n
    assert tuple(dw.coords.shape) == (dw.coords.shape[0], n) and dw.coords.stride(0) == ld
    K, F = fe.integrate(dw.problem, wl.elem, dw.coords, dw.coeffs, dw.rule)
    torch.cuda.synchronize()
    assert K.shape[1] == n and K.stride(0) == ld and F.stride(0) == ld
    assert K.data_ptr() % 256 == 0 and F.data_ptr() % 256 == 0
    P.assert_parity(wl, prec, K.cpu().numpy(), F.cpu().numpy())
    # the same call on unpadded contiguous copies gives the same bits
    c = dw.coords.contiguous()
    k = dw.coeffs.contiguous() if dw.coeffs is not None and dw.coeffs.dim() == 2 else dw.coeffs
    K2 = torch.empty((K.shape[0], n), dtype=K.dtype, device="cuda")
    F2 = torch.empty((F.shape[0], n), dtype=F.dtype, device="cuda")
    fe.integrate(dw.problem, wl.elem, c, k, dw.rule, out_K=K2, out_F=F2)
    torch.cuda.synchronize()
    assert torch.equal(K, K2) and torch.equal(F, F2)


def test_caller_entry_overrides_builtin():
    wl = P.small("tet_poisson")
    dw = fe.to_device(wl, "fp64")
    v = fe.variant(64, 2, 1, 2, 0, 1, 1, 1)
    fe.tuning_set(dw.problem, "tet4", 1, v)
    try:
        assert fe.tuning_get(dw.problem, "tet4", 1) == v.as_tuple()
        K, F = fe.integrate(dw.problem, "tet4", dw.coords, None, dw.rule)
        torch.cuda.synchronize()
        P.assert_parity(wl, "fp64", K.cpu().numpy(), F.cpu().numpy())
    finally:
        fe.tuning_clear()
    if fe.tuning_builtin()[0]:
        assert fe.tuning_get(dw.problem, "tet4", 1) == _committed()[(0, 0, 0, 33, 0, 1, 1)]
