"""GPU parity of the general 3-component problem beyond the small workloads:
per-point coefficients, block masks, and both precisions, against the FP64
oracle element by element."""
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


def _per_point(wl, seed):
    """The same mesh with independent 156-slot values at every point (rows
    slot * n_q + q)."""
    n, nq = wl.n_elem, wl.n_q
    vals = inputs.vector_per_element(n * nq, np.random.default_rng(seed))
    qp = np.ascontiguousarray(vals.reshape(inputs.N_VECTOR_SLOTS, n, nq).transpose(0, 2, 1)
                              .reshape(inputs.N_VECTOR_SLOTS * nq, n))
    return inputs.Workload(wl.name + "_qp", wl.elem, "vector", nq, "qp", wl.mask, wl.uniform,
                           "full", wl.mesh, qp)


@pytest.mark.parametrize("name", ["tet_vector", "prism_vector"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_per_point_coefficients(name, precision):
    wl = _per_point(P.small(name), 61)
    print(f"[vector] {wl.name} {precision} n={wl.n_elem}", flush=True)
    K, F = P.gpu_raw(wl, precision)
    P.assert_parity(wl, precision, K, F)


@pytest.mark.parametrize("name", ["tet_vector", "prism_vector"])
@pytest.mark.parametrize("mode", ["element", "qp"])
def test_block_masks(name, mode):
    base = P.small(name)
    if mode == "qp":
        base = _per_point(base, 62)
    nq = base.n_q if mode == "qp" else 1
    for mask in (1 << 16, (1 << 5) | (1 << 10) | (1 << 15), 0b1111 << 16 | 0b1011_0110_0101_0011):
        wl = inputs.Workload(base.name, base.elem, "vector", base.n_q, mode, mask, base.uniform,
                             "full", base.mesh, inputs.vector_compact(base.coeffs, mask, nq))
        print(f"[vector] {wl.name} {mode} mask={mask:#x}", flush=True)
        K, F = P.gpu_raw(wl, "fp64")
        P.assert_parity(wl, "fp64", K, F)


