"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (rows padded to a leading dimension that is a multiple of
256 elements, the committed MI355X tuning table): every output finite, and a
sample of elements (the first, the last, random ones and, for prisms, part of
the sliver layer) against the oracle element by element."""
import functools
import os

import numpy as np
import pytest

import bench
from paper_1504_01023_amd import fe
from tests import _parity as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TUNING = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "paper_1504_01023_amd", "tuning_mi355x.txt")
CASES = [("tet_poisson", "fp64"), ("tet_poisson", "fp32"), ("tet_poisson_qp", "fp64"),
         ("tet_cdr", "fp64"), ("tet_cdr", "fp32"), ("prism_cdr_qp", "fp64"),
         ("prism_cdr_qp", "fp32"), ("prism_cdr", "fp64"), ("prism_poisson_qp", "fp64"),
         ("tet_elasticity", "fp64"), ("tet_elasticity", "fp32"), ("prism_elasticity", "fp64"),
         ("prism_elasticity", "fp32"), ("tet_vector", "fp64"), ("prism_vector", "fp64"),
         ("prism_vector", "fp32")]
ALIGN = 256


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fe.lib()
    fe.tuning_load(TUNING)
    yield
    _workload.cache_clear()
    torch.cuda.empty_cache()


@functools.lru_cache(maxsize=1)
def _workload(name):
    return bench.WORKLOADS[name][0]()


def _sample(wl, rng):
    n = wl.n_elem
    idx = [np.array([0, n - 1]), rng.choice(n, 3000, replace=False)]
    if wl.elem == "prism6":
        # the sliver layer (thickness 1e-3 of the cell size) sits at layer L // 2
        m = wl.mesh
        dz = m.coords[[11, 14, 17]].mean(axis=0) - m.coords[[2, 5, 8]].mean(axis=0)
        thin = np.nonzero(dz < 1e-4)[0]
        assert thin.size > 0
        idx.append(rng.choice(thin, min(300, thin.size), replace=False))
    return np.unique(np.concatenate(idx))


@pytest.mark.parametrize("name,precision", CASES)
def test_full_size_sampled_parity(name, precision):
    wl = _workload(name)
    n = wl.n_elem
    print(f"[full] {name} {precision} n={n}", flush=True)
    dw = fe.to_device(wl, precision)
    ld = (n + ALIGN - 1) // ALIGN * ALIGN

    def padded(t):
        out = torch.zeros((t.shape[0], ld), dtype=t.dtype, device="cuda")
        out[:, :n] = t
        return out

    coords = padded(dw.coords)
    coeffs = dw.coeffs
    if coeffs is not None and wl.coef_mode != "function":
        coeffs = padded(coeffs)
    del dw.coords
    dt = torch.float64 if precision == "fp64" else torch.float32
    K = torch.empty((fe.k_entries(dw.problem, wl.elem), ld), dtype=dt, device="cuda")
    F = torch.empty((fe.f_entries(dw.problem, wl.elem), ld), dtype=dt, device="cuda")
    fe.integrate(dw.problem, wl.elem, coords, coeffs, dw.rule, K, F, n_elem=n)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(K[:, :n]).all()) and bool(torch.isfinite(F[:, :n]).all())
    s = _sample(wl, np.random.default_rng(2024))
    sd = torch.from_numpy(s).cuda()
    Kh = K[:, sd].cpu().numpy()
    Fh = F[:, sd].cpu().numpy()
    del coords, coeffs, K, F
    torch.cuda.empty_cache()
    Kg, Fg = P.to_full(Kh, Fh, wl)
    Ko, Fo = P.oracle_run(wl, precision, elements=s)
    ek, ef = P.rel_errors(Kg, Fg, Ko, Fo)
    tol = P.TOL[precision]
    print(f"[full] {name} {precision}: {len(s)} sampled, max rel err K {ek.max():.2e} F {ef.max():.2e}",
          flush=True)
    assert ek.max() <= tol, f"K rel err {ek.max():.3e} at element {int(s[ek.argmax()])}"
    assert ef.max() <= tol, f"F rel err {ef.max():.3e} at element {int(s[ef.argmax()])}"
