"""GPU parity on degenerate elements: mirrored (det J < 0) and partly
inverted prisms are integrated as written with the signed determinant, as
the oracle does, to the usual tolerance; flat elements (det J = 0) give
non-finite results on exactly the elements where the oracle's are, and
leave their neighbours untouched."""
import dataclasses

import numpy as np
import pytest

from paper_1504_01023_amd import fe
from tests import _parity as P
from tests.test_gpu_orient import plant

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NAMES = ["tet_cdr", "tet_elasticity", "prism_cdr_qp", "prism_cdr", "prism_elasticity", "tet_vector",
         "prism_vector"]


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fe.lib()
    yield


def _with_coords(wl, coords):
    return dataclasses.replace(wl, mesh=dataclasses.replace(wl.mesh, coords=coords))


def _split(wl, rng):
    """Planted coordinates, and the elements that were flattened."""
    before = wl.mesh.coords
    c = plant(wl.mesh, rng, frac=0.08)
    nv = c.shape[0] // 3
    flat = np.nonzero(np.all(c.reshape(nv, 3, -1)[:, 2] == 0.5, axis=0) &
                      ~np.all(before.reshape(nv, 3, -1)[:, 2] == 0.5, axis=0))[0]
    return c, flat


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_inverted_elements_match_oracle(name, precision):
    wl = P.small(name)
    c, flat = _split(wl, np.random.default_rng(77))
    # undo the flattening: this test keeps only mirrored and partly inverted elements
    c[:, flat] = wl.mesh.coords[:, flat]
    w2 = _with_coords(wl, c)
    print(f"[degenerate] {name} {precision} n={wl.n_elem}", flush=True)
    K, F = P.gpu_raw(w2, precision)
    assert np.all(np.isfinite(K)) and np.all(np.isfinite(F))
    P.assert_parity(w2, precision, K, F)


@pytest.mark.parametrize("name", ["tet_cdr", "prism_cdr_qp", "tet_elasticity", "prism_elasticity"])
def test_flat_elements_nonfinite_where_the_oracle_is(name):
    wl = P.small(name)
    c, flat = _split(wl, np.random.default_rng(78))
    assert flat.size > 0
    w2 = _with_coords(wl, c)
    K, F = P.gpu_raw(w2, "fp64")
    Kg, Fg = P.to_full(K, F, w2)
    Ko, Fo = P.oracle_run(w2, "fp64")
    bad_g = ~(np.isfinite(Kg).all(axis=(1, 2)) & np.isfinite(Fg).all(axis=1))
    bad_o = ~(np.isfinite(Ko).all(axis=(1, 2)) & np.isfinite(Fo).all(axis=1))
    assert np.array_equal(np.nonzero(bad_o)[0], flat)
    assert np.array_equal(bad_g, bad_o)
    good = ~bad_o
    ek, ef = P.rel_errors(Kg[good], Fg[good], Ko[good], Fo[good])
    assert ek.max() <= P.TOL["fp64"] and ef.max() <= P.TOL["fp64"]
