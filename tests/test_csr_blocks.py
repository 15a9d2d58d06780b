"""Host logic of the node blocks (fe_csr_blocks) for the LDS-staged
row-ownership assembly: every block's nodes, elements and vertices within
the limits, its element slots exactly the elements at its nodes (in order of
first appearance along their incidence lists), its vertex slots exactly
those elements' vertices (ascending), the block-local connectivity and the
recoded incidence lists decoding to the global ones, and the capacity and
argument errors. No GPU."""
import numpy as np
import pytest

from paper_1504_01023_amd import fe, inputs
from tests import _parity as P

LIMITS = {"nodes": 256, "elems": 3072, "verts": 1024}


def _decode_and_check(elem, conn, n_nodes, bl, ip, inc):
    nv = conn.shape[1]
    blk = bl.blk.reshape(-1, 3)
    assert blk.shape[0] == bl.n_blocks + 1
    assert blk[0].tolist() == [0, 0, 0]
    assert blk[-1].tolist() == [n_nodes, len(bl.elems), len(bl.verts)]
    assert np.all(np.diff(blk, axis=0) >= 0) and np.all(np.diff(blk[:, 0]) > 0)
    for b in range(bl.n_blocks):
        n0, es, vs = blk[b]
        n1, ee, ve = blk[b + 1]
        assert n1 - n0 <= LIMITS["nodes"]
        assert ee - es <= LIMITS["elems"] and ve - vs <= LIMITS["verts"]
        # elements: those at the block's nodes, in order of first appearance
        want = []
        seen = set()
        for k in range(ip[n0], ip[n1]):
            e = inc[k] // nv
            if e not in seen:
                seen.add(e)
                want.append(e)
        assert bl.elems[es:ee].tolist() == want
        # vertices: those of the block's elements, ascending
        vset = np.unique(conn[want].ravel())
        assert bl.verts[vs:ve].tolist() == vset.tolist()
        # block-local connectivity decodes to the global one
        lc = bl.lconn[es * nv: ee * nv].reshape(-1, nv).astype(np.int64)
        assert np.all(lc < ve - vs)
        assert np.array_equal(bl.verts[vs + lc], conn[want])
        # recoded incidence: same element, same local vertex, same order
        li = bl.linc[ip[n0]: ip[n1]].astype(np.int64)
        assert np.array_equal(bl.elems[es + li // nv], inc[ip[n0]: ip[n1]] // nv)
        assert np.array_equal(li % nv, inc[ip[n0]: ip[n1]] % nv)
    # the blocks together are a greedy partition: a block stops only where
    # the next node would break a limit
    return blk


@pytest.mark.parametrize("name", ["tet_poisson", "tet_cdr", "prism_cdr"])
def test_blocks_decode(name):
    wl = P.small(name)
    conn = wl.mesh.conn.astype(np.int64)
    nn = wl.mesh.nodes.shape[0]
    ip, inc = fe.node_incidence(wl.elem, wl.mesh.conn, nn)
    bl = fe.csr_blocks(wl.elem, wl.mesh.conn, nn, ip, inc)
    assert bl.n_blocks >= 2
    _decode_and_check(wl.elem, conn, nn, bl, ip, inc)


def test_blocks_morton_order_and_greedy():
    wl = inputs.reordered(inputs.tet_poisson(14, 1), "morton")
    conn = wl.mesh.conn.astype(np.int64)
    nn = wl.mesh.nodes.shape[0]
    ip, inc = fe.node_incidence(wl.elem, wl.mesh.conn, nn)
    bl = fe.csr_blocks(wl.elem, wl.mesh.conn, nn, ip, inc)
    blk = _decode_and_check(wl.elem, conn, nn, bl, ip, inc)
    # greedy: adding the next block's first node to a block breaks a limit
    for b in range(bl.n_blocks - 1):
        n0, n1 = blk[b, 0], blk[b + 1, 0]
        els = np.unique(inc[ip[n0]: ip[n1 + 1]] // 4)
        vs = np.unique(conn[els].ravel())
        assert (n1 + 1 - n0 > LIMITS["nodes"] or len(els) > LIMITS["elems"]
                or len(vs) > LIMITS["verts"])
    # a Z-ordered mesh keeps the blocks full
    assert np.mean(np.diff(blk[:-1, 0])) > 128


def test_blocks_hub_node_too_large():
    # one node shared by more elements than a block holds
    rng = np.random.default_rng(3)
    n_other = 5000
    n_el = 3200
    conn = np.zeros((n_el, 4), dtype=np.int32)
    conn[:, 1:] = rng.integers(1, n_other, size=(n_el, 3))
    nn = n_other
    ip, inc = fe.node_incidence("tet4", conn, nn)
    with pytest.raises(fe.FeError) as ex:
        fe.csr_blocks("tet4", conn, nn, ip, inc)
    assert ex.value.status == 5  # FE_ERR_CAPACITY


def test_blocks_bad_arguments():
    wl = P.small("tet_poisson")
    nn = wl.mesh.nodes.shape[0]
    ip, inc = fe.node_incidence(wl.elem, wl.mesh.conn, nn)
    bad = inc.copy()
    bad[5] = wl.n_elem * 4 + 7  # codes no element
    with pytest.raises(fe.FeError) as ex:
        fe.csr_blocks(wl.elem, wl.mesh.conn, nn, ip, bad)
    assert ex.value.status == 1  # FE_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        fe.csr_blocks(wl.elem, wl.mesh.conn, nn + 1, ip, inc)
