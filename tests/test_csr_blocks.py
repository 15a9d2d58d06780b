"""Host logic of the node blocks (fe_csr_blocks) for the LDS-staged
row-ownership assembly: every block's nodes, elements and vertices within
the limits, its element slots exactly the elements at its nodes (in order of
first appearance along their incidence lists), its vertex slots exactly
those elements' vertices (ascending), the block-local connectivity and the
recoded incidence lists decoding to the global ones with the row positions
of the element's vertices, and the capacity and argument errors. No GPU."""
import numpy as np
import pytest

from paper_1504_01023_amd import fe, inputs
from tests import _parity as P

LIMITS = {"nodes": 256, "elems": 2432, "verts": 768}


def _build(wl_conn, nn, elem="tet4"):
    ip, inc = fe.node_incidence(elem, wl_conn, nn)
    rp, ci = fe.csr_pattern(elem, wl_conn, nn, 1)
    return ip, inc, rp, ci, fe.csr_blocks(elem, wl_conn, nn, ip, inc, rp, ci)


def _decode_and_check(elem, conn, n_nodes, bl, ip, inc, rp, ci):
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
        # recoded incidence: same element, same local vertex, same order,
        # and the row positions of the element's other vertices
        code = bl.linc[ip[n0]: ip[n1]].astype(np.int64)
        li = code & 0x3FFF
        assert np.array_equal(bl.elems[es + li // nv], inc[ip[n0]: ip[n1]] // nv)
        assert np.array_equal(li % nv, inc[ip[n0]: ip[n1]] % nv)
        for i in range(n0, n1):
            cols = ci[rp[i]: rp[i + 1]].tolist()
            for k in range(ip[i], ip[i + 1]):
                c = int(bl.linc[k])
                e, lv = inc[k] // nv, inc[k] % nv
                others = [u for u in range(nv) if u != lv]
                for f, u in enumerate(others):
                    field = (c >> (14 + 6 * f)) & 63
                    g = int(conn[e, u])
                    if g in cols and cols.index(g) < 62:
                        assert field == cols.index(g)
                    elif g in cols:
                        assert field == 63
                    else:
                        assert field == 62
    # the blocks together are a greedy partition: a block stops only where
    # the next node would break a limit
    return blk


@pytest.mark.parametrize("name", ["tet_poisson", "tet_cdr"])
def test_blocks_decode(name):
    wl = P.small(name)
    conn = wl.mesh.conn.astype(np.int64)
    nn = wl.mesh.nodes.shape[0]
    ip, inc, rp, ci, bl = _build(wl.mesh.conn, nn)
    assert bl.n_blocks >= 2
    _decode_and_check(wl.elem, conn, nn, bl, ip, inc, rp, ci)


def test_blocks_positions_absent_and_far():
    # a pattern without some couplings (62) and a hub row longer than 62
    # entries (63 past offset 61)
    from tests.test_gpu_csr_long_rows import _with_hubs
    wl = _with_hubs(P.small("tet_cdr"), 5)
    conn = wl.mesh.conn.astype(np.int64)
    nn = wl.mesh.nodes.shape[0]
    ip, inc = fe.node_incidence(wl.elem, wl.mesh.conn, nn)
    rp, ci = fe.csr_pattern(wl.elem, wl.mesh.conn, nn, 1)
    assert np.diff(rp).max() > 62
    # drop the couplings of the first element's vertices 1 and 2
    e0 = wl.mesh.conn[0]
    keep = np.ones(len(ci), dtype=bool)
    for r, c in ((e0[1], e0[2]), (e0[2], e0[1])):
        j = rp[r] + np.searchsorted(ci[rp[r]: rp[r + 1]], c)
        keep[j] = False
    rows = np.repeat(np.arange(nn), np.diff(rp))[keep]
    ci2 = ci[keep]
    rp2 = np.zeros(nn + 1, dtype=np.int64)
    np.add.at(rp2, rows + 1, 1)
    rp2 = np.cumsum(rp2)
    bl = fe.csr_blocks(wl.elem, wl.mesh.conn, nn, ip, inc, rp2, ci2)
    _decode_and_check(wl.elem, conn, nn, bl, ip, inc, rp2, ci2)
    fields = np.stack([(bl.linc.astype(np.int64) >> (14 + 6 * f)) & 63 for f in range(3)])
    assert (fields == 62).any() and (fields == 63).any()


def test_blocks_morton_order_and_greedy():
    wl = inputs.reordered(inputs.tet_poisson(14, 1), "morton")
    conn = wl.mesh.conn.astype(np.int64)
    nn = wl.mesh.nodes.shape[0]
    ip, inc, rp, ci, bl = _build(wl.mesh.conn, nn)
    blk = _decode_and_check(wl.elem, conn, nn, bl, ip, inc, rp, ci)
    # greedy: adding the next block's first node to a block breaks a limit
    for b in range(bl.n_blocks - 1):
        n0, n1 = blk[b, 0], blk[b + 1, 0]
        els = np.unique(inc[ip[n0]: ip[n1 + 1]] // 4)
        vs = np.unique(conn[els].ravel())
        assert (n1 + 1 - n0 > LIMITS["nodes"] or len(els) > LIMITS["elems"]
                or len(vs) > LIMITS["verts"])
    # a Z-ordered mesh keeps the blocks full
    assert np.mean(np.diff(blk[:-1, 0])) >= 0.9 * LIMITS["nodes"]


def test_blocks_hub_node_too_large():
    # one node shared by more elements than a block holds
    rng = np.random.default_rng(3)
    n_other = 5000
    n_el = 3200
    conn = np.zeros((n_el, 4), dtype=np.int32)
    conn[:, 1:] = rng.integers(1, n_other, size=(n_el, 3))
    nn = n_other
    with pytest.raises(fe.FeError) as ex:
        _build(conn, nn)
    assert ex.value.status == 5  # FE_ERR_CAPACITY


def test_blocks_bad_arguments():
    wl = P.small("tet_poisson")
    nn = wl.mesh.nodes.shape[0]
    ip, inc, rp, ci, _ = _build(wl.mesh.conn, nn)
    bad = inc.copy()
    bad[5] = wl.n_elem * 4 + 7  # codes no element
    with pytest.raises(fe.FeError) as ex:
        fe.csr_blocks(wl.elem, wl.mesh.conn, nn, ip, bad, rp, ci)
    assert ex.value.status == 1  # FE_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        fe.csr_blocks(wl.elem, wl.mesh.conn, nn + 1, ip, inc, rp, ci)
    # prisms: not built
    wp = P.small("prism_cdr")
    npn = wp.mesh.nodes.shape[0]
    ipp, incp = fe.node_incidence(wp.elem, wp.mesh.conn, npn)
    rpp, cip = fe.csr_pattern(wp.elem, wp.mesh.conn, npn, 1)
    with pytest.raises(fe.FeError) as ex:
        fe.csr_blocks(wp.elem, wp.mesh.conn, npn, ipp, incp, rpp, cip)
    assert ex.value.status == 2  # FE_ERR_UNSUPPORTED
