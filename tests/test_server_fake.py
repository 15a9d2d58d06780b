"""The serving scheduler on the CPU, with the FAKE backend (a timing model
instead of the device): admission by HBM budget and slots, arrival order,
failure isolation, output residency until release, latency bookkeeping."""
import time

import numpy as np
import pytest

from paper_1504_01023_amd import fe, serve

# Host "inputs": the fake backend never reads them, any address will do.
DUMMY = np.zeros(16)
PTR = DUMMY.ctypes.data


def kinds():
    cdr = fe.problem("scalar", "fp64", "element", (1 << 20) - 1, None, "full")
    el = fe.problem("elasticity", "fp32", "element", 31, None, "packed")
    return [(cdr, "tet4", fe.builtin_rule("tet4", 4)), (el, "prism6", fe.builtin_rule("prism6", 6))]


def bytes_of(kind, n):
    ld = (n + 63) // 64 * 64
    r = lambda b: (b + 255) // 256 * 256
    if kind == 0:  # tet CDR fp64: coords 12, coeffs 20, K 16, F 4
        return r(8 * 12 * ld) + r(8 * 20 * ld) + r(8 * 16 * ld) + r(8 * 4 * ld)
    return r(8 * 18 * ld) + r(4 * 5 * ld) + r(4 * 171 * ld) + r(4 * 18 * ld)


def drain(s, n, timeout=20.0):
    out = []
    t0 = time.time()
    while len(out) < n and time.time() - t0 < timeout:
        out += s.poll(64, 0.05)
    return out


def test_all_complete_in_order_with_latency_breakdown():
    with serve.Server(kinds(), max_slots=4, hbm_budget_bytes=1 << 30, chunk_elems=1024,
                      max_chunks=16, backend=serve.FAKE, fake_ns_per_elem=5.0,
                      fake_h2d_bytes_per_s=20e9) as s:
        ids = [s.submit(i % 2, 1000 + 500 * i, PTR, PTR, tag=100 + i) for i in range(12)]
        done = drain(s, 12)
        assert len(done) == 12
        assert all(c.status == 0 for c in done)
        assert sorted(c.tag for c in done) == list(range(100, 112))
        by_id = {c.id: c for c in done}
        for i, rid in enumerate(ids):
            c = by_id[rid]
            assert c.t_submit <= c.t_admit <= c.t_ready <= c.t_done
            assert c.n_elem == 1000 + 500 * i
            assert c.ld_out % 64 == 0 and c.ld_out >= c.n_elem
        # admission follows arrival order
        adm = [by_id[r].t_admit for r in ids]
        assert adm == sorted(adm)
        st = s.stats()
        lat = np.array([c.t_done - c.t_submit for c in done])
        assert st["completed"] == 12 and st["failed"] == 0
        assert st["p50_s"] == pytest.approx(np.percentile(lat, 50), rel=1e-9, abs=1e-12)
        assert st["p99_s"] == pytest.approx(np.percentile(lat, 99), rel=1e-9, abs=1e-12)
        assert st["elements_done"] == sum(1000 + 500 * i for i in range(12))
        # outputs stay resident until released
        assert st["bytes_in_use"] == sum(bytes_of(i % 2, 1000 + 500 * i) for i in range(12))
        for c in done:
            s.release(c.id)
        assert s.stats()["bytes_in_use"] == 0


def test_budget_and_slots_bound_admission():
    n = 20000
    per = bytes_of(0, n)
    budget = 3 * per + 1000          # room for three requests at a time
    with serve.Server(kinds(), max_slots=8, hbm_budget_bytes=budget, chunk_elems=4096,
                      max_chunks=64, backend=serve.FAKE, fake_ns_per_elem=50.0,
                      fake_h2d_bytes_per_s=50e9) as s:
        for i in range(9):
            s.submit(0, n, PTR, PTR, tag=i)
        got, peak_inflight = [], 0
        t0 = time.time()
        while len(got) < 9 and time.time() - t0 < 30:
            st = s.stats()
            assert st["bytes_in_use"] <= budget
            peak_inflight = max(peak_inflight, st["in_flight"])
            for c in s.poll(16, 0.01):
                got.append(c)
                s.release(c.id)    # the consumer frees memory as it goes
        assert len(got) == 9 and all(c.status == 0 for c in got)
        assert peak_inflight <= 3
        assert s.stats()["bytes_peak"] <= budget


def test_slot_limit():
    with serve.Server(kinds(), max_slots=2, hbm_budget_bytes=1 << 32, chunk_elems=1024,
                      max_chunks=64, backend=serve.FAKE, fake_ns_per_elem=200.0) as s:
        for i in range(6):
            s.submit(1, 3000, PTR, PTR)
        seen = 0
        t0 = time.time()
        while seen < 6 and time.time() - t0 < 30:
            assert s.stats()["in_flight"] <= 2
            seen += len(s.poll(8, 0.005))
        assert seen == 6


def test_oversized_request_fails_alone():
    budget = bytes_of(0, 50000)
    with serve.Server(kinds(), max_slots=4, hbm_budget_bytes=budget, chunk_elems=1024,
                      max_chunks=64, backend=serve.FAKE, fake_ns_per_elem=1.0) as s:
        a = s.submit(0, 1000, PTR, PTR)
        big = s.submit(0, 10_000_000, PTR, PTR)
        b = s.submit(0, 2000, PTR, PTR)
        done = {c.id: c for c in drain(s, 3)}
        assert done[big].status == 5 and not done[big].out_K
        assert done[a].status == 0 and done[b].status == 0
        st = s.stats()
        assert st["failed"] == 1 and st["completed"] == 2


def test_continuous_batching_joins_running_work():
    # a long request is running when short ones arrive; they are admitted
    # and finish before it (their chunks join the next ticks)
    with serve.Server(kinds(), max_slots=8, hbm_budget_bytes=1 << 32, chunk_elems=4096,
                      max_chunks=8, backend=serve.FAKE, fake_ns_per_elem=20.0,
                      fake_tick_overhead_s=1e-5) as s:
        long_id = s.submit(0, 2_000_000, PTR, PTR)
        time.sleep(0.005)
        short = [s.submit(0, 4096, PTR, PTR) for _ in range(3)]
        done = {c.id: c for c in drain(s, 4, timeout=60)}
        assert all(done[i].t_done < done[long_id].t_done for i in short)
        assert s.stats()["ticks"] > 8


def test_submit_validation():
    with serve.Server(kinds(), backend=serve.FAKE) as s:
        with pytest.raises(fe.FeError):
            s.submit(5, 10, PTR, PTR)
        with pytest.raises(fe.FeError):
            s.submit(0, 0, PTR, PTR)
        with pytest.raises(fe.FeError):
            s.submit(0, 10, PTR, None)
        with pytest.raises(fe.FeError):
            s.submit(0, 10, PTR, PTR, on_device=True, ld_in=5)
        with pytest.raises(fe.FeError):
            s.submit(0, 10, PTR, PTR, ld_in=5)
        with pytest.raises(fe.FeError):
            s.release(12345)
