#!/usr/bin/env python3
"""Benchmark: element integration throughput on one MI355X.

Default workload (the headline one): scalar Poisson (c^{i;j} = identity,
d^0 = 1) on the jittered unit cube with N = 119 cells per side split into
6 Kuhn tetrahedra (10,110,954 elements, seed 1), 1-point rule, packed 4x4 K
and 4-vector F, FP64. One "step" is one fe_integrate call over the whole
mesh with inputs already resident in HBM, in the library's default layout
(rows of fe_ld_for(n) elements) and launch variant (its built-in table).

Timing: W untimed warm-up steps, then K timed steps back to back between
device synchronisations. `value` (elements/s) and `ms_per_step` come from the
host clock over that region; `roofline.achieved` divides the algorithmic
bytes by the average kernel duration from one pair of HIP events on the
launch stream around the same region; `wall_frac` is `value` x bytes over
the peak. Per-launch durations (min / median) come from a separate pass.

The default run then reports the rest of the metric in the same line:
`fp32` (the same workload in the FP32 bulk tier, its speed-up over FP64
against the byte-ratio bound, and its error against the FP64 oracle) and
`served` (the mixed request stream of one jittered mesh per request through
the continuous-batching server: saturation throughput with host and with
resident inputs, the speed-ups over one-at-a-time fe_integrate, p50/p99 at
offered load 0.7 with the queue / H2D / device split, and the alone-vs-mix
bitwise check). --headline-only skips both.

Extra workloads (--workload): tet_cdr (N=119, 4-point rule, per-element
coefficients, full K), prism_cdr_qp (141x141x100 prisms with per-point
coefficients), tet_elasticity (N=94, packed 12x12), prism_elasticity, and
more; `served` runs the full served protocol (loads 0.5, 0.7, 0.9);
--precision fp32 selects the FP32 bulk tier.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E peak, vendor figure

WORKLOADS = {
    # name: (builder, description)
    "tet_poisson": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).tet_poisson(119, 1),
                    "Poisson on jittered unit cube N=119 x 6 Kuhn tets (10,110,954), tet 1-point rule, packed K"),
    "tet_poisson_qp": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).tet_poisson_qp_rhs(119, 1),
                       "Poisson with d^0 per point of the tet 4-point rule, full K (36 words/element), N=119"),
    "tet_cdr": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).tet_cdr(119, 2),
                "convection-diffusion-reaction, 20 coefficients per element, tet 4-point rule, full K, N=119"),
    "prism_cdr_qp": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).prism_cdr_qp(141, 100, 3),
                     "prisms 141x141x100 (3,976,200, 1% slivers), 20 smooth coefficients per point, 6-point rule, full K"),
    "prism_poisson_qp": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).prism_poisson_qp_rhs(141, 100, 3),
                         "prisms 141x141x100 (3,976,200), Laplacian with d^0 per point of the 6-point rule, full K (66 words/element)"),
    "prism_cdr": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).prism_cdr_element(141, 100, 3),
                  "prisms 141x141x100 (3,976,200), 20 coefficients per element, 6-point rule, full K (80 words/element)"),
    "prism_cdr_fn": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).prism_cdr_fn(141, 100, 3),
                     "prisms 141x141x100 (3,976,200), 20 smooth coefficient fields evaluated in the kernel at the 6 points, full K"),
    "tet_cdr_fn": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).tet_cdr_fn(119, 2),
                   "tets N=119, 20 smooth coefficient fields evaluated in the kernel at the 4 points, full K"),
    "tet_elasticity": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).tet_elasticity(94, 4),
                       "isotropic elasticity on tets N=94 (4,983,504), per-element E, nu, f, 1-point rule, packed 12x12"),
    "prism_elasticity": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).prism_elasticity(100, 100, 4),
                         "isotropic elasticity on prisms 100x100x100 (2,000,000), per-element E, nu, f, 6-point rule, packed 18x18"),
    "tet_vector": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).tet_vector(94, 6),
                   "general 3-component CDR on tets N=94 (4,983,504), 156 coefficients per element, 4-point rule, full 12x12"),
    "prism_vector": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).prism_vector(100, 100, 7),
                     "general 3-component CDR on prisms 100x100x100 (2,000,000), 156 coefficients per element, 6-point rule, full 18x18"),
}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


KERNEL_UNITS = {
    ("tet_poisson", "fp64"): "fe_k_tet_scalar_f64_poisson.hip",
    ("tet_poisson", "fp32"): "fe_k_tet_scalar_f32_poisson.hip",
    ("tet_poisson_qp", "fp64"): "fe_k_tet_scalar_f64_poisson.hip",
    ("tet_poisson_qp", "fp32"): "fe_k_tet_scalar_f32_poisson.hip",
    ("tet_cdr", "fp64"): "fe_k_tet_scalar_f64_full.hip",
    ("tet_cdr", "fp32"): "fe_k_tet_scalar_f32_full.hip",
    ("prism_cdr_qp", "fp64"): "fe_k_prism_scalar_f64_full.hip",
    ("prism_cdr_qp", "fp32"): "fe_k_prism_scalar_f32_full.hip",
    ("tet_elasticity", "fp64"): "fe_k_tet_elast_f64.hip",
    ("tet_elasticity", "fp32"): "fe_k_tet_elast_f32.hip",
    ("prism_elasticity", "fp64"): "fe_k_prism_elast_f64.hip",
    ("prism_poisson_qp", "fp64"): "fe_k_prism_scalar_f64_poisson.hip",
    ("prism_poisson_qp", "fp32"): "fe_k_prism_scalar_f32_poisson.hip",
    ("prism_cdr", "fp64"): "fe_k_prism_scalar_f64_full.hip",
    ("prism_cdr", "fp32"): "fe_k_prism_scalar_f32_full.hip",
    ("prism_cdr_fn", "fp64"): "fe_k_prism_scalar_f64_full.hip",
    ("prism_cdr_fn", "fp32"): "fe_k_prism_scalar_f32_full.hip",
    ("tet_cdr_fn", "fp64"): "fe_k_tet_scalar_f64_full.hip",
    ("tet_cdr_fn", "fp32"): "fe_k_tet_scalar_f32_full.hip",
    ("prism_elasticity", "fp32"): "fe_k_prism_elast_f32.hip",
    ("tet_vector", "fp64"): "fe_k_tet_vector_f64.hip",
    ("tet_vector", "fp32"): "fe_k_tet_vector_f32.hip",
    ("prism_vector", "fp64"): "fe_k_prism_vector_f64.hip",
    ("prism_vector", "fp32"): "fe_k_prism_vector_f32.hip",
}


def source_hash(workload: str, precision: str) -> str:
    """Hash of the sources that define the measured kernel (device code,
    shared headers, the family's instantiation unit); a stored counter
    reading is only reused while this matches."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1504_01023_amd", "csrc")
    for name in ("fe_device.h", "fe_internal.h", "fe_register.h",
                 KERNEL_UNITS[(workload, precision)]):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(workload: str, precision: str, src_hash: str):
    """HBM bytes per launch measured with rocprofv3 counters for this kernel
    (profiles/<workload>_<precision>_pmc.md), if the sources still match."""
    path = os.path.join(ROOT, "profiles", f"{workload}_{precision}_pmc.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel_source_hash:\s*(\w+)", txt)
    m_val = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_val or m_hash.group(1) != src_hash:
        return None
    return float(m_val.group(1))


def host_threads() -> int:
    """Threads for host-side work: the CPUs this process may run on (its
    affinity), capped by OMP_NUM_THREADS where the machine sets one (a GPU
    share of a larger host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def cpu_description() -> dict:
    """The host CPU: lscpu's model name (else /proc/cpuinfo's), nproc (the
    affinity) and the logical CPU count of the machine."""
    import subprocess
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.strip().startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if not model:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": nproc, "cpu_count": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(wl, min_s: float = 10.0, max_s: float = 30.0):
    """The oracle as it stands, timed on the host cores on passes over the
    same workload (whole passes until about min_s seconds have elapsed)."""
    import oracle
    threads = host_threads()
    done, passes = 0, 0
    t0 = time.perf_counter()
    chunk = min(wl.n_elem, 2_000_000)
    while True:
        for e0 in range(0, wl.n_elem, chunk):
            idx = np.arange(e0, min(wl.n_elem, e0 + chunk))
            oracle.integrate_workload(wl, threads=threads, elements=idx)
            done += len(idx)
            if time.perf_counter() - t0 > max_s:
                break
        passes += 1
        el = time.perf_counter() - t0
        if el >= min_s or el > max_s:
            break
    el = time.perf_counter() - t0
    # one thread on the first 500,000 elements, for the per-core rate
    n1 = min(wl.n_elem, 500_000)
    t1 = time.perf_counter()
    oracle.integrate_workload(wl, threads=1, elements=np.arange(n1))
    single = n1 / (time.perf_counter() - t1)
    out = {"value": done / el, "unit": "elements/s", "cores": threads, "kind": "oracle",
           "sample": f"{done} elements ({passes} pass(es) over the {wl.n_elem}-element workload, "
                     f"chunks of {chunk}), {el:.1f} s wall, {threads} threads",
           "single_thread_value": single, "single_thread_sample": f"first {n1} elements"}
    out.update(cpu_description())
    return out


# ---------------------------------------------------------------- serving
SERVED_KINDS = [("tet4", "scalar"), ("tet4", "elasticity"), ("prism6", "scalar"),
                ("prism6", "elasticity")]


def served_requests(n_req, seed=5):
    """The mixed request stream: per request, in this order from one seeded
    stream: unit-rate exponential inter-arrival gap (scaled by 1/lambda
    later), n = exp(U[ln 1e3, ln 2e6]), element type 50/50, problem 70/30
    scalar CDR / elasticity, tier 50/50, mesh seed."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_req):
        gap = rng.exponential(1.0)
        n = int(round(np.exp(rng.uniform(np.log(1e3), np.log(2e6)))))
        elem = "tet4" if rng.random() < 0.5 else "prism6"
        prob = "scalar" if rng.random() < 0.7 else "elasticity"
        tier = "fp64" if rng.random() < 0.5 else "fp32"
        mseed = int(rng.integers(0, 2 ** 31))
        kind = SERVED_KINDS.index((elem, prob)) + (0 if tier == "fp64" else 4)
        out.append({"gap": gap, "n": n, "kind": kind, "elem": elem, "prob": prob, "tier": tier,
                    "seed": mseed})
    return out


def served_workload(r):
    """Request r's own mesh, built from its drawn seed: a jittered unit cube
    of about r["n"] elements (tets: N = max(1, round((n/6)^(1/3))) cells per
    side, 6 N^3 elements; prisms: n = L = max(1, round((n/2)^(1/3))),
    2 n^2 L elements), with per-element coefficients drawn as for the tet
    CDR (20 slots) or elasticity (E, nu, f) workloads."""
    from paper_1504_01023_amd import inputs
    seed = r["seed"]
    if r["elem"] == "tet4":
        N = inputs.tet_n_for(r["n"])
        return inputs.tet_cdr(N, seed) if r["prob"] == "scalar" else inputs.tet_elasticity(N, seed)
    m = inputs.prism_n_for(r["n"])
    return (inputs.prism_cdr_element(m, m, seed, sliver=False) if r["prob"] == "scalar"
            else inputs.prism_elasticity(m, m, seed, sliver=False))


def served_count(r):
    """Elements of request r's mesh (the formulas of served_workload)."""
    from paper_1504_01023_amd import inputs
    if r["elem"] == "tet4":
        return 6 * inputs.tet_n_for(r["n"]) ** 3
    return 2 * inputs.prism_n_for(r["n"]) ** 3


SLAB_BYTES = 1 << 32


class PinnedSlabs:
    """Pinned host memory carved into 256-byte aligned pieces from 4 GiB
    slabs (few large pinned allocations instead of one per request)."""

    def __init__(self, torch):
        self.torch = torch
        self.slabs = []
        self.used = SLAB_BYTES

    def take(self, nbytes, dtype, shape):
        torch = self.torch
        nb = (nbytes + 255) // 256 * 256
        if nb > SLAB_BYTES:
            raise ValueError("request larger than a slab")
        if self.used + nb > SLAB_BYTES:
            self.slabs.append(torch.empty(SLAB_BYTES, dtype=torch.uint8, pin_memory=True))
            self.used = 0
        v = self.slabs[-1][self.used:self.used + nbytes]
        self.used += nb
        return v.view(dtype).view(shape)


def served_payloads(reqs, torch, threads):
    """Every request's inputs in pinned host memory: SoA coordinates (FP64)
    and per-element coefficients in the request's tier, each with leading
    dimension n. Generated in parallel (numpy releases the interpreter lock
    in its array work); each request's arrays depend on its seed only."""
    import concurrent.futures as cf
    slabs = PinnedSlabs(torch)
    plan = []
    for r in reqs:
        n = served_count(r)
        nv = 4 if r["elem"] == "tet4" else 6
        rows_k = 20 if r["prob"] == "scalar" else 5
        dt = torch.float64 if r["tier"] == "fp64" else torch.float32
        c = slabs.take(8 * 3 * nv * n, torch.float64, (3 * nv, n))
        k = slabs.take((8 if r["tier"] == "fp64" else 4) * rows_k * n, dt, (rows_k, n))
        r["n_actual"] = n
        plan.append((r, c, k))

    def fill(item):
        r, c, k = item
        wl = served_workload(r)
        assert wl.n_elem == r["n_actual"] and wl.coeffs.shape == tuple(k.shape)
        c.copy_(torch.from_numpy(wl.mesh.coords))
        k.copy_(torch.from_numpy(wl.coeffs).to(k.dtype))
        return r["n_actual"]

    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(fill, plan))
    return [(c, k) for _, c, k in plan], slabs


def served_kinds(fe):
    """The eight served kinds: (tet, prism) x (CDR, elasticity) x (FP64, FP32),
    with the rules of the tet CDR (4 points), tet elasticity (1) and prism
    (6) workloads."""
    from paper_1504_01023_amd import inputs
    kinds = []
    for tier in ("fp64", "fp32"):
        for elem, prob in SERVED_KINDS:
            if elem == "tet4":
                wl = inputs.tet_cdr(1, 1) if prob == "scalar" else inputs.tet_elasticity(1, 1)
            else:
                wl = (inputs.prism_cdr_element(1, 1, 1, sliver=False) if prob == "scalar"
                      else inputs.prism_elasticity(1, 1, 1, sliver=False))
            kinds.append((fe.problem_for(wl, tier), elem, fe.builtin_rule(elem, wl.n_q)))
    return kinds


def run_served(a, torch, fe, serve, n_meas, n_warm, rhos, sample=20) -> dict:
    dev = torch.device("cuda:0")
    kinds = served_kinds(fe)
    reqs = served_requests(n_warm + n_meas)
    t0 = time.time()
    threads = host_threads()
    payloads, slabs = served_payloads(reqs, torch, threads)
    meas = reqs[n_warm:]
    mpay = payloads[n_warm:]
    tot_elems = sum(r["n_actual"] for r in meas)
    host_bytes = sum(c.numel() * c.element_size() + k.numel() * k.element_size()
                     for c, k in payloads)
    log(f"[served] {n_warm + n_meas} per-request meshes ({tot_elems} measured elements, "
        f"{host_bytes / 1e9:.1f} GB pinned) generated in {time.time() - t0:.1f}s on {threads} threads")

    stream = torch.cuda.current_stream()
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy2DAsync.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                     ctypes.c_size_t, ctypes.c_size_t, ctypes.c_size_t,
                                     ctypes.c_int, ctypes.c_void_p]

    def dev_ld(n):
        return (n + 3) // 4 * 4

    def h2d_rows(dst, src):
        """Copy a pinned (rows, n) host array into a device (rows, ld) array
        as the server does (one pitched copy)."""
        es = src.element_size()
        st = hip.hipMemcpy2DAsync(ctypes.c_void_p(dst.data_ptr()), dst.shape[1] * es,
                                  ctypes.c_void_p(src.data_ptr()), src.shape[1] * es,
                                  src.shape[1] * es, src.shape[0], 1,
                                  ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise RuntimeError(f"hipMemcpy2DAsync failed: {st}")

    # inputs staged on the device for the resident mode (rows padded to a
    # multiple of 4 elements, as the server pads its own copies)
    t0 = time.time()
    resident = []
    for (c, k), r in zip(mpay, meas):
        ld = dev_ld(r["n_actual"])
        dc = torch.empty((c.shape[0], ld), dtype=c.dtype, device=dev)
        dk = torch.empty((k.shape[0], ld), dtype=k.dtype, device=dev)
        h2d_rows(dc, c)
        h2d_rows(dk, k)
        resident.append((dc, dk))
    torch.cuda.synchronize()
    log(f"[served] resident copies staged in {time.time() - t0:.1f}s")

    def plain_one(i, r, pay, on_dev):
        k = kinds[r["kind"]]
        n = r["n_actual"]
        if on_dev:
            dc, dk = resident[i]
        else:
            c, kk = pay
            ld = dev_ld(n)
            dc = torch.empty((c.shape[0], ld), dtype=c.dtype, device=dev)
            dk = torch.empty((kk.shape[0], ld), dtype=kk.dtype, device=dev)
            h2d_rows(dc, c)
            h2d_rows(dk, kk)
        return fe.integrate(k[0], k[1], dc, dk, k[2], n_elem=n)

    # sequential plain service (the capacity): one request at a time through
    # fe_integrate, H2D of its inputs included or inputs resident
    for r, pay in zip(reqs[:n_warm], payloads[:n_warm]):
        plain_one(0, r, pay, False)
    torch.cuda.synchronize()
    seq = {}
    for on_dev in (False, True):
        ts = []
        for i, (r, pay) in enumerate(zip(meas, mpay)):
            w0 = time.perf_counter()
            plain_one(i, r, pay, on_dev)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - w0)
        seq["resident" if on_dev else "h2d"] = {
            "mean_service_s": float(np.mean(ts)), "elements_per_s": tot_elems / float(np.sum(ts)),
            "p50_s": float(np.percentile(ts, 50)), "p99_s": float(np.percentile(ts, 99))}
    log(f"[served] sequential plain: {seq}")

    def fetch(c, r):
        k = kinds[r["kind"]]
        dt_ = torch.float64 if r["tier"] == "fp64" else torch.float32
        out = []
        for ptr, rows in ((c.out_K, fe.k_entries(k[0], k[1])), (c.out_F, fe.f_entries(k[0], k[1]))):
            buf = torch.empty((rows, c.ld_out), dtype=dt_, device=dev)
            fe.lib().fe_stream_copy(ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(ptr),
                                    buf.numel() * buf.element_size(),
                                    ctypes.c_void_p(stream.cuda_stream))
            out.append(buf[:, :r["n_actual"]].contiguous().cpu().numpy())
        return out

    def serve_run(srv, rate, on_dev, sample_ids=()):
        """Submit the measured requests at the given arrival rate (None: all
        at t = 0), consume completions; latencies, and the outputs of
        sample_ids."""
        import threading
        srv.reset_stats()
        gaps = [r["gap"] for r in meas]
        arrivals = np.cumsum(gaps) / rate if rate else np.zeros(len(meas))
        outs = {}
        t_start = serve.now()
        done = []

        def submitter():
            for i, r in enumerate(meas):
                target = t_start + arrivals[i]
                while True:
                    dt = target - serve.now()
                    if dt <= 0:
                        break
                    time.sleep(min(dt, 0.002))
                if on_dev:
                    dc, dk = resident[i]
                    srv.submit(r["kind"], r["n_actual"], dc.data_ptr(), dk.data_ptr(),
                               on_device=True, ld_in=dc.shape[1], tag=i)
                else:
                    c, k = mpay[i]
                    srv.submit(r["kind"], r["n_actual"], c.data_ptr(), k.data_ptr(),
                               ld_in=c.shape[1], tag=i)

        th = threading.Thread(target=submitter)
        th.start()
        while len(done) < len(meas):
            for c in srv.poll(256, 0.01):
                if c.status != 0:
                    raise RuntimeError(f"served request failed with status {c.status}")
                if c.tag in sample_ids:
                    outs[c.tag] = fetch(c, meas[c.tag])
                srv.release(c.id)
                done.append(c)
        th.join()
        t_end = max(c.t_done for c in done)
        lat = np.array([c.t_done - c.t_submit for c in done])
        st = srv.stats()
        return {"requests": len(done), "elements": tot_elems,
                "elements_per_s": tot_elems / (t_end - t_start),
                "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "mean_s": float(lat.mean()),
                "mean_queue_s": st["mean_queue_s"], "mean_h2d_s": st["mean_h2d_s"],
                "mean_device_s": st["mean_device_s"], "ticks": st["ticks"],
                "peak_bytes": st["bytes_peak"]}, outs

    budget = 64 << 30
    counts = {}
    for r in meas:
        key = f"{r['elem']}/{r['prob']}/{r['tier']}"
        counts[key] = counts.get(key, 0) + 1
    out = {"n_requests": n_meas, "warmup_requests": n_warm, "total_elements": tot_elems,
           "mean_elements_per_request": tot_elems / n_meas,
           "requests_by_kind": counts,
           "meshes": "one jittered cube mesh per request, built from the request's drawn seed",
           "hbm_budget_bytes": budget, "max_slots": a.served_slots, "sequential_plain": seq}
    rng = np.random.default_rng(55)
    sample_ids = set(int(x) for x in rng.choice(n_meas, size=min(sample, n_meas), replace=False))
    with serve.Server(kinds, max_slots=a.served_slots, hbm_budget_bytes=budget, max_chunks=2048,
                      chunk_elems=4096, blocks_per_kind=a.served_blocks_per_kind) as srv:
        for r, (c, k) in zip(reqs[:n_warm], payloads[:n_warm]):
            srv.submit(r["kind"], r["n_actual"], c.data_ptr(), k.data_ptr(), ld_in=c.shape[1])
        got = 0
        while got < n_warm:
            for c in srv.poll(64, 0.05):
                srv.release(c.id)
                got += 1
        sat, mix_out = serve_run(srv, None, False, sample_ids)
        out["saturation"] = sat
        out["served_speedup"] = sat["elements_per_s"] / seq["h2d"]["elements_per_s"]
        log(f"[served] saturation: {sat}")
        sat_r, _ = serve_run(srv, None, True)
        out["saturation_resident"] = sat_r
        out["served_speedup_resident"] = sat_r["elements_per_s"] / seq["resident"]["elements_per_s"]
        cap = 1.0 / seq["h2d"]["mean_service_s"]
        cap_r = 1.0 / seq["resident"]["mean_service_s"]
        out["load"] = {}
        for rho in rhos:
            res, _ = serve_run(srv, rho * cap, False)
            res_r, _ = serve_run(srv, rho * cap_r, True)
            out["load"][f"rho_{rho}"] = {"rate_per_s": rho * cap, "h2d": res,
                                         "rate_resident_per_s": rho * cap_r, "resident": res_r}
            log(f"[served] rho {rho}: p50 {res['p50_s']*1e3:.2f} ms p99 {res['p99_s']*1e3:.2f} ms; "
                f"resident p50 {res_r['p50_s']*1e3:.2f} ms p99 {res_r['p99_s']*1e3:.2f} ms")
        # the sampled requests again, one at a time through the server: the
        # same bits alone as in the mix
        same = 0
        for i in sorted(sample_ids):
            r = meas[i]
            c, k = mpay[i]
            srv.submit(r["kind"], r["n_actual"], c.data_ptr(), k.data_ptr(), ld_in=c.shape[1], tag=i)
            got = []
            while not got:
                got = srv.poll(4, 0.05)
            alone = fetch(got[0], r)
            same += int(all(np.array_equal(x, y) for x, y in zip(alone, mix_out[i])))
            srv.release(got[0].id)
        out["alone_vs_mix_bitwise_equal"] = f"{same}/{len(sample_ids)}"
    del resident, payloads, mpay, slabs
    torch.cuda.empty_cache()
    return out


# ------------------------------------------- the paper's order experiment
# The four cases of Sec. 4.1 / Table 7 (words per element and operation
# counts of Table 4 for the QSS, SQS and SSQ orders) and the measured
# Tesla K20m times of Table 7 (ns per element), quoted as context.
PAPER_CASES = [
    # (name, workload, words, {order: paper ops}, {order: K20m ns})
    ("tet Poisson", "tet_poisson_qp", 36, {"QSS": 290, "SQS": 290, "SSQ": 290},
     {"QSS": 2.02, "SQS": 2.02, "SSQ": 2.02}),
    ("prism Poisson", "prism_poisson_qp", 66, {"QSS": 2700, "SQS": 10416, "SSQ": 54876},
     {"QSS": 12.80, "SQS": 38.39, "SSQ": 94.99}),
    ("tet conv-diff", "tet_cdr", 52, {"QSS": 986, "SQS": 986, "SSQ": 1623},
     {"QSS": 4.46, "SQS": 6.05, "SSQ": 6.13}),
    ("prism conv-diff", "prism_cdr", 80, {"QSS": 4806, "SQS": 12492, "SSQ": 65232},
     {"QSS": 15.58, "SQS": 64.81, "SSQ": 194.93}),
]
ORDER_CODE = {"QSS": 1, "SQS": 2, "SSQ": 3}


def model_bound_ns(words: float, ops: float, stream_gbps: float, dgemm_tflops: float) -> float:
    """The execution-time estimate of Sec. 4.5 (the table of execution
    times): the longer of the time to move 8-byte words at the STREAM rate
    and the time to perform the operations at the DGEMM rate, in ns per
    element."""
    return max(8.0 * words / stream_gbps, ops / (dgemm_tflops * 1e3))


def run_paper(a, torch, fe) -> dict:
    import oracle
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    # the model's two "benchmark" rates, measured here: a streaming copy and
    # an FP64 matrix product (the paper used STREAM and DGEMM)
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        fe.stream_copy(dst, src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(20):
        fe.stream_copy(dst, src)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbps = 2 * src.numel() * 8 * 20 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    m = 8192
    A = torch.rand((m, m), dtype=torch.float64, device=dev)
    B = torch.rand((m, m), dtype=torch.float64, device=dev)
    for _ in range(2):
        torch.matmul(A, B)
    e0.record(stream)
    for _ in range(5):
        torch.matmul(A, B)
    e1.record(stream)
    torch.cuda.synchronize()
    dgemm_tf = 2 * m ** 3 * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e12
    del A, B
    log(f"[paper] copy {copy_gbps:.0f} GB/s, FP64 matmul {dgemm_tf:.1f} TFLOP/s")
    rows = []
    for name, wname, words, ops, k20 in PAPER_CASES:
        wl = WORKLOADS[wname][0]()
        dw = fe.to_device(wl, "fp64", device=dev)
        p, rule = dw.problem, dw.rule
        K = torch.empty((fe.k_entries(p, wl.elem), wl.n_elem), dtype=torch.float64, device=dev)
        F = torch.empty((fe.f_entries(p, wl.elem), wl.n_elem), dtype=torch.float64, device=dev)
        orders = ["QSS", "SQS", "SSQ"] if wl.elem == "prism6" else ["QSS"]
        for order in orders:
            best = None
            for wg in (64, 128, 256):
                for nt in (1, 2):
                    v = fe.variant(wg_size=wg, nontemporal=nt, loop_order=ORDER_CODE[order],
                                   elems_per_thread=2 if wl.elem == "tet4" else 1)
                    try:
                        fe.integrate(p, wl.elem, dw.coords, dw.coeffs, rule, K, F, variant=v)
                    except fe.FeError:
                        continue
                    e0.record(stream)
                    for _ in range(5):
                        fe.integrate(p, wl.elem, dw.coords, dw.coeffs, rule, K, F, variant=v)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    ms = e0.elapsed_time(e1) / 5
                    if best is None or ms < best[0]:
                        best = (ms, (wg, nt))
            ms, (wg, nt) = best
            fe.integrate(p, wl.elem, dw.coords, dw.coeffs, rule, K, F,
                         variant=fe.variant(wg_size=wg, nontemporal=nt, loop_order=ORDER_CODE[order],
                                            elems_per_thread=2 if wl.elem == "tet4" else 1))
            torch.cuda.synchronize()
            sample = np.arange(0, wl.n_elem, max(1, wl.n_elem // 2000))
            idx = torch.from_numpy(sample).to(dev)
            Ks = K.index_select(1, idx).cpu().numpy()
            Fs = F.index_select(1, idx).cpu().numpy()
            Ko, Fo = oracle.integrate(wl.elem, wl.kind, wl.mesh.coords[:, sample],
                                      oracle.quad_rule(wl.elem, wl.n_q), wl.coef_mode, wl.mask,
                                      wl.uniform, None if wl.coeffs is None else wl.coeffs[:, sample],
                                      threads=host_threads())
            N = oracle.n_dof(wl.elem, wl.kind)
            Kg = fe.unpack_full(Ks, N, False)
            ek = float(np.sqrt(((Kg - Ko) ** 2).sum(axis=(1, 2)) / (Ko ** 2).sum(axis=(1, 2))).max())
            ns = ms * 1e6 / wl.n_elem
            bound = model_bound_ns(words, ops[order], copy_gbps, dgemm_tf)
            rows.append({"case": name, "order": order, "n_elem": wl.n_elem, "ns_per_element": ns,
                         "elements_per_s": wl.n_elem / (ms * 1e-3),
                         "GBps": 8 * words * wl.n_elem / (ms * 1e-3) / 1e9,
                         "model_bound_ns": bound, "pct_of_bound": 100 * bound / ns,
                         "K20m_ns": k20[order], "speedup_vs_K20m": k20[order] / ns,
                         "variant_wg_nt": [wg, nt], "parity_max_rel_err_K": ek})
            log(f"[paper] {name:16s} {order}: {ns:.3f} ns/elem ({100 * bound / ns:.0f}% of bound "
                f"{bound:.3f}), K20m {k20[order]} ns, parity {ek:.1e}")
        del dw, K, F
        torch.cuda.empty_cache()
    return {"copy_GBps": copy_gbps, "fp64_matmul_TFLOPs": dgemm_tf, "rows": rows}


NATURAL_BASES = ("tet_poisson", "tet_poisson_qp", "tet_cdr", "tet_elasticity", "prism_cdr",
                 "prism_poisson_qp", "prism_cdr_qp", "prism_elasticity", "tet_vector",
                 "prism_vector")
APPLY_BASES = ("tet_poisson", "tet_cdr", "tet_elasticity", "prism_cdr", "prism_poisson_qp",
               "prism_elasticity", "tet_vector", "prism_vector")


def run_apply(a, torch, fe, oracle, base: str, dev, csr: bool = False) -> dict:
    """Matrix-free operator application y += A x over the whole mesh (element
    matrices formed in registers, never stored), coloured launches with plain
    updates; one step = one application. Parity: y at sampled nodes against
    the oracle's element matrices of every element touching them.

    csr: the assembly of the global matrix into CSR storage instead (one
    step = one assembly, values += A); parity: the sampled nodes' rows."""
    from paper_1504_01023_amd import inputs
    wl = WORKLOADS[base][0]()
    if a.apply_order != "generator":
        t0 = time.time()
        wl = inputs.reordered(wl, a.apply_order)
        log(f"[bench] {a.apply_order} node and element order ({time.time() - t0:.1f}s)")
    nodes_np, conn_np = wl.mesh.nodes, wl.mesh.conn
    n, nv = conn_np.shape
    n_nodes = nodes_np.shape[0]
    t0 = time.time()
    perm, ptr = fe.color_elements(wl.elem, conn_np, n_nodes)
    log(f"[bench] {n} elements, {n_nodes} nodes, {len(ptr) - 1} colours ({time.time() - t0:.1f}s)")
    dw = fe.to_device(wl, a.precision, device=dev)
    p, rule = dw.problem, dw.rule
    conn = torch.from_numpy(np.ascontiguousarray(conn_np[perm].T.astype(np.int32))).to(dev)
    coeffs = dw.coeffs
    if coeffs is not None and wl.coef_mode not in ("uniform", "function"):
        coeffs = coeffs[:, torch.from_numpy(perm.astype(np.int64)).to(dev)].contiguous()
    del dw
    nodes = torch.from_numpy(nodes_np).to(dev).contiguous()
    nc = 1 if wl.kind == "scalar" else 3
    dt = torch.float64 if a.precision == "fp64" else torch.float32
    tsz = 8 if a.precision == "fp64" else 4
    x64 = np.random.default_rng(7).standard_normal(n_nodes * nc)
    x = torch.from_numpy(x64).to(device=dev, dtype=dt)
    y = torch.zeros_like(x)
    stream = torch.cuda.current_stream()
    if csr:
        t0 = time.time()
        rp, ci = fe.csr_pattern(wl.elem, conn_np, n_nodes, nc)
        log(f"[bench] CSR pattern: {len(ci)} entries ({time.time() - t0:.1f}s)")
        rpd = torch.from_numpy(rp).to(dev)
        cid = torch.from_numpy(ci).to(dev)
        vals = torch.zeros(len(ci), dtype=dt, device=dev)
        ip, inc = fe.node_incidence(wl.elem, conn_np[perm], n_nodes)
        ipd = torch.from_numpy(ip).to(dev)
        incd = torch.from_numpy(inc).to(dev)
        # node blocks for the LDS-staged row ownership (scalar tets)
        bld = None
        if wl.elem == "tet4" and wl.kind == "scalar":
            t0 = time.time()
            blocks = fe.csr_blocks(wl.elem, conn_np[perm], n_nodes, ip, inc, rp, ci)
            bld = blocks.to(dev)
            log(f"[bench] node blocks: {blocks.n_blocks}, element slots "
                f"{len(blocks.elems) / n:.2f} per element ({time.time() - t0:.1f}s)")

    def step(cp=ptr):
        if csr:
            fe.assemble_csr(p, wl.elem, nodes, conn, coeffs, rule, rpd, cid, values=vals,
                            color_ptr=cp)
        else:
            fe.apply_indexed(p, wl.elem, nodes, conn, coeffs, rule, x, y, None, color_ptr=cp)

    def step_rows():
        fe.assemble_csr_rows(p, wl.elem, nodes, conn, coeffs, rule, rpd, cid, ipd, incd,
                             values=vals)

    def step_blocks():
        fe.assemble_csr_blocks(p, wl.elem, nodes, coeffs, rule, rpd, cid, ipd, bld, values=vals)

    if csr:
        # element-contiguous inputs and outputs for the stored schedule
        x_nat = torch.from_numpy(np.ascontiguousarray(
            nodes_np[conn_np[perm]].reshape(n, 3 * nv))).to(dev)
        c_nat = coeffs
        if coeffs is not None and wl.coef_mode not in ("uniform", "function"):
            c_nat = coeffs.t().contiguous()
        Kst = torch.empty((n, fe.k_entries(p, wl.elem)), dtype=dt, device=dev)
        Fst = torch.empty((n, fe.f_entries(p, wl.elem)), dtype=dt, device=dev)

    def step_stored():
        # integrate with K, F stored element by element, then assemble the
        # stored matrices by rows
        fe.integrate_natural(p, wl.elem, x_nat, c_nat, rule, out_K=Kst, out_F=Fst)
        fe.assemble_csr_stored(p, wl.elem, conn, n_nodes, Kst, Fst, rpd, cid, ipd, incd,
                               values=vals, elem_major=True)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(a.steps)]
    w0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    # the same application as one launch with atomic adds (order-dependent
    # last bits), timed the same way
    ev_at = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(a.steps)]
    for _ in range(a.warmup):
        step(None)
    for e0, e1 in ev_at:
        e0.record(stream)
        step(None)
        e1.record(stream)
    torch.cuda.synchronize()
    ms_at = np.array([e0.elapsed_time(e1) for e0, e1 in ev_at])
    ms_rows = ms_blocks = None

    def timed(fn):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(a.steps)]
        for _ in range(a.warmup):
            fn()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for e0, e1 in evs:
            e0.record(stream)
            fn()
            e1.record(stream)
        torch.cuda.synchronize()
        return np.array([e0.elapsed_time(e1) for e0, e1 in evs]), time.perf_counter() - w0

    if csr:
        # by row ownership (one lane per node, no colours, no atomics), plain
        # and over node blocks staged in LDS
        ms_rows, wall_rows = timed(step_rows)
        wall = wall_rows
        if bld is not None:
            ms_blocks, wall = timed(step_blocks)
        ev_s = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for _ in range(a.steps)]
        for _ in range(a.warmup):
            step_stored()
        for e0, e1 in ev_s:
            e0.record(stream)
            step_stored()
            e1.record(stream)
        torch.cuda.synchronize()
        ms_stored = np.array([e0.elapsed_time(e1) for e0, e1 in ev_s])
    # one clean application (assembly) for the parity check
    (vals if csr else y).zero_()
    step()
    torch.cuda.synchronize()
    rng = np.random.default_rng(99)
    snodes = rng.choice(n_nodes, size=min(2000, n_nodes), replace=False)
    mark = np.zeros(n_nodes, dtype=bool)
    mark[snodes] = True
    touch = np.nonzero(mark[conn_np].any(axis=1))[0]
    cf = None
    if wl.coeffs is not None and wl.coef_mode == "function":
        cf = wl.coeffs
    elif wl.coeffs is not None:
        cf = wl.coeffs[:, touch]
        if a.precision == "fp32":
            cf = cf.astype(np.float32).astype(np.float64)
    K, _ = oracle.integrate(wl.elem, wl.kind, wl.mesh.coords[:, touch], oracle.quad_rule(wl.elem, wl.n_q),
                            wl.coef_mode, wl.mask, wl.uniform, cf, threads=host_threads())
    dof = (conn_np[touch][:, :, None] * nc + np.arange(nc)[None, None, :]).reshape(len(touch), nv * nc)
    sd = (snodes[:, None] * nc + np.arange(nc)[None, :]).ravel()
    tol = 1e-12 if a.precision == "fp64" else 2e-5
    ncoef = fe.coeff_entries(p, wl.elem, rule.n_q) if wl.coef_mode != "function" else 0
    if csr:
        # rows of the sampled unknowns: the oracle's element matrices added at
        # their couplings, against the GPU's CSR rows; rounding relative to
        # the row's largest sum of |K^e|
        import scipy.sparse as sp
        nd = n_nodes * nc
        rows = np.repeat(dof[:, :, None], dof.shape[1], axis=2).ravel()
        cols = np.repeat(dof[:, None, :], dof.shape[1], axis=1).ravel()
        R = sp.csr_matrix((K.ravel(), (rows, cols)), shape=(nd, nd))[sd]
        Ra = sp.csr_matrix((np.abs(K).ravel(), (rows, cols)), shape=(nd, nd))[sd]
        den = np.maximum(Ra.max(axis=1).toarray().ravel(), 1e-300)
        err = 0.0
        rows_vals = None
        blocks_equal = None
        for mode in ("coloured", "rows", "blocks"):
            if mode == "blocks" and bld is None:
                continue
            if mode != "coloured":
                vals.zero_()
                (step_rows if mode == "rows" else step_blocks)()
                torch.cuda.synchronize()
            if mode == "rows":
                rows_vals = vals.clone()
            if mode == "blocks":
                blocks_equal = bool(torch.equal(rows_vals, vals))
            G = sp.csr_matrix((vals.double().cpu().numpy(), ci, rp), shape=(nd, nd))[sd]
            D = abs(G - R)
            err = max(err, float((D.max(axis=1).toarray().ravel() / den).max()))
        nnz = len(ci)
        # inputs once, the pattern once, every value read and written once
        bpe = 4 * nv + tsz * ncoef + (24 * n_nodes + 8 * (nd + 1) + (4 + 2 * tsz) * nnz) / n
    else:
        yg = y.double().cpu().numpy()
        xo = x.double().cpu().numpy()
        yr = np.zeros(n_nodes * nc)
        ya = np.zeros(n_nodes * nc)
        np.add.at(yr, dof.ravel(), np.einsum("ers,es->er", K, xo[dof]).ravel())
        np.add.at(ya, dof.ravel(), np.einsum("ers,es->er", np.abs(K), np.abs(xo[dof])).ravel())
        err = float((np.abs(yg[sd] - yr[sd]) / np.maximum(ya[sd], 1e-300)).max())
        bpe = 4 * nv + tsz * ncoef + (24 + 3 * tsz * nc) * n_nodes / n
    if csr:
        # the value is the row-ownership assembly (over node blocks where they
        # are built); the coloured one beside it
        ms, ms_col = (ms_blocks if ms_blocks is not None else ms_rows), ms
    avg = float(ms.mean()) * 1e-3
    return {"wl": wl, "n_elem": n, "n_nodes": n_nodes, "colours": int(len(ptr) - 1),
            "ms_avg": float(ms.mean()), "ms_min": float(ms.min()), "ms_median": float(np.median(ms)),
            "wall_s": wall,
            "stored_ms_avg": float(ms_stored.mean()) if csr else None,
            "stored_elements_per_s": n / (float(ms_stored.mean()) * 1e-3) if csr else None,
            "coloured_ms_avg": float(ms_col.mean()) if csr else None,
            "coloured_elements_per_s": n / (float(ms_col.mean()) * 1e-3) if csr else None,
            "atomic_ms_avg": float(ms_at.mean()), "atomic_elements_per_s": n / (float(ms_at.mean()) * 1e-3),
            "elements_per_s": n / avg, "bytes_per_element": bpe,
            "achieved_GBps": bpe * n / avg / 1e9,
            "nnz": int(len(ci)) if csr else None,
            "rows_ms_avg": float(ms_rows.mean()) if csr else None,
            "rows_elements_per_s": n / (float(ms_rows.mean()) * 1e-3) if csr else None,
            "blocks": ({"n_blocks": int(bld.n_blocks),
                        "element_slots_per_element": float(bld.elems.numel() / n),
                        "vertex_slots_per_node": float(bld.verts.numel() / n_nodes)}
                       if csr and bld is not None else None),
            "parity": {"sampled_nodes": int(len(snodes)),
                       ("max_rel_err_rows" if csr else "max_rel_err_y"): err, "tol": tol,
                       "ok": bool(err <= tol and (not csr or blocks_equal is not False)),
                       **({"blocks_equal_rows_bitwise": blocks_equal} if csr else {})}}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="tet_poisson",
                    choices=sorted(WORKLOADS) + [w + "_indexed" for w in sorted(WORKLOADS)]
                    + [w + "_apply" for w in APPLY_BASES]
                    + [w + "_csr" for w in APPLY_BASES]
                    + [w + "_natural" for w in NATURAL_BASES]
                    + ["served", "paper"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--tune", action="store_true",
                    help="run the exhaustive variant search (fe_autotune) during warm-up")
    ap.add_argument("--tuning-file", default=None,
                    help="tuning table to load over the library's built-in one (the committed "
                         "MI355X table, compiled in)")
    ap.add_argument("--save-tuning", default=None, help="write the tuning table here after the run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--parity-sample", type=int, default=20000)
    ap.add_argument("--apply-order", default="morton", choices=["morton", "generator"],
                    help="node and element order of the matrix-free runs: Z-order renumbering, "
                         "or the generator's lexicographic order")
    ap.add_argument("--ld-align", type=int, default=256,
                    help="leading dimension of inputs and outputs: a multiple of this many "
                         "elements (256: the library's default, fe_ld_for; 0: ld = n_elem)")
    ap.add_argument("--served-requests", type=int, default=1000)
    ap.add_argument("--served-blocks-per-kind", type=int, default=0,
                    help="workgroups of each kind's persistent batched kernel (0: the library's default)")
    ap.add_argument("--served-warmup", type=int, default=50)
    ap.add_argument("--served-slots", type=int, default=64)
    ap.add_argument("--served-rho", type=float, nargs="*", default=[0.5, 0.7, 0.9])
    ap.add_argument("--workloads", default=None,
                    help="several workloads in one process, e.g. tet_cdr:fp64,prism_cdr:fp32 "
                         "(one JSON line each; for profiling runs that cover many kernels)")
    ap.add_argument("--headline-only", action="store_true",
                    help="default workload: only the FP64 line, without the FP32 tier and the "
                         "served summary")
    ap.add_argument("--summary-served-requests", type=int, default=1000,
                    help="measured requests of the served summary in the default run")
    a = ap.parse_args()

    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              "(elements are independent, so a multi-GPU run would shard contiguous element "
              "ranges with no communication).", file=sys.stderr)
        return 2

    import torch

    import oracle
    from paper_1504_01023_amd import fe

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if a.workload == "paper":
        res = run_paper(a, torch, fe)
        line = {"metric": "ns per element by loop order (the paper's Table 7 experiment on MI355X)",
                "value": None, "unit": "ns/element", "n_gpus": 1, "steps": 5, "warmup": 1,
                "ms_per_step": None, "higher_is_better": False, "scaling": "weak",
                "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                "config": {"workload": "paper"}, "paper": res}
        print(json.dumps(line), flush=True)
        return 0

    if a.workload.endswith("_apply") or a.workload.endswith("_csr"):
        csr = a.workload.endswith("_csr")
        base = a.workload[: -len("_csr" if csr else "_apply")]
        r = run_apply(a, torch, fe, oracle, base, dev, csr)
        # a counter reading stored for this workload's timed kernel is used
        # while the sources that define it are unchanged
        shash = (source_hash(base, a.precision) if (base, a.precision) in KERNEL_UNITS
                 else None)
        traffic = stored_traffic(a.workload, a.precision, shash) if shash else None
        line = {"metric": ("elements/s of assembly into CSR storage (K^e never stored)" if csr else
                           "elements/s of matrix-free operator application (K^e never stored)"),
                "value": r["elements_per_s"], "unit": "elements/s", "n_gpus": 1, "steps": a.steps,
                "warmup": a.warmup, "ms_per_step": r["wall_s"] * 1e3 / a.steps,
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f64" if a.precision == "fp64" else "f32 (FP64 Jacobian)",
                "data": "synthetic",
                "config": {"workload": a.workload,
                           "description": WORKLOADS[base][1] + (
                               ("; values += A, one lane per node (row ownership"
                                + (", node blocks staged in LDS)" if r["blocks"] else ")"))
                               if csr else "; y += A x, coloured launches"),
                           "n_elem": r["n_elem"], "n_nodes": r["n_nodes"], "colours": r["colours"],
                           "nnz": r["nnz"],
                           "node_element_order": a.apply_order,
                           "precision": a.precision, "bytes_per_element": r["bytes_per_element"],
                           "parallelism": "single GPU"},
                "roofline": {"bound": "hbm", "achieved": r["achieved_GBps"], "peak": HBM_PEAK_GBPS,
                             "unit": "GB/s", "frac": r["achieved_GBps"] / HBM_PEAK_GBPS,
                             "traffic": traffic},
                "cpu_baseline": None, "kernel_ms_avg": r["ms_avg"], "kernel_ms_min": r["ms_min"],
                "kernel_ms_median": r["ms_median"],
                "atomic": {"ms_avg": r["atomic_ms_avg"], "elements_per_s": r["atomic_elements_per_s"]},
                "coloured": ({"ms_avg": r["coloured_ms_avg"],
                              "elements_per_s": r["coloured_elements_per_s"]} if csr else None),
                "row_ownership_plain": ({"ms_avg": r["rows_ms_avg"],
                                         "elements_per_s": r["rows_elements_per_s"]}
                                        if csr else None),
                "node_blocks": r["blocks"],
                "stored": ({"ms_avg": r["stored_ms_avg"], "elements_per_s": r["stored_elements_per_s"],
                            "what": "fe_integrate_natural (K, F stored element by element) + "
                                    "fe_assemble_csr_stored"}
                           if csr else None),
                "parity": r["parity"], "kernel_source_hash": shash}
        print(json.dumps(line), flush=True)
        return 0 if r["parity"]["ok"] else 3

    if a.workload == "served":
        from paper_1504_01023_amd import serve
        if a.tuning_file:
            fe.tuning_load(a.tuning_file)
        res = run_served(a, torch, fe, serve, a.served_requests, a.served_warmup, a.served_rho)
        sat = res["saturation"]
        line = {"metric": "served elements/s (continuous batching, mixed stream, H2D included)",
                "value": sat["elements_per_s"], "unit": "elements/s", "n_gpus": 1,
                "steps": res["n_requests"], "warmup": res["warmup_requests"],
                "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "f64/f32 mix", "data": "synthetic",
                "config": {"workload": "served", "mix": SERVED_MIX}, "served": res}
        print(json.dumps(line), flush=True)
        return 0

    if a.workloads:
        ok = True
        for item in a.workloads.split(","):
            w, _, prec = item.partition(":")
            r = measure_plain(a, torch, fe, oracle, w, prec or "fp64", dev, a.parity_sample,
                              with_cpu=False)
            print(json.dumps(r), flush=True)
            ok = ok and r["parity"]["ok"]
        return 0 if ok else 3

    out = measure_plain(a, torch, fe, oracle, a.workload, a.precision, dev, a.parity_sample,
                        with_cpu=not a.no_cpu)
    if a.workload == "tet_poisson" and a.precision == "fp64" and not a.headline_only:
        # the rest of the metric: the FP32 bulk tier of the same workload and
        # the served mixed stream, against the plain FP64 form on this GPU
        t0 = time.time()
        f32 = measure_plain(a, torch, fe, oracle, "tet_poisson", "fp32", dev,
                            min(a.parity_sample, 5000), with_cpu=False)
        bpe64, bpe32 = out["config"]["bytes_per_element"], f32["config"]["bytes_per_element"]
        out["fp32"] = {
            "workload": "tet_poisson", "precision": "fp32 (FP64 Jacobian terms)",
            "value": f32["value"], "unit": "elements/s", "ms_per_step": f32["ms_per_step"],
            "kernel_ms_avg": f32["kernel_ms_avg"], "roofline": f32["roofline"],
            "speedup_vs_fp64": f32["value"] / out["value"],
            "speedup_vs_fp64_kernel": out["kernel_ms_avg"] / f32["kernel_ms_avg"],
            "byte_bound_speedup": bpe64 / bpe32,
            "max_rel_err_vs_fp64_oracle": {"K": f32["parity"]["max_rel_err_K"],
                                           "F": f32["parity"]["max_rel_err_F"],
                                           "sampled_elements": f32["parity"]["sampled_elements"],
                                           "tol": f32["parity"]["tol"], "ok": f32["parity"]["ok"]},
            "access_pattern": f32["access_pattern"],
            "kernel_source_hash": f32["kernel_source_hash"]}
        log(f"[bench] fp32 tier: {f32['value']:.3e} elements/s ({time.time() - t0:.1f}s)")
        t0 = time.time()
        from paper_1504_01023_amd import serve
        res = run_served(a, torch, fe, serve, a.summary_served_requests,
                         max(1, a.summary_served_requests // 20), [0.7])
        rho = res["load"]["rho_0.7"]
        out["served"] = {
            "mix": SERVED_MIX, "n_requests": res["n_requests"],
            "warmup_requests": res["warmup_requests"], "total_elements": res["total_elements"],
            "requests_by_kind": res["requests_by_kind"], "meshes": res["meshes"],
            "hbm_budget_bytes": res["hbm_budget_bytes"], "max_slots": res["max_slots"],
            "saturation_elements_per_s": {"h2d": res["saturation"]["elements_per_s"],
                                          "resident": res["saturation_resident"]["elements_per_s"]},
            "sequential_plain_elements_per_s": {
                "h2d": res["sequential_plain"]["h2d"]["elements_per_s"],
                "resident": res["sequential_plain"]["resident"]["elements_per_s"]},
            "served_speedup": {"h2d": res["served_speedup"],
                               "resident": res["served_speedup_resident"]},
            "rho_0.7": {mode: {"p50_ms": rho[mode]["p50_s"] * 1e3, "p99_ms": rho[mode]["p99_s"] * 1e3,
                               "mean_ms": rho[mode]["mean_s"] * 1e3,
                               "mean_queue_ms": rho[mode]["mean_queue_s"] * 1e3,
                               "mean_h2d_ms": rho[mode]["mean_h2d_s"] * 1e3,
                               "mean_device_ms": rho[mode]["mean_device_s"] * 1e3}
                        for mode in ("h2d", "resident")},
            "saturation_split_ms": {
                "mean_queue_ms": res["saturation"]["mean_queue_s"] * 1e3,
                "mean_h2d_ms": res["saturation"]["mean_h2d_s"] * 1e3,
                "mean_device_ms": res["saturation"]["mean_device_s"] * 1e3},
            "alone_vs_mix_bitwise_equal": res["alone_vs_mix_bitwise_equal"]}
        log(f"[bench] served summary ({time.time() - t0:.1f}s)")
    print(json.dumps(out), flush=True)
    ok = out["parity"]["ok"] and (out.get("fp32") is None or out["fp32"]["max_rel_err_vs_fp64_oracle"]["ok"])
    return 0 if ok else 3


SERVED_MIX = ("50/50 tet/prism, 70/30 CDR/elasticity, 50/50 FP64/FP32, n log-uniform in "
              "[1e3, 2e6], Poisson arrivals, seed 5")


def measure_plain(a, torch, fe, oracle, workload, precision, dev, parity_sample, with_cpu):
    """One workload through fe_integrate (or its indexed / natural forms):
    warm-up, K timed steps, a sampled parity check against the oracle, and
    the JSON record of the measurement."""
    indexed = workload.endswith("_indexed")
    natural = workload.endswith("_natural")
    base = workload[: -len("_indexed")] if indexed else (
        workload[: -len("_natural")] if natural else workload)
    t0 = time.time()
    wl = WORKLOADS[base][0]()
    log(f"[bench] generated {workload}: {wl.n_elem} elements in {time.time() - t0:.1f}s")
    # The library's default layout: fe.to_device puts the input rows in
    # buffers of fe_ld_for(n) columns (whole 2 KiB / 1 KiB lines of FP64 /
    # FP32 elements per row) and the outputs take the same leading
    # dimension, so every wavefront reads and writes whole cache lines of
    # every row; rows that start mid-line leave partial lines at both ends of
    # every wavefront's segment and cut the write rate. --ld-align 0 runs
    # the unpadded layout (ld = n) for comparison.
    dw = fe.to_device(wl, precision, device=dev)
    p, rule = dw.problem, dw.rule
    n = wl.n_elem
    if natural:
        ld = n
    elif a.ld_align == 256:
        ld = fe.ld_for(n)
    else:
        ld = (n + a.ld_align - 1) // a.ld_align * a.ld_align if a.ld_align > 0 else n

        def relaid(t):
            out = torch.zeros((t.shape[0], ld), dtype=t.dtype, device=dev)
            out[:, :n] = t
            return out[:, :n]

        dw.coords = relaid(dw.coords)
        if dw.coeffs is not None and wl.coef_mode != "function":
            dw.coeffs = relaid(dw.coeffs)
    nk, nf = fe.k_entries(p, wl.elem), fe.f_entries(p, wl.elem)
    dt = torch.float64 if precision == "fp64" else torch.float32
    ld_out = ld
    K = torch.empty((nk, ld_out), dtype=dt, device=dev)[:, :n]
    F = torch.empty((nf, ld_out), dtype=dt, device=dev)[:, :n]
    bpe = fe.bytes_per_element(p, wl.elem, rule.n_q)
    stream = torch.cuda.current_stream()
    nv = 4 if wl.elem == "tet4" else 6
    if indexed:
        # per element: connectivity (4 B per vertex) instead of 24 B per vertex
        # of coordinates, plus every node's 24 B read once
        nodes = torch.from_numpy(wl.mesh.nodes).to(dev).contiguous()
        conn = torch.from_numpy(np.ascontiguousarray(wl.mesh.conn.T.astype(np.int32))).to(dev)
        bpe = bpe - 24 * nv + 4 * nv + 24.0 * wl.mesh.nodes.shape[0] / wl.n_elem

    if natural:
        # element-contiguous inputs and outputs; K and F below are row views
        # of the natural-order outputs for the parity sample
        x_nat = dw.coords.t().contiguous()
        c_nat = dw.coeffs
        if c_nat is not None and wl.coef_mode != "function":
            c_nat = c_nat.t().contiguous()
        K_nat = torch.empty((wl.n_elem, nk), dtype=dt, device=dev)
        F_nat = torch.empty((wl.n_elem, nf), dtype=dt, device=dev)
        K, F = K_nat.t(), F_nat.t()

    def step():
        if natural:
            fe.integrate_natural(p, wl.elem, x_nat, c_nat, rule, out_K=K_nat, out_F=F_nat)
        elif indexed:
            fe.integrate_indexed(p, wl.elem, nodes, conn, dw.coeffs, rule, out_K=K, out_F=F,
                                 n_elem=wl.n_elem)
        else:
            fe.integrate(p, wl.elem, dw.coords, dw.coeffs, rule, out_K=K, out_F=F, n_elem=wl.n_elem)

    if a.tuning_file:
        fe.tuning_load(a.tuning_file)
    if not natural and (a.tune or fe.tuning_get(p, wl.elem, rule.n_q) is None):
        tuned, tms = fe.autotune(p, wl.elem, dw.coords, dw.coeffs, rule, K, F, reps=5,
                                 n_elem=wl.n_elem)
        log(f"[bench] autotuned variant (wg, vec, ref, nt, blocks) = {tuned}: {tms:.4f} ms")
    if a.save_tuning:
        fe.tuning_save(a.save_tuning)
    variant_used = fe.tuning_get(p, wl.elem, rule.n_q)
    if natural:
        variant_used = "natural order: tiles of 64 elements, one wavefront, LDS transposition"

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()

    # copy ceiling on the same byte volume (context for the roofline)
    nbytes = int(bpe * wl.n_elem) // 32 * 16
    src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    for _ in range(3):
        fe.stream_copy(dst, src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(10):
        fe.stream_copy(dst, src)
    ev1.record(stream)
    torch.cuda.synchronize()
    copy_gbps = 2 * nbytes * 10 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del src, dst

    # the kernel's own access pattern with the arithmetic removed: the same
    # rows read (coordinates, coefficient rows as FP64-row equivalents) and
    # written (K and F in the tier's type), one element per lane
    pattern = None
    if not (indexed or natural):
        ncoef = fe.coeff_entries(p, wl.elem, rule.n_q) if wl.coef_mode != "function" else 0
        tsz = 8 if precision == "fp64" else 4
        rows_in = 3 * nv + (ncoef * tsz + 7) // 8
        rows_out = nk + nf
        pin = torch.zeros((rows_in, ld), dtype=torch.float64, device=dev)
        pout = torch.empty((rows_out, ld), dtype=dt, device=dev)
        for _ in range(3):
            fe.stream_pattern(pin, pout, wl.n_elem)
        ev0.record(stream)
        for _ in range(10):
            fe.stream_pattern(pin, pout, wl.n_elem)
        ev1.record(stream)
        torch.cuda.synchronize()
        pt = ev0.elapsed_time(ev1) * 1e-3 / 10
        pbytes = wl.n_elem * (8 * rows_in + tsz * rows_out)
        pattern = {"rows_in_fp64": rows_in, "rows_out": rows_out, "ms": pt * 1e3,
                   "GBps": pbytes / pt / 1e9}
        del pin, pout

    # The timed region: K back-to-back steps between device synchronisations.
    # The host clock gives `value`; one pair of HIP events on the launch
    # stream brackets the same region and gives the average kernel duration
    # of the roofline (both clocks see the same launches, gaps included).
    ev_a, ev_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev_a.record(stream)
    for _ in range(a.steps):
        step()
    ev_b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    avg_kern_s = ev_a.elapsed_time(ev_b) * 1e-3 / a.steps
    ms_per_step = wall / a.steps * 1e3
    value = wl.n_elem / (wall / a.steps)
    # after the timed region, the same steps with an event pair around each
    # one: the distribution of single-launch durations (not part of `value`)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps)]
    for i in range(a.steps):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    torch.cuda.synchronize()
    kern_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]

    # parity on a sample of the measured outputs
    rng = np.random.default_rng(12345)
    sample = np.sort(rng.choice(wl.n_elem, size=min(parity_sample, wl.n_elem), replace=False))
    idx = torch.from_numpy(sample).to(dev)
    Ks = K.index_select(1, idx).cpu().numpy().astype(np.float64)
    Fs = F.index_select(1, idx).cpu().numpy().astype(np.float64)
    coeffs = None
    if wl.coeffs is not None and wl.coef_mode == "function":
        coeffs = wl.coeffs
    elif wl.coeffs is not None:
        coeffs = wl.coeffs[:, sample]
        if precision == "fp32":
            coeffs = coeffs.astype(np.float32).astype(np.float64)
    Ko, Fo = oracle.integrate(wl.elem, wl.kind, wl.mesh.coords[:, sample],
                              oracle.quad_rule(wl.elem, wl.n_q), wl.coef_mode, wl.mask, wl.uniform,
                              coeffs, threads=host_threads())
    N = oracle.n_dof(wl.elem, wl.kind)
    Kg = fe.unpack_full(Ks, N, wl.k_format == "packed")
    ek = np.sqrt(((Kg - Ko) ** 2).sum(axis=(1, 2)) / (Ko ** 2).sum(axis=(1, 2)))
    ef = np.sqrt(((Fs.T - Fo) ** 2).sum(axis=1) / np.maximum((Fo ** 2).sum(axis=1), 1e-300))
    tol = 1e-12 if precision == "fp64" else 2e-5

    achieved = bpe * wl.n_elem / avg_kern_s / 1e9
    shash = source_hash(base, precision)
    traffic = stored_traffic(workload, precision, shash)
    cpu = None
    if with_cpu:
        log("[bench] timing the CPU oracle baseline")
        cpu = cpu_baseline(wl)

    out = {
        "metric": "elements/s + % HBM roofline, tet Poisson FP64; FP32/served speedup, p50/p99 latency",
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32 (FP64 Jacobian)",
        "data": "synthetic",
        "config": {"workload": workload,
                   "description": WORKLOADS[base][1] + (" (indexed geometry: node array + int32 "
                                                        "connectivity)" if indexed else "")
                   + (" (natural element-contiguous order, LDS-tiled)" if natural else ""),
                   "n_elem": wl.n_elem, "precision": precision, "n_q": rule.n_q,
                   "k_format": wl.k_format, "bytes_per_element": bpe,
                   "ld_in": int(dw.coords.stride(0)), "ld_out": ld_out,
                   "variant_wg_vec_ref_nt_blocks": variant_used,
                   "variant_source": ("natural-order form" if natural else
                                      "tuned in this run" if a.tune else
                                      "tuning file " + os.path.basename(a.tuning_file)
                                      if a.tuning_file else
                                      "the library's built-in table" if fe.tuning_builtin()[0]
                                      else "the library's base variant"),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic},
        "cpu_baseline": cpu,
        # the timed region by the host clock: value x bytes / peak
        "wall_frac": value * bpe / 1e9 / HBM_PEAK_GBPS,
        "kernel_ms_avg": avg_kern_s * 1e3,
        "kernel_ms_single_launch": {"avg": float(np.mean(kern_ms)), "min": float(np.min(kern_ms)),
                                    "median": float(np.median(kern_ms))},
        "copy_ceiling_GBps": copy_gbps,
        "frac_of_copy_ceiling": achieved / copy_gbps,
        "access_pattern": (dict(pattern, kernel_vs_pattern=pattern["ms"] / (avg_kern_s * 1e3))
                           if pattern else None),
        "parity": {"sampled_elements": int(len(sample)), "max_rel_err_K": float(ek.max()),
                   "max_rel_err_F": float(ef.max()), "tol": tol,
                   "ok": bool(ek.max() <= tol and ef.max() <= tol)},
        "kernel_source_hash": shash,
    }
    del dw, K, F
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    sys.exit(main())
