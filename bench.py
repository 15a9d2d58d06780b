#!/usr/bin/env python3
"""Benchmark: element integration throughput on one MI355X.

Default workload (the headline one): scalar Poisson (c^{i;j} = identity,
d^0 = 1) on the jittered unit cube with N = 119 cells per side split into
6 Kuhn tetrahedra (10,111,074 elements, seed 1), 1-point rule, packed 4x4 K
and 4-vector F, FP64. One "step" is one fe_integrate call over the whole
mesh with inputs already resident in HBM.

Prints one JSON line (rank 0). Timing: W untimed warm-up steps (the first
runs the exhaustive variant search of fe_autotune unless --no-tune), then K
timed steps between device synchronisations; the kernel's own duration is
taken with HIP events recorded on the launch stream around every step.

Extra workloads (--workload): tet_cdr (N=119, 4-point rule, per-element
coefficients, full K), prism_cdr_qp (141x141x100 prisms with per-point
coefficients), tet_elasticity (N=94, packed 12x12), prism_elasticity;
--precision fp32 selects the FP32 bulk tier.
"""
from __future__ import annotations

import argparse
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
                    "Poisson on jittered unit cube N=119 x 6 Kuhn tets (10,111,074), tet 1-point rule, packed K"),
    "tet_poisson_qp": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).tet_poisson_qp_rhs(119, 1),
                       "Poisson with d^0 per point of the tet 4-point rule, full K (36 words/element), N=119"),
    "tet_cdr": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).tet_cdr(119, 2),
                "convection-diffusion-reaction, 20 coefficients per element, tet 4-point rule, full K, N=119"),
    "prism_cdr_qp": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).prism_cdr_qp(141, 100, 3),
                     "prisms 141x141x100 (3,976,200, 1% slivers), 20 smooth coefficients per point, 6-point rule, full K"),
    "tet_elasticity": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).tet_elasticity(94, 4),
                       "isotropic elasticity on tets N=94 (4,983,504), per-element E, nu, f, 1-point rule, packed 12x12"),
    "prism_elasticity": (lambda: __import__("paper_1504_01023_amd.inputs", fromlist=["x"]).prism_elasticity(100, 100, 4),
                         "isotropic elasticity on prisms 100x100x100 (2,000,000), per-element E, nu, f, 6-point rule, packed 18x18"),
}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def source_hash() -> str:
    """Hash of the kernel sources; a stored counter reading is only reused
    while this matches."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1504_01023_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".h", ".hip", ".cpp")):
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


def cpu_baseline(wl, min_s: float = 10.0, max_s: float = 30.0):
    """The oracle as it stands, timed on the host cores on passes over the
    same workload (whole passes until about min_s seconds have elapsed)."""
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
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
    return {"value": done / el, "unit": "elements/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} elements ({passes} pass(es) over the {wl.n_elem}-element workload, "
                      f"chunks of {chunk}), {el:.1f} s wall"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="tet_poisson", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--parity-sample", type=int, default=20000)
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

    t0 = time.time()
    wl = WORKLOADS[a.workload][0]()
    log(f"[bench] generated {a.workload}: {wl.n_elem} elements in {time.time() - t0:.1f}s")
    dw = fe.to_device(wl, a.precision, device=dev)
    p, rule = dw.problem, dw.rule
    nk, nf = fe.k_entries(p, wl.elem), fe.f_entries(p, wl.elem)
    dt = torch.float64 if a.precision == "fp64" else torch.float32
    K = torch.empty((nk, wl.n_elem), dtype=dt, device=dev)
    F = torch.empty((nf, wl.n_elem), dtype=dt, device=dev)
    bpe = fe.bytes_per_element(p, wl.elem, rule.n_q)
    stream = torch.cuda.current_stream()

    tuned = None
    if not a.no_tune:
        tuned, tms = fe.autotune(p, wl.elem, dw.coords, dw.coeffs, rule, K, F, reps=5)
        log(f"[bench] autotuned variant (wg, vec, ref, nt, blocks) = {tuned}: {tms:.4f} ms")
    variant_used = fe.tuning_get(p, wl.elem, rule.n_q)

    for _ in range(a.warmup):
        fe.integrate(p, wl.elem, dw.coords, dw.coeffs, rule, out_K=K, out_F=F)
    torch.cuda.synchronize()

    # copy ceiling on the same byte volume (context for the roofline)
    nbytes = (bpe * wl.n_elem) // 32 * 16
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

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(a.steps):
        starts[i].record(stream)
        fe.integrate(p, wl.elem, dw.coords, dw.coeffs, rule, out_K=K, out_F=F)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    kern_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    avg_kern_s = float(np.mean(kern_ms)) * 1e-3
    ms_per_step = wall / a.steps * 1e3
    value = wl.n_elem / (wall / a.steps)

    # parity on a sample of the measured outputs
    rng = np.random.default_rng(12345)
    sample = np.sort(rng.choice(wl.n_elem, size=min(a.parity_sample, wl.n_elem), replace=False))
    idx = torch.from_numpy(sample).to(dev)
    Ks = K.index_select(1, idx).cpu().numpy().astype(np.float64)
    Fs = F.index_select(1, idx).cpu().numpy().astype(np.float64)
    coeffs = None
    if wl.coeffs is not None:
        coeffs = wl.coeffs[:, sample]
        if a.precision == "fp32":
            coeffs = coeffs.astype(np.float32).astype(np.float64)
    Ko, Fo = oracle.integrate(wl.elem, wl.kind, wl.mesh.coords[:, sample],
                              oracle.quad_rule(wl.elem, wl.n_q), wl.coef_mode, wl.mask, wl.uniform,
                              coeffs, threads=max(1, min(16, os.cpu_count() or 1)))
    N = oracle.n_dof(wl.elem, wl.kind)
    Kg = fe.unpack_full(Ks, N, wl.k_format == "packed")
    ek = np.sqrt(((Kg - Ko) ** 2).sum(axis=(1, 2)) / (Ko ** 2).sum(axis=(1, 2)))
    ef = np.sqrt(((Fs.T - Fo) ** 2).sum(axis=1) / np.maximum((Fo ** 2).sum(axis=1), 1e-300))
    tol = 1e-12 if a.precision == "fp64" else 2e-5

    achieved = bpe * wl.n_elem / avg_kern_s / 1e9
    shash = source_hash()
    traffic = stored_traffic(a.workload, a.precision, shash)
    cpu = None
    if not a.no_cpu:
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
        "dtype": "f64" if a.precision == "fp64" else "f32 (FP64 Jacobian)",
        "data": "synthetic",
        "config": {"workload": a.workload, "description": WORKLOADS[a.workload][1],
                   "n_elem": wl.n_elem, "precision": a.precision, "n_q": rule.n_q,
                   "k_format": wl.k_format, "bytes_per_element": bpe,
                   "variant_wg_vec_ref_nt_blocks": variant_used, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic},
        "cpu_baseline": cpu,
        "kernel_ms_avg": avg_kern_s * 1e3,
        "kernel_ms_min": float(np.min(kern_ms)),
        "copy_ceiling_GBps": copy_gbps,
        "frac_of_copy_ceiling": achieved / copy_gbps,
        "parity": {"sampled_elements": int(len(sample)), "max_rel_err_K": float(ek.max()),
                   "max_rel_err_F": float(ef.max()), "tol": tol,
                   "ok": bool(ek.max() <= tol and ef.max() <= tol)},
        "kernel_source_hash": shash,
    }
    print(json.dumps(out), flush=True)
    return 0 if out["parity"]["ok"] else 3


if __name__ == "__main__":
    sys.exit(main())
