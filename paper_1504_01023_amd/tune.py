"""Regenerate the tuning table: exhaustive variant search (fe_autotune, the
parameter-based tuning of Sec. 4.3) on the standard synthetic workloads, one
entry per kernel family, written in the format libfe compiles in.

Usage: python -m paper_1504_01023_amd.tune [--out FILE] [--only NAME ...]

Each workload is generated at its benchmark size, uploaded in the library's
default layout (rows of fe_ld_for(n) elements) and searched on the current
GPU. The table begins with the device's architecture and ROCm version, the
key under which libfe applies a compiled-in table.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

from paper_1504_01023_amd import fe, inputs

# (name, builder, precisions): the families of the compiled-in table
WORKLOADS = [
    ("tet_poisson", lambda: inputs.tet_poisson(119, 1), ("fp64", "fp32")),
    ("tet_poisson_qp", lambda: inputs.tet_poisson_qp_rhs(119, 1), ("fp64",)),
    ("tet_cdr", lambda: inputs.tet_cdr(119, 2), ("fp64", "fp32")),
    ("tet_cdr_fn", lambda: inputs.tet_cdr_fn(119, 2), ("fp64",)),
    ("tet_elasticity", lambda: inputs.tet_elasticity(94, 4), ("fp64", "fp32")),
    ("tet_vector", lambda: inputs.tet_vector(94, 6), ("fp64", "fp32")),
    ("prism_poisson_qp", lambda: inputs.prism_poisson_qp_rhs(141, 100, 3), ("fp64", "fp32")),
    ("prism_cdr", lambda: inputs.prism_cdr_element(141, 100, 3), ("fp64", "fp32")),
    ("prism_cdr_qp", lambda: inputs.prism_cdr_qp(141, 100, 3), ("fp64", "fp32")),
    ("prism_cdr_fn", lambda: inputs.prism_cdr_fn(141, 100, 3), ("fp64",)),
    ("prism_elasticity", lambda: inputs.prism_elasticity(100, 100, 4), ("fp64", "fp32")),
    ("prism_vector", lambda: inputs.prism_vector(100, 100, 7), ("fp64", "fp32")),
]


def main() -> int:
    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="tuning_table.txt")
    ap.add_argument("--only", nargs="*", default=None, help="workload names to tune")
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    if not torch.cuda.is_available():
        print("tune.py needs a GPU", file=sys.stderr)
        return 1
    fe.tuning_clear()
    dev = torch.device("cuda:0")
    for name, build, precs in WORKLOADS:
        if a.only and name not in a.only:
            continue
        t0 = time.time()
        wl = build()
        for prec in precs:
            dw = fe.to_device(wl, prec, device=dev)
            p = dw.problem
            n = wl.n_elem
            ld = fe.ld_for(n)
            dt = torch.float64 if prec == "fp64" else torch.float32
            K = torch.empty((fe.k_entries(p, wl.elem), ld), dtype=dt, device=dev)[:, :n]
            F = torch.empty((fe.f_entries(p, wl.elem), ld), dtype=dt, device=dev)[:, :n]
            best, ms = fe.autotune(p, wl.elem, dw.coords, dw.coeffs, dw.rule, K, F, reps=a.reps)
            print(f"{name} {prec}: {best} {ms:.4f} ms ({n / (ms * 1e-3):.3e} elements/s)",
                  flush=True)
            del dw, K, F
            torch.cuda.empty_cache()
        print(f"  ({time.time() - t0:.1f} s)", flush=True)
    tmp = a.out + ".tmp"
    fe.tuning_save(tmp)
    import ctypes
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    v = ctypes.c_int(0)
    ctypes.CDLL("libamdhip64.so").hipRuntimeGetVersion(ctypes.byref(v))
    rocm = f"{v.value // 10_000_000}.{v.value // 100_000 % 100}"  # major * 1e7 + minor * 1e5 + patch
    with open(tmp) as f:
        lines = f.read().splitlines()
    with open(a.out, "w") as f:
        f.write(lines[0] + "\n")
        f.write(f"# measured on a {arch} device (HIP runtime {rocm}) by paper_1504_01023_amd.tune\n")
        f.write(f"# arch {arch}\n# rocm {rocm}\n")
        for line in lines[1:]:
            f.write(line + "\n")
    os.remove(tmp)
    print(f"wrote {a.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
