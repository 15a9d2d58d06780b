"""Sanitizer builds of host code (CPU only; nothing runs on a device):
the oracle under address + undefined-behaviour and thread sanitizers,
driven over every element type, problem kind and coefficient mode in one and
several threads; the continuous-batching server (scheduler thread, hand-over
queues, statistics) on its host-only timing backend under thread and
address + undefined-behaviour sanitizers, with concurrent submitters, a
poller that releases, and a statistics reader."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1504_01023_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
SERVER_SRCS = ("fe_server.cpp", "fe_api.cpp", "fe_batch.cpp", "fe_tune.cpp")


def _run(cmd, env=None, timeout=300):
    p = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert p.returncode == 0, f"{' '.join(cmd)}\n{p.stdout[-3000:]}\n{p.stderr[-6000:]}"
    return p.stdout


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_oracle_under_sanitizer(tmp_path, san):
    exe = str(tmp_path / "oracle_driver")
    flags = ["-fsanitize=" + san, "-fno-sanitize-recover=all"] if san != "thread" else ["-fsanitize=thread"]
    _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", *flags, "-o", exe,
          os.path.join(HERE, "csrc", "oracle_driver.c"), os.path.join(ROOT, "oracle", "fe_oracle.c"),
          "-lm", "-lpthread"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    env.pop("LD_PRELOAD", None)
    out = _run([exe], env=env)
    assert "0 failures" in out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("san", [("thread",), ("address", "undefined")])
def test_server_under_sanitizer(tmp_path, san):
    # host-side sanitizers only: each -fsanitize= applies to the host pass
    host = []
    for s in san:
        host += ["-Xarch_host", "-fsanitize=" + s]
    common = ["-O1", "-g", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", *host,
              "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    procs = []
    from paper_1504_01023_amd import build as fe_build
    os.makedirs(fe_build.BUILD, exist_ok=True)
    table = fe_build._tuning_source()  # the built-in tuning table's unit
    for src in SERVER_SRCS + ("server_stress.cpp", table):
        path = (os.path.join(HERE, "csrc", src) if src == "server_stress.cpp" else
                src if os.path.isabs(src) else os.path.join(CSRC, src))
        src = os.path.basename(src)
        obj = str(tmp_path / (src + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, *common, "-fPIC", "-c", path, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        out, err = p.communicate(timeout=600)
        assert p.returncode == 0, err[-4000:]
    exe = str(tmp_path / "server_stress")
    _run([HIPCC, *host, "--offload-arch=gfx950", *objs, "-o", exe, "-L/opt/rocm/lib",
          "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=0")
    env.pop("LD_PRELOAD", None)
    out = _run([exe], env=env, timeout=300)
    assert "dup 0 in use 0" in out
