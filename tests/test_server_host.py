"""The serving scheduler (paper_2607_20211_amd/csrc/drsf_server.hip) on the
host, under the address and undefined-behaviour sanitizers: the committed
source is compiled with g++ against host stand-ins for HIP and for the
library's context calls (tests/server_host/: contexts with a simulated
device time per apply, tracked allocations and streams), then drives the
benchmark's served sequence (serial saturation; loads 0.5, 0.8, 0.95 and
1.5 of the plain service rate in overlapped, serial and coalescing mode;
the verification pair) on a seeded synthetic stream: a resident graph plus
tenants arriving staggered under a budget that holds the resident graph
and three tenants, requests of 10^U(2,4) edges with Poisson arrivals.
Every request must complete without failure and the sanitizers must stay
silent.  No GPU is used."""
from __future__ import annotations

import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "server_host")


def _workload(path, seed=5, tenants=9, nreq=3000):
    rng = np.random.default_rng(seed)
    ns = [200_000] + [int(10 ** rng.uniform(4, 5)) for _ in range(tenants - 1)]
    arrive = [0.0] + [float(x) for x in np.sort(rng.uniform(0, 0.6 * nreq, tenants - 1))]
    # requests: Poisson at rate 1, each to a tenant already arrived
    t = np.cumsum(rng.exponential(1.0, nreq))
    lines = [f"{tenants} {nreq}"]
    lines += [f"{n} {8 * n} {a!r}" for n, a in zip(ns, arrive)]
    for k in range(nreq):
        live = [g for g in range(tenants) if arrive[g] <= t[k]]
        g = int(rng.choice(live))
        b = int(round(10 ** rng.uniform(2, 4)))
        lines.append(f"{g} {b} {k % 2} {float(t[k])!r}")
    open(path, "w").write("\n".join(lines) + "\n")


def test_scheduler_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    # the committed scheduler source with the stand-ins beside it
    (tmp_path / "hip").mkdir()
    (tmp_path / "include").mkdir()
    (tmp_path / "a" / "b").mkdir(parents=True)
    shutil.copy(os.path.join(HERE, "hip_runtime_stub.h"), tmp_path / "hip" / "hip_runtime.h")
    shutil.copy(os.path.join(ROOT, "include", "drsf.h"), tmp_path / "include" / "drsf.h")
    shutil.copy(os.path.join(ROOT, "paper_2607_20211_amd", "csrc", "drsf_server.hip"),
                tmp_path / "a" / "b" / "drsf_server.cpp")
    shutil.copy(os.path.join(HERE, "drsf_kernels_stub.h"), tmp_path / "a" / "b" / "drsf_kernels.h")
    exe = tmp_path / "server_host"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", f"-I{tmp_path}", f"-I{tmp_path / 'include'}",
           os.path.join(HERE, "driver.cpp"), os.path.join(HERE, "stubs.cpp"),
           str(tmp_path / "a" / "b" / "drsf_server.cpp"), "-lpthread", "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    wl = tmp_path / "wl.txt"
    _workload(wl)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe), str(wl)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    runs = [ln for ln in r.stdout.splitlines() if ln.startswith("serial")]
    assert len(runs) == 1 + 4 * 3 + 2, r.stdout
    assert all("failed 0" in ln for ln in runs), r.stdout
