"""The oracle (oracle/lbo.c) and the host decomposition lists
(paper_1007_4895_amd/csrc/lb_lists.hpp, through tests/lists_driver.cpp)
built with AddressSanitizer and UndefinedBehaviorSanitizer on the CPU and run
over every lattice configuration the tests use; any invalid access, leak or
undefined operation fails the test."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _need(tool):
    path = shutil.which(tool)
    if path is None:
        pytest.skip(f"{tool} not available")
    return path


def test_oracle_under_sanitizers(tmp_path):
    gcc = _need("gcc")
    exe = str(tmp_path / "oracle_san")
    subprocess.run([gcc, *SAN, "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-std=c11", "-o", exe,
                    os.path.join(HERE, "oracle_sanitizer_driver.c"), os.path.join(ROOT, "oracle", "lbo.c"), "-lm"],
                   check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "failures 0" in r.stdout


def test_host_lists_under_sanitizers(tmp_path):
    gxx = _need("g++")
    exe = str(tmp_path / "lists_san")
    subprocess.run([gxx, *SAN, "-std=c++17", "-o", exe, os.path.join(HERE, "lists_driver.cpp")], check=True)
    g = np.random.default_rng(5)
    lines = []
    for k in range(40):
        nx = int(g.integers(2, 300))
        ny = int(g.integers(4, 80))
        xbc, ybc, iface = int(g.integers(0, 2)), int(g.integers(0, 2)), int(g.integers(0, 2))
        tw = nx if iface or k % 3 == 0 else 64
        nt = (nx + tw - 1) // tw
        if iface:
            b = int(g.integers(0, max(1, (ny - 3) // 2)))
            lo = hi = [b] * nt
        else:
            lo = list(g.integers(0, ny // 2 + 1, nt))
            hi = list(g.integers(0, ny // 2 + 1, nt))
        lines.append(" ".join(str(v) for v in [nx, ny, xbc, ybc, iface, tw, *lo, *hi]))
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert len(r.stdout.splitlines()) == len(lines)
