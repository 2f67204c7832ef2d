"""The library's host C++ (the FP64 operator tables: Hankel functions, the embedded G_D kernel and
its FFT, the receiver operator and incident fields) built with AddressSanitizer and
UndefinedBehaviorSanitizer and run on several geometries; its tables must equal the oracle's."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import operators as ops

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_13805_amd", "csrc")


@pytest.mark.slow
def test_host_tables_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = tmp_path / "tables_asan"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(os.path.dirname(__file__), "sanitize_tables_main.cpp"),
           os.path.join(CSRC, "tables.cpp"), "-o", str(exe), "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = tmp_path / "tables.bin"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe), str(out)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "SANITIZED_OK" in r.stdout, r.stdout + r.stderr
    raw = out.read_bytes()
    pos = 0
    k0 = ops.wavenumber(4e8)
    for _ in range(4):
        M, ni, ns = np.frombuffer(raw, np.int32, 3, pos)
        pos += 12
        tx = np.frombuffer(raw, np.float64, 2 * ni, pos).reshape(ni, 2)
        pos += 16 * ni
        rx = np.frombuffer(raw, np.float64, 2 * ns, pos).reshape(ns, 2)
        pos += 16 * ns
        P, N = 2 * M, M * M
        ghat = np.frombuffer(raw, np.complex128, P * P, pos).reshape(P, P)
        pos += 16 * P * P
        gs = np.frombuffer(raw, np.complex128, ns * N, pos).reshape(ns, N)
        pos += 16 * ns * N
        einc = np.frombuffer(raw, np.complex128, ni * N, pos).reshape(ni, N)
        pos += 16 * ni * N
        h = 1.5 / M
        ref = ops.gd_spectrum(M, h, k0)
        assert np.max(np.abs(ghat - ref)) < 1e-11 * np.max(np.abs(ref)), M
        ref = ops.gs_matrix(rx, M, 1.5, k0, 0.01, -0.02)
        assert np.max(np.abs(gs - ref)) < 1e-12 * np.max(np.abs(ref)), M
        ref = ops.einc_matrix(tx, M, 1.5, k0, 0.01, -0.02)
        assert np.max(np.abs(einc - ref)) < 1e-12 * np.max(np.abs(ref)), M
    assert pos == len(raw)
