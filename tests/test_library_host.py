"""Host-side checks of the C-ABI library that need no GPU: the shared object
loads and exports every function include/pdf.h declares, the FP64 host tables
equal the oracle's, defaults are the paper's constants, and argument errors
are reported without touching the device."""
import ctypes
import json
import os
import re
import subprocess

import numpy as np
import pytest

import seeded_inputs as si
from oracle import operators as ops

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_constants.json")))

pdf = pytest.importorskip("paper_2602_13805_amd")


def lib_or_skip():
    if not os.path.exists(pdf.binding.LIB_PATH):
        pytest.skip("libpdf.so not built")
    return pdf.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pdf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pdf_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = lib_or_skip()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
        assert n in pdf.binding.SIGNATURES, n


def test_default_params_are_the_papers():
    lib_or_skip()
    p = pdf.default_params()
    assert p.beta == GOLD["beta"]["value"]
    assert p.lam_bound == GOLD["lam_bound"]["value"]
    assert p.lam_tv == GOLD["lam_tv"]["value"]
    assert p.lam_bridge == GOLD["lam_bridge"]["value"]
    assert p.tau_b == GOLD["tau_b"]["value"]
    assert p.cco_tau == GOLD["cco_tau"]["value"]
    assert p.cco_eta_max == GOLD["cco_eta_max"]["value"]
    assert p.cco_delta == GOLD["cco_delta"]["value"]
    assert p.lr == GOLD["adam_lr"]["value"]


def test_ctypes_layout_matches_c(tmp_path):
    # sizeof / offsetof of every ABI struct, as the C compiler lays them out
    B = pdf.binding
    prog = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pdf.h"', 'int main(void) {']
    for cname, py in (("pdf_params", B.Params), ("pdf_grid", B.Grid), ("pdf_array", B.Array),
                      ("pdf_report", B.Report), ("pdf_freq", B.Freq)):
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    prog.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = []
    for py in (B.Params, B.Grid, B.Array, B.Report, B.Freq):
        want.append(ctypes.sizeof(py))
        want += [getattr(py, f).offset for f, _ in py._fields_]
    assert got == want


@pytest.mark.parametrize("M", [8, 32, 64])
def test_host_tables_match_oracle(M):
    lib_or_skip()
    wl = si.WORKLOADS["cfg2"]
    tx = si.antenna_positions(5, wl.radius, angle_offsets=np.linspace(0, 0.01, 5))
    rx = si.antenna_positions(7, wl.radius)
    ghat, gs, einc = pdf.tables_host(M, wl.side, wl.freq_hz, tx, rx)
    k0 = ops.wavenumber(wl.freq_hz)
    h = wl.side / M
    assert np.max(np.abs(ghat - ops.gd_spectrum(M, h, k0))) < 1e-12 * np.max(np.abs(ghat))
    assert np.max(np.abs(gs - ops.gs_matrix(rx, M, wl.side, k0))) < 1e-13 * np.max(np.abs(gs))
    assert np.max(np.abs(einc - ops.einc_matrix(tx, M, wl.side, k0))) < 1e-13 * np.max(np.abs(einc))


def test_host_tables_paper_geometry():
    # 20 lambda antenna circle: large Hankel arguments
    lib_or_skip()
    wl = si.WORKLOADS["paper"]
    tx = si.antenna_positions(wl.n_tx, wl.radius)
    rx = si.antenna_positions(wl.n_rx, wl.radius)
    _, gs, einc = pdf.tables_host(16, wl.side, wl.freq_hz, tx, rx)
    k0 = ops.wavenumber(wl.freq_hz)
    assert np.max(np.abs(gs - ops.gs_matrix(rx, 16, wl.side, k0))) < 1e-12 * np.max(np.abs(gs))
    assert np.max(np.abs(einc - ops.einc_matrix(tx, 16, wl.side, k0))) < 1e-12 * np.max(np.abs(einc))


def test_argument_errors_without_device():
    lib = lib_or_skip()
    B = pdf.binding
    g = B.Grid(32, 1.5, 0.0, 0.0)
    xy = np.zeros((4, 2))
    arr = B.Array(4, xy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    h = ctypes.c_void_p()
    p = pdf.default_params()
    # null stream, K > M, bad version, unsupported M: all rejected on the host
    assert lib.pdf_setup(ctypes.byref(g), 4e8, ctypes.byref(arr), ctypes.byref(arr), 9, 1, ctypes.byref(p),
                         None, ctypes.byref(h)) == B.PDF_EINVAL
    assert lib.pdf_setup(ctypes.byref(g), 4e8, ctypes.byref(arr), ctypes.byref(arr), 33, 1, ctypes.byref(p),
                         ctypes.c_void_p(1), ctypes.byref(h)) == B.PDF_EINVAL
    assert b"K" in lib.pdf_last_error(None)
    p.version = 99
    assert lib.pdf_setup(ctypes.byref(g), 4e8, ctypes.byref(arr), ctypes.byref(arr), 9, 1, ctypes.byref(p),
                         ctypes.c_void_p(1), ctypes.byref(h)) == B.PDF_EINVAL
    p.version = 1  # a version-1 struct (without cco_in_loss) is still accepted
    for m_bad, prec in ((40, B.FP32), (100, B.FP64), (512, B.FP32)):  # grids without a plan
        p.precision = prec
        gb = B.Grid(m_bad, 1.5, 0.0, 0.0)
        assert lib.pdf_setup(ctypes.byref(gb), 4e8, ctypes.byref(arr), ctypes.byref(arr), 9, 1, ctypes.byref(p),
                             ctypes.c_void_p(1), ctypes.byref(h)) == B.PDF_EUNSUPPORTED, m_bad
    p.precision = B.FP32
    # the loss on the CCO image: 0 or 1 only, LDS-resident grids only (a current-version struct:
    # version 1 ends before the field)
    p.version = pdf.default_params().version
    assert p.version == 2
    p.cco_in_loss = 2
    assert lib.pdf_setup(ctypes.byref(g), 4e8, ctypes.byref(arr), ctypes.byref(arr), 9, 1, ctypes.byref(p),
                         ctypes.c_void_p(1), ctypes.byref(h)) == B.PDF_EINVAL
    assert b"cco_in_loss" in lib.pdf_last_error(None)
    p.cco_in_loss = 1
    for m_big, prec in ((128, B.FP32), (96, B.FP64)):
        p.precision = prec
        gb = B.Grid(m_big, 1.5, 0.0, 0.0)
        assert lib.pdf_setup(ctypes.byref(gb), 4e8, ctypes.byref(arr), ctypes.byref(arr), 9, 1, ctypes.byref(p),
                             ctypes.c_void_p(1), ctypes.byref(h)) == B.PDF_EUNSUPPORTED, m_big
    f2 = np.array([4e8, 5e8])
    fr = B.Freq(2, f2.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert lib.pdf_setup_freq(ctypes.byref(g), ctypes.byref(fr), ctypes.byref(arr), ctypes.byref(arr), 9, 1,
                              ctypes.byref(p), ctypes.c_void_p(1), ctypes.byref(h)) == B.PDF_EUNSUPPORTED
    p.cco_in_loss = 0
    p.precision = B.FP32
    bad = np.array([[np.nan, 0.0]] * 4)
    arr2 = B.Array(4, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert lib.pdf_setup(ctypes.byref(g), 4e8, ctypes.byref(arr2), ctypes.byref(arr), 9, 1, ctypes.byref(p),
                         ctypes.c_void_p(1), ctypes.byref(h)) == B.PDF_EINVAL
    assert lib.pdf_loss_grad(None, None, None, None) == B.PDF_EINVAL
    lib.pdf_destroy(None)
