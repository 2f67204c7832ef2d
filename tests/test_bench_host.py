"""Host logic of the benchmark (no GPU): the rocprofv3 summaries its roofline figures come from
(copy-kernel calibration of the HBM counters, the source hash that invalidates them, the matrix-core
busy fraction), the algorithmic cost models, and the refusal of more than one GPU."""
import csv
import dataclasses
import math
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import seeded_inputs as si  # noqa: E402
from oracle import fcnn as ofcnn  # noqa: E402


def _write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


ADJ = "void pdfk::k_adj_conv<float, 64, false>(pdfk::AdjArgs<float>)"
COPY = "void at::native::elementwise_kernel<AUnaryFunctor<float, float, float, MulFunctor>>(...)"


def test_traffic_summary_calibrates_with_the_copy_kernel(tmp_path, monkeypatch):
    # a 256 MiB copy that the counters see as 128 MiB fetched and 256 MiB written: fetch scale 2, write 1
    mib = 256
    _write_counters(str(tmp_path / "FETCH_SIZE"), [(COPY, "FETCH_SIZE", mib * 1024 / 2),
                                                   (ADJ, "FETCH_SIZE", 1000.0), (ADJ, "FETCH_SIZE", 1200.0)])
    _write_counters(str(tmp_path / "WRITE_SIZE"), [(COPY, "WRITE_SIZE", mib * 1024),
                                                   (ADJ, "WRITE_SIZE", 300.0), (ADJ, "WRITE_SIZE", 300.0)])
    text = bench.summarize_rocprof([str(tmp_path / "FETCH_SIZE"), str(tmp_path / "WRITE_SIZE")], "pmc", mib)
    lines = dict(l.split(": ", 1) for l in text.splitlines() if ": " in l and not l.startswith("kernel"))
    assert float(lines["fetch_scale"]) == pytest.approx(2.0) and float(lines["write_scale"]) == pytest.approx(1.0)
    row = [l for l in text.splitlines() if l.startswith("kernel adj_conv")][0]
    got = dict(kv.split("=") for kv in row.split()[3:])
    assert float(got["bytes"]) == pytest.approx((1100.0 * 2 + 300.0) * 1024)
    assert got["dispatches"] == "2"
    # the summary round-trips through measured_traffic while the sources hash to it
    f = tmp_path / "traffic.txt"
    f.write_text(text + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    b, src = bench.measured_traffic("adj_conv", "k_adj_conv<float,64,false>")
    assert b == pytest.approx((1100.0 * 2 + 300.0) * 1024) and "FETCH_SIZE" in src
    assert bench.measured_traffic("adj_conv", "k_adj_conv<float,64,true>")[0] is None
    f.write_text(text.replace(bench.kernel_source_hash(), "0" * 64))
    b, src = bench.measured_traffic("adj_conv", "k_adj_conv<float,64,false>")
    assert b is None and "changed" in src


def test_traffic_summary_needs_the_calibration_kernel(tmp_path):
    _write_counters(str(tmp_path / "F"), [(ADJ, "FETCH_SIZE", 1.0), (ADJ, "WRITE_SIZE", 1.0)])
    with pytest.raises(SystemExit):
        bench.summarize_rocprof([str(tmp_path / "F")], "pmc", 256)


def test_mfma_summary_busy_fraction(tmp_path):
    name = "void pdfk::k_adj_gemm_mfma<2, 4>(cx<float> const*, ...)"
    _write_counters(str(tmp_path), [(name, "SQ_VALU_MFMA_BUSY_CYCLES", 64.0 * 1000), (name, "SQ_INSTS_MFMA", 1000.0)])
    with open(tmp_path / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for d in (90_000, 100_000, 500_000):   # ns; the median (100 us) is used
            w.writerow({"Kernel_Name": name, "Start_Timestamp": 0, "End_Timestamp": d})
    text = bench.summarize_rocprof([str(tmp_path)], "mfma", 256)
    row = [l for l in text.splitlines() if l.startswith("kernel adj_gemm")][0]
    got = dict(kv.split("=") for kv in row.split()[3:])
    assert float(got["median_us"]) == pytest.approx(100.0)
    assert float(got["mfma_busy_frac"]) == pytest.approx(64e3 / (100e-6 * 2.4e9 * 1024), abs=1e-3)


def test_kernel_variants_of_the_tile_choices():
    wl = si.WORKLOADS["cfg2"]
    v = bench.tuned_variants(wl, (4, 8, 0, 1))
    assert v["pixel_reduce"] == "k_pixel_reduce_mfma<2,1,8>" and v["adj_gemm"] == "k_adj_gemm_mfma<2,4>"
    # K = 15 <= 32: the convolutions run on the compact tile under every plan choice
    assert v["fwd_conv"] == "k_fwd_conv_c<float,64,true>" and v["adj_conv"] == "k_adj_conv_c<float,64,true>"
    assert bench.tuned_variants(dataclasses.replace(wl, K=21), (4, 8, 0, 1))["adj_conv"] == "k_adj_conv_c<float,64,false>"
    wide = dataclasses.replace(wl, K=33)
    v = bench.tuned_variants(wide, (4, 8, 0, 1))
    assert v["fwd_conv"] == "k_fwd_conv<float,64,true,false>" and v["adj_conv"] == "k_adj_conv<float,64,true>"
    assert bench.kernel_variant(ADJ) == "k_adj_conv<float,64,false>"
    assert bench._short_kernel("void pdfk::k_adj_conv_c<float, 64, true>(pdfk::AdjArgs<float>)") == "adj_conv"
    assert bench._short_kernel("void pdfk::k_fwd_conv_c<float, 64, true>(pdfk::FwdArgs<float>)") == "fwd_conv"


def test_cost_models():
    wl = si.WORKLOADS["cfg2"]
    B = 256
    by, fl = bench.workload_cost(wl, B, 16)
    # the adjoint convolution: 8192 (instance, incidence) units of 24 N + 48 K^2 + 20 N / N_i bytes
    # plus the spectrum once (the per-unit figure quoted for the roofline)
    N = wl.M ** 2
    unit = 24 * N + 48 * wl.K ** 2 + 20 * N / wl.n_tx
    assert by["adj_conv"] == pytest.approx(B * wl.n_tx * unit + (2 * wl.M) ** 2 * 8)
    assert fl["adj_gemm"] == B * wl.n_tx * N * 8 * wl.n_rx
    assert all(v > 0 for v in by.values()) and all(v > 0 for v in fl.values())
    # the coefficient network: its parameter count is the oracle's, and Adam moves at least 24 bytes
    # (theta, m, v read and written) per parameter
    cost, P = bench.fcnn_cost(B, 32, 15, 256)
    assert P == ofcnn.n_params(15, 256)
    assert cost["adam"][0] >= 24 * P * B
    assert cost["fwd"][1] == 2 * B * 32 * (450 * 256 + 256 * 256 + 256 * 450)
    assert math.isclose(cost["bwd"][1], 2 * B * 32 * (256 * 256 + 256 * 450))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_seeded_weight_and_position_draws():
    a = si.fcnn_theta(5, 2, 3, 4, out_scale=0.0)
    b = si.fcnn_theta(5, 2, 3, 4, out_scale=0.0)
    assert np.array_equal(a, b) and a.shape == (2, ofcnn.n_params(3, 4))
    D = 18
    assert np.all(a[:, -(4 + 1) * D:] == 0.0)                    # output block zero
    assert np.all(np.abs(a[:, :(D + 1) * 4]) <= 1 / np.sqrt(D))  # U[-1/sqrt(in), 1/sqrt(in)]
    t1, r1 = si.draw_position_errors(7, 32, 32, 1e-3)
    t2, _ = si.draw_position_errors(7, 32, 32, 2e-3)
    assert t1.shape == (32, 2) and np.allclose(t2, 2 * t1)       # one draw, scaled by sigma
    assert 0.5e-3 < np.std(np.concatenate([t1, r1])) < 1.5e-3


def test_fixed_target_counts_count_only_instances_that_start_above_the_target():
    import numpy as np
    import bench
    err0 = np.array([0.50, 0.35, 0.25, 0.60, 0.45])
    # first checked step at or below 0.40 / 0.30 (0 = already at the start, -1 = never)
    first = {0.40: np.array([30, 0, 0, -1, 10]), 0.30: np.array([50, 20, 0, -1, -1])}
    clock = {0: 0.1, 10: 1.0, 20: 2.0, 30: 3.0, 40: 4.0, 50: 5.0}
    out = bench.fixed_target_counts(first, lambda t: clock[t], err0)
    a, b = out["0.40"], out["0.30"]
    # 0.40: instances 0, 3, 4 start above it; 0 and 4 reach it, the last at step 30
    assert (a["n_counted"], a["n_reached"], a["mean_iters"], a["seconds"]) == (3, 2, 20.0, 3.0)
    assert a["per_s"] == 2 / 3.0
    # 0.30: instances 0, 1, 3, 4; 0 at 50 and 1 at 20 (instance 2 starts below: never counted)
    assert (b["n_counted"], b["n_reached"], b["mean_iters"], b["seconds"]) == (4, 2, 35.0, 5.0)
    assert abs(b["frac_reached"] - 0.5) < 1e-15


def test_floor_bytes_of_the_benchmark_instance():
    import bench
    # 8 B x [32*4096 + 2*32*4096 + 2*128^2 + 32*32 + 6*32*225]
    assert bench.floor_bytes(64, 32, 32, 15) == 8 * (32 * 4096 + 64 * 4096 + 2 * 16384 + 1024 + 6 * 32 * 225)


def test_valu_summary_issue_fraction(tmp_path):
    name = "void pdfk::k_adj_conv_c<float, 64, true>(pdfk::AdjArgs<float>)"
    _write_counters(str(tmp_path), [(name, "SQ_INSTS_VALU", 3.0e6), (name, "SQ_ACTIVE_INST_VALU", 1.5e6),
                                    (name, "SQ_INSTS_VALU_FMA_F32", 1.0e6), (name, "SQ_INSTS_VALU_ADD_F32", 0.5e6),
                                    (name, "SQ_INSTS_VALU_MUL_F32", 0.25e6), (name, "SQ_INSTS_LDS", 7.0)])
    with open(tmp_path / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        w.writerow({"Kernel_Name": name, "Start_Timestamp": 0, "End_Timestamp": 100_000})
    text = bench.summarize_rocprof([str(tmp_path)], "valu", 256)
    row = [l for l in text.splitlines() if l.startswith("kernel adj_conv")][0]
    got = dict(kv.split("=") for kv in row.split()[3:])
    cycles = 100e-6 * 2.4e9 * 256
    assert float(got["valu_issue_frac"]) == pytest.approx(3.0e6 / cycles, abs=1e-3)
    assert float(got["valu_busy_frac"]) == pytest.approx(1.5e6 / cycles, abs=1e-3)
    flops = 64 * (2 * 1.0e6 + 0.5e6 + 0.25e6)
    assert float(got["fp32_flops"]) == pytest.approx(flops, rel=1e-3)
    assert float(got["flops_per_valu_inst"]) == pytest.approx(flops / 3.0e6, abs=0.05)
    assert float(got["fp32_frac"]) == pytest.approx(flops / 100e-6 / 157.3e12, abs=1e-3)
