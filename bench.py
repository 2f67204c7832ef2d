#!/usr/bin/env python3
"""Throughput of the PDF hot path on one MI355X.

Workload (cfg2): 64 x 64 inversion grid over a 2-wavelength domain, 32
transmitters and 32 receivers on a 3-wavelength circle, K = 15 Fourier modes
per axis, FP32.  Each of the `batch` instances has its own random profile
(1-3 discs / ellipses, eps_r in [2, 4]) whose measured fields come from the
library's FP64 method-of-moments solve on a 128 x 128 grid with +-2 degree
antenna-angle jitter, plus 10 % complex AWGN.

One step = one loss + gradient + Adam iteration of every instance in the
batch (all hot-path kernels).  `value` = instance-iterations per second over
the timed steps, inputs resident in HBM.  Also reported: per-kernel times
(HIP events on the library's stream), the roofline of the dominant kernel,
reconstructions per second to a fixed image error, single-instance numbers,
the warm-started reconstructions (network trained here on fresh MoM pairs)
to the same errors, and the FP64 oracle timed on the host (`cpu_baseline`).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PDF loss+grad iters/s and reconstructions/s at 64² to fixed rel. image error"
HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
FP32_PEAK = 157.3e12       # flop/s, MI355X FP32 vector (= FP32 matrix)
CLOCK_HZ = 2.4e9           # MI355X peak engine clock
N_CU = 256                 # compute units (4 SIMDs each)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# kernel names in the library's timing order, and how they appear in profiler output
KERNEL_SYMBOLS = {   # symbol prefixes of the step kernels (every tuning variant, both tiles)
    "fwd_conv": ("k_fwd_conv<float, 64, true,", "k_fwd_conv_c<float, 64,"),
    "pixel_reduce": ("k_pixel_reduce_mfma<",),
    "image_reg": ("k_image_reg<float>",),
    "adj_gemm": ("k_adj_gemm_mfma<",),
    "adj_conv": ("k_adj_conv<float, 64,", "k_adj_conv_c<float, 64,"),
}
COMPACT_MAX_K = 32   # 64 x 64 FP32 with K <= 32: the convolutions run on the compact tile


def kernel_variant(name):
    """The template instance of a kernel symbol without spaces, e.g. k_adj_conv<float,64,false>."""
    m = re.search(r"(k_\w+<[^>]*>)", name)
    return m.group(1).replace(" ", "") if m else name.replace(" ", "")


def tuned_variants(wl, tuned):
    """Template instance of each step kernel that the tile / plan choice `tuned` launches."""
    ct, pb, fpp, app = tuned
    tf = lambda b: "true" if b else "false"
    nrt, nct, nrta = -(-wl.n_rx // 16), -(-wl.n_tx // 32), -(-wl.n_tx // 16)
    compact = wl.M == 64 and wl.K <= COMPACT_MAX_K   # every plan choice runs the compact kernels
    # K <= 16: the forward's beta U and the adjoint's g_J row transform wait in the compact tile's spare columns
    spare = tf(2 * wl.K <= COMPACT_MAX_K)
    return {"fwd_conv": f"k_fwd_conv_c<float,{wl.M},{spare}>" if compact else f"k_fwd_conv<float,{wl.M},true,{tf(fpp)}>",
            "pixel_reduce": f"k_pixel_reduce_mfma<{nrt},{nct},{pb}>",
            "image_reg": "k_image_reg<float>",
            "adj_gemm": f"k_adj_gemm_mfma<{nrta},{ct}>",
            "adj_conv": (f"k_adj_conv_c<float,{wl.M},{spare}>" if compact
                         else f"k_adj_conv<float,{wl.M},{tf(app)}>")}
CALIBRATION_SYMBOL = "AUnaryFunctor<float, float"   # torch.mul(src, 1.0, out=dst)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cfg2_b256.txt")


# the sources the step kernels and their launches are built from
STEP_SOURCES = ("csrc/api.hip", "csrc/conv_kernels.h", "csrc/cplx.h", "csrc/fft_lds.h", "csrc/handle.h",
                "csrc/init_kernels.h", "csrc/pixel_kernels.h", "build.py")   # build.py: the compiler flags


def kernel_source_hash():
    """SHA-256 over the step kernels' sources and compiler flags: traffic counts are valid only for the
    code they were taken on."""
    import hashlib
    d = os.path.join(ROOT, "paper_2602_13805_amd")
    h = hashlib.sha256()
    for name in STEP_SOURCES:
        h.update(name.encode())
        with open(os.path.join(d, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _short_kernel(name):
    for k, syms in KERNEL_SYMBOLS.items():
        if any(sym in name for sym in syms):
            return k
    if CALIBRATION_SYMBOL in name:
        return "calibration_copy"
    return None


def summarize_rocprof(dirs, kind, copy_mib):
    """Text summary of rocprofv3 CSV output (kernel-trace stats, or FETCH_SIZE / WRITE_SIZE passes)."""
    import csv
    import glob
    lines = []
    if kind == "stats":
        rows = []
        for d in dirs:
            for f in glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True):
                with open(f) as fh:
                    rows += list(csv.DictReader(fh))
        rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
        lines.append("| kernel | calls | total ms | average us | min us | max us | % |")
        lines.append("|---|---|---|---|---|---|---|")
        for r in rows[:16]:
            lines.append(f"| {r['Name'][:80]} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                         f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                         f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
        return "\n".join(lines)
    if kind == "mfma":
        return _summarize_mfma(dirs)
    if kind == "valu":
        return _summarize_valu(dirs)
    acc = {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    k = _short_kernel(r["Kernel_Name"])
                    if k is None:
                        continue
                    if k != "calibration_copy":
                        k = (k, kernel_variant(r["Kernel_Name"]))
                    acc.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    avg = {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}
    cal = avg.get("calibration_copy", {})
    if "FETCH_SIZE" not in cal or "WRITE_SIZE" not in cal:
        raise SystemExit("the calibration copy kernel is missing from the counter output")
    cbytes = copy_mib * 2 ** 20
    f_scale = cbytes / (cal["FETCH_SIZE"] * 1024.0)
    w_scale = cbytes / (cal["WRITE_SIZE"] * 1024.0)
    lines.append(f"source_sha256: {kernel_source_hash()}")
    lines.append(f"calibration_bytes: {cbytes}")
    lines.append(f"calibration_fetch_kib: {cal['FETCH_SIZE']:.1f}")
    lines.append(f"calibration_write_kib: {cal['WRITE_SIZE']:.1f}")
    lines.append(f"fetch_scale: {f_scale:.4f}")
    lines.append(f"write_scale: {w_scale:.4f}")
    order = list(KERNEL_SYMBOLS)
    for k in sorted((k for k in avg if k != "calibration_copy"), key=lambda k: (order.index(k[0]), k[1])):
        if "FETCH_SIZE" not in avg[k] or "WRITE_SIZE" not in avg[k]:
            continue
        fb = avg[k]["FETCH_SIZE"] * 1024.0 * f_scale
        wb = avg[k]["WRITE_SIZE"] * 1024.0 * w_scale
        n = len(acc[k]["FETCH_SIZE"])
        lines.append(f"kernel {k[0]} {k[1]} fetch_kib={avg[k]['FETCH_SIZE']:.1f} "
                     f"write_kib={avg[k]['WRITE_SIZE']:.1f} bytes={fb + wb:.0f} dispatches={n}")
    return "\n".join(lines)


def _counters_and_durations(dirs):
    """Per step-kernel variant: the mean of each counter over its dispatches, and the sorted
    durations (s) of the kernel trace taken in the same run."""
    import csv
    import glob
    cnt, dur = {}, {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    k = _short_kernel(r["Kernel_Name"])
                    if k is not None and k != "calibration_copy":
                        key = (k, kernel_variant(r["Kernel_Name"]))
                        cnt.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    k = _short_kernel(r["Kernel_Name"])
                    if k is not None and k != "calibration_copy":
                        key = (k, kernel_variant(r["Kernel_Name"]))
                        dur.setdefault(key, []).append(
                            (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) * 1e-9)
    order = list(KERNEL_SYMBOLS)
    out = []
    for key in sorted(cnt, key=lambda k: (order.index(k[0]), k[1])):
        ts = sorted(dur.get(key, []))
        if ts:
            out.append((key, {n: sum(v) / len(v) for n, v in cnt[key].items()}, ts))
    return out


def _summarize_mfma(dirs):
    """Matrix-core use per step kernel from one counter pass (SQ_INSTS_MFMA, SQ_VALU_MFMA_BUSY_CYCLES)
    taken together with a kernel trace: busy cycles over the kernel's duration times the clock and the
    1024 SIMDs of the chip."""
    lines = [f"source_sha256: {kernel_source_hash()}",
             f"clock_hz: {CLOCK_HZ:.3g}", f"simds: {4 * N_CU}"]
    for key, c, ts in _counters_and_durations(dirs):
        if "SQ_VALU_MFMA_BUSY_CYCLES" not in c:
            continue
        t = ts[len(ts) // 2]
        busy = c["SQ_VALU_MFMA_BUSY_CYCLES"]
        lines.append(f"kernel {key[0]} {key[1]} dispatches={len(ts)} mfma_insts={c.get('SQ_INSTS_MFMA', 0.0):.0f} "
                     f"mfma_busy_cycles={busy:.0f} median_us={t * 1e6:.1f} "
                     f"mfma_busy_frac={busy / (t * CLOCK_HZ * 4 * N_CU):.3f}")
    return "\n".join(lines)


VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_ADD_F32",
                 "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_TRANS_F32", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT")


def _summarize_valu(dirs):
    """Vector-unit use per step kernel from one counter pass (VALU_COUNTERS) taken together with a
    kernel trace.  A wave64 VALU instruction holds one 16-lane SIMD for four cycles, so the chip
    issues at most N_CU of them per cycle: valu_issue_frac = SQ_INSTS_VALU / (median duration x
    clock x N_CU).  valu_busy_frac is rocprof's VALUBusy (SQ_ACTIVE_INST_VALU over CUs x cycles).
    fp32_flops counts 64 lanes per instruction, an FMA as two; fp32_frac is the resulting rate over
    FP32_PEAK (which counts packed two-lane instructions; the library is built without them, so
    its vector code reaches at most half of it)."""
    lines = [f"source_sha256: {kernel_source_hash()}",
             f"clock_hz: {CLOCK_HZ:.3g}", f"compute_units: {N_CU}"]
    for key, c, ts in _counters_and_durations(dirs):
        if "SQ_INSTS_VALU" not in c:
            continue
        t = ts[len(ts) // 2]
        cycles = t * CLOCK_HZ * N_CU
        flops = 64.0 * (2 * c.get("SQ_INSTS_VALU_FMA_F32", 0.0) + c.get("SQ_INSTS_VALU_ADD_F32", 0.0)
                        + c.get("SQ_INSTS_VALU_MUL_F32", 0.0) + c.get("SQ_INSTS_VALU_TRANS_F32", 0.0))
        lines.append(f"kernel {key[0]} {key[1]} dispatches={len(ts)} median_us={t * 1e6:.1f} "
                     f"valu_insts={c['SQ_INSTS_VALU']:.0f} valu_issue_frac={c['SQ_INSTS_VALU'] / cycles:.3f} "
                     f"valu_busy_frac={c.get('SQ_ACTIVE_INST_VALU', 0.0) / cycles:.3f} "
                     f"fp32_flops={flops:.4g} flops_per_valu_inst={flops / max(c['SQ_INSTS_VALU'], 1.0):.1f} "
                     f"fp32_frac={flops / t / FP32_PEAK:.3f} "
                     f"lds_insts={c.get('SQ_INSTS_LDS', 0.0):.0f} "
                     f"lds_bank_conflict_frac={c.get('SQ_LDS_BANK_CONFLICT', 0.0) / cycles:.3f}")
    return "\n".join(lines)


def measured_traffic(kernel, variant):
    """HBM bytes per launch of `kernel` (template instance `variant`) from the committed counter
    summary, if taken on these sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, "no counter summary"
    meta, per = {}, {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            line = line.strip()
            if line.startswith("kernel "):
                parts = line.split()
                per[(parts[1], parts[2])] = dict(kv.split("=") for kv in parts[3:])
            elif ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                meta[k.strip()] = v.strip()
    if meta.get("source_sha256") != kernel_source_hash():
        return None, "kernel sources changed since the counters were taken"
    if (kernel, variant) not in per:
        return None, f"{variant} not in the counter summary"
    return (float(per[(kernel, variant)]["bytes"]),
            f"rocprofv3 FETCH_SIZE + WRITE_SIZE of {variant}, scaled by a copy kernel of known size")


def workload_cost(wl, B, ntiles):
    """Algorithmic HBM bytes and flops per launch of each kernel (FP32, 8-byte complex).

    Bytes count what a kernel must move at least: per-instance arrays once,
    tables shared by the batch once.  Flops count 5 n log2 n per length-n FFT,
    8 per complex multiply-add, 6 per complex multiply."""
    M, K, Ni, Ns = wl.M, wl.K, wl.n_tx, wl.n_rx
    N, P, c = M * M, 2 * M, 8
    lg = lambda n: math.log2(n)
    fft = lambda n: 5 * n * lg(n)
    conv = (M + P + P + M) * fft(P) + 6 * P * P
    synth = (K + M) * fft(M)
    bytes_ = {
        "fwd_conv": B * Ni * K * K * c + Ni * N * c + P * P * c + 2 * B * Ni * N * c,
        "pixel_reduce": 2 * B * Ni * N * c + Ns * N * c + B * N * (8 + 4 + 8) + B * ntiles * (Ni * Ns * c + 8),
        "image_reg": B * N * 16 + B * ntiles * Ni * Ns * c + 2 * B * Ni * Ns * c + B * N * c,
        "adj_gemm": Ns * N * c + B * Ni * Ns * c + B * Ni * N * c,
        "adj_conv": 3 * B * Ni * N * c + B * N * (8 + 4 + 8) + P * P * c + B * Ni * K * K * 48,
    }
    flops = {
        "fwd_conv": B * Ni * (synth + conv + 6 * N),
        "pixel_reduce": B * Ni * N * (8 * Ns + 16),
        "image_reg": B * N * 150,
        "adj_gemm": B * Ni * N * 8 * Ns,
        "adj_conv": B * Ni * (conv + (M + K) * fft(M) + 60 * N),
    }
    return bytes_, flops


def synthesize_batch(pdf, si, wl, B, dev, noise=None):
    """Measured fields of B random instances: FP64 MoM on the fine grid with jittered antennas, plus
    noise of relative level `noise` (default: the workload's)."""
    import numpy as np
    Ni, Ns, M = wl.n_tx, wl.n_rx, wl.M
    from concurrent.futures import ThreadPoolExecutor

    def draw(b):
        shapes = si.draw_profile(wl, b)
        jt, jr = si.draw_jitter(b, Ni, Ns, wl.jitter_deg)
        return (si.antenna_positions(Ni, wl.radius, angle_offsets=jt),
                si.antenna_positions(Ns, wl.radius, angle_offsets=jr),
                si.rasterize(shapes, wl.M_fine, wl.side), si.rasterize(shapes, M, wl.side))

    with ThreadPoolExecutor(max_workers=8) as pool:
        drawn = list(pool.map(draw, range(B)))
    txs = [d[0] for d in drawn]
    rxs = [d[1] for d in drawn]
    eps_f = np.stack([d[2] for d in drawn])
    eps = np.stack([d[3] for d in drawn])
    e = pdf.synthesize_batch(wl.M_fine, wl.side, wl.freq_hz, txs, rxs, eps_f, tol=1e-10, device=dev)
    esca = np.zeros((B, Ni, Ns), np.complex128)
    for b in range(B):
        n1, n2 = si.draw_noise(b, e[b].shape)
        esca[b] = si.add_noise(e[b], wl.noise if noise is None else noise, n1, n2)
    return esca, eps


def cpu_baseline(si, wl, esca0, seconds):
    """The FP64 oracle's loss + gradient + Adam on one cfg2 instance, timed twice: with every host
    core this process may use (BLAS threads and scipy.fft workers = that count), and with one
    thread."""
    import numpy as np
    import scipy.fft
    from threadpoolctl import threadpool_limits
    from oracle import adam, init, loss
    tx = si.antenna_positions(wl.n_tx, wl.radius)
    rx = si.antenna_positions(wl.n_rx, wl.radius)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()

    def run(threads):
        with threadpool_limits(limits=threads), scipy.fft.set_workers(threads):
            prob = loss.build_problem(wl.M, wl.K, wl.side, [wl.freq_hz], tx, rx, esca0)
            a, _ = init.alpha0(prob)
            m = np.zeros(a.shape + (2,))
            v = np.zeros(a.shape + (2,))
            n = 0
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < seconds:
                out = loss.evaluate(a, prob)
                a, m, v = adam.adam_step(a, out["g_alpha"], m, v, n + 1)
                n += 1
            return n, time.perf_counter() - t0

    n_all, dt_all = run(cores)
    n_one, dt_one = run(1)
    return dict(value=n_all / dt_all, unit="instance-iters/s", cores=cores, kind="oracle",
                sample=f"{n_all} loss+grad+Adam iterations of one cfg2 instance (64x64, 32/32, K=15, FP64 "
                       f"NumPy/SciPy, {cores} BLAS threads and FFT workers) in {dt_all:.1f} s",
                single_thread=dict(value=n_one / dt_one, cores=1,
                                   sample=f"{n_one} iterations with one thread in {dt_one:.1f} s"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--recon-iters", type=int, default=1000)
    ap.add_argument("--no-recon", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB before the steps, as a "
                         "reference of known traffic for hardware byte counters")
    ap.add_argument("--warm-pairs", type=int, default=20000,
                    help="training pairs of the warm-start network (0: skip the warm-start leg)")
    ap.add_argument("--warm-epochs", type=int, default=40)
    ap.add_argument("--mlp-forward-only", type=int, default=0, metavar="CALLS",
                    help="only time this many forwards of 256 rows through the warm-start network (seeded "
                         "weights, seeded inputs, no data synthesis) and print the per-call time")
    ap.add_argument("--fcnn-iters", type=int, default=300,
                    help="Adam steps of the coefficient-network leg (0: skip it)")
    ap.add_argument("--fcnn-hidden", type=int, default=256, help="hidden width of the coefficient network")
    ap.add_argument("--no-csi", dest="csi", action="store_false", help="skip the full-CSI-start leg")
    ap.add_argument("--positions", type=int, default=100,
                    help="realisations per sigma of the antenna-position leg (0: skip it)")
    ap.add_argument("--sweep-batch", type=int, default=32,
                    help="instances per (beta, M_F, SNR) combination of the parameter-sweep leg (0: skip it)")
    ap.add_argument("--uneven", type=int, default=512,
                    help="instances of the uneven-shape batch leg (0: skip it)")
    ap.add_argument("--large", type=int, default=500,
                    help="Adam steps of the large multi-frequency leg (256x256, 4 frequencies, K=41; 0: skip it)")
    ap.add_argument("--large-fields", metavar="NPZ",
                    help="the large leg's measured fields: loaded from this file if it exists, else synthesised "
                         "and written to it (with --save-fields: written, then exit)")
    ap.add_argument("--summarize-rocprof", nargs="+", metavar="DIR",
                    help="print a summary of rocprofv3 CSV output in these directories and exit")
    ap.add_argument("--summary-kind", choices=["stats", "pmc", "mfma", "valu"], default="stats")
    ap.add_argument("--save-fields", metavar="NPZ",
                    help="synthesise the batch's measured fields, write them to this file and exit")
    ap.add_argument("--load-fields", metavar="NPZ",
                    help="take the batch's measured fields from a file written by --save-fields instead of "
                         "synthesising them (profiled runs: only the step's kernels run on the device)")
    ap.add_argument("--tiles", metavar="CT,PB,FPP,APP",
                    help="use this tile / FFT-plan choice instead of autotuning (counter runs: no tuning "
                         "launches mixed into the step kernels' averages)")
    ap.add_argument("--all-variants", action="store_true",
                    help="after the timed steps, run one step under every tile / plan choice (counter runs: "
                         "every variant of every step kernel measured inside a step)")
    args = ap.parse_args()
    if args.summarize_rocprof:
        print(summarize_rocprof(args.summarize_rocprof, args.summary_kind, args.copy_calibration_mib or 256))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: instances are independent, so N GPUs would each run their own "
              "batch with no communication; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2602_13805_amd as pdf
    import seeded_inputs as si

    dev = "cuda:0"
    if args.mlp_forward_only:
        print(json.dumps(mlp_forward_only(pdf, si, args.mlp_forward_only, dev)))
        return
    wl = si.WORKLOADS["cfg2"]
    B = args.batch
    t0 = time.time()
    if args.load_fields:
        with np.load(args.load_fields) as f:
            esca, eps = f["esca"], f["eps"]
            if esca.shape[0] != B or int(f["seed0"]) != 0:
                raise SystemExit(f"{args.load_fields} holds another batch")
        log(f"loaded the measured fields of {B} instances")
    else:
        esca, eps = synthesize_batch(pdf, si, wl, B, dev)
        log(f"synthesised {B} instances in {time.time() - t0:.1f} s")
    synth_s = time.time() - t0
    if args.save_fields:
        np.savez(args.save_fields, esca=esca, eps=eps, seed0=0)
        if args.large_fields:
            large_fields(pdf, si, dev, args.large_fields)
        return

    if args.copy_calibration_mib:
        # an elementwise kernel (not a DMA copy): reads and writes exactly this many MiB each
        src = torch.ones(args.copy_calibration_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    tx = si.antenna_positions(wl.n_tx, wl.radius)
    rx = si.antenna_positions(wl.n_rx, wl.radius)
    s = pdf.Solver(wl.M, wl.side, wl.freq_hz, tx, rx, wl.K, batch=B, device=dev)
    s.set_data(torch.tensor(esca, dtype=s.cdtype, device=dev))
    alpha = s.init_alpha()
    if args.tiles:
        tuned = tuple(int(x) for x in args.tiles.split(","))
        s.set_tiles(*tuned)
    else:
        tuned, _ = s.autotune(5)   # tile shapes and FFT plans; results do not depend on them
    log(f"tiles (column tiles, load batch, forward plan, adjoint plan) = {tuned}")
    m, v, t = s.new_state()
    loss = torch.empty((B, pdf.LOSS_STRIDE), dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        s.step(alpha, m, v, t, loss)
    torch.cuda.synchronize()
    # the timed steps carry no instrumentation; the per-kernel durations come from a second pass of
    # the same number of steps with HIP events between the kernels
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.step(alpha, m, v, t, loss)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.timing(True, args.steps)
    for _ in range(args.steps):
        s.step(alpha, m, v, t, loss)
    kern_ms, nrec = s.timing_read()
    s.timing(False)
    value = B * args.steps / dt
    log(f"{args.steps} steps x {B} instances in {dt:.3f} s: {value:.1f} instance-iters/s; kernels {kern_ms}")
    if not np.all(np.isfinite(loss.cpu().numpy()[:, 5])):
        raise RuntimeError("non-finite loss in the timed steps")
    if args.all_variants:
        for ct in (1, 2, 4):
            for pb in (4, 8):
                for plan in range(4):
                    s.set_tiles(ct, pb, plan >> 1, plan & 1)
                    s.step(alpha, m, v, t, loss)
        s.set_tiles(*tuned)
        torch.cuda.synchronize()

    bytes_, flops = workload_cost(wl, B, s_ntiles(wl.M))
    dom = max(kern_ms, key=kern_ms.get)
    dur = kern_ms[dom] * 1e-3
    t_hbm, t_alu = bytes_[dom] / HBM_PEAK, flops[dom] / FP32_PEAK
    if t_alu > t_hbm:
        roof = dict(bound="alu", achieved=flops[dom] / dur / 1e12, peak=FP32_PEAK / 1e12, unit="TFLOP/s")
    else:
        roof = dict(bound="hbm", achieved=bytes_[dom] / dur / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"], roof["traffic_source"] = measured_traffic(dom, tuned_variants(wl, tuned)[dom])
    roof["kernel"] = dom
    roof["algorithmic_bytes"] = bytes_[dom]
    roof["algorithmic_flops"] = flops[dom]
    roof["hbm_frac"] = bytes_[dom] / dur / HBM_PEAK
    roof["alu_frac"] = flops[dom] / dur / FP32_PEAK
    per_kernel = {k: dict(ms=kern_ms[k], GBps=bytes_[k] / (kern_ms[k] * 1e-3) / 1e9,
                          TFLOPs=flops[k] / (kern_ms[k] * 1e-3) / 1e12) for k in kern_ms}
    # the receiver GEMMs run their complex products as FP32 MFMA (8 N_s real flops per pixel and
    # incidence); their MFMA utilisation against the dense FP32 matrix peak
    mfma_flops = {"pixel_reduce": B * wl.n_tx * wl.M ** 2 * 8 * wl.n_rx,
                  "adj_gemm": B * wl.n_tx * wl.M ** 2 * 8 * wl.n_rx}
    mfma_util = {k: v / (kern_ms[k] * 1e-3) / FP32_PEAK for k, v in mfma_flops.items()}

    extra = {}
    eps_t = torch.tensor(eps, dtype=s.cdtype, device=dev)
    net_run = None
    if args.fcnn_iters > 0:
        # first use of the network path (its buffers, the kernels' code objects) outside the clock
        network_errors(pdf, si, s, eps_t, args.fcnn_hidden, 10, dev=dev)
        net_run = network_errors(pdf, si, s, eps_t, args.fcnn_hidden, args.fcnn_iters, dev=dev)
    if not args.no_recon and net_run is not None:
        extra["reconstructions"] = reconstruction_leg(pdf, s, eps_t, net_run, args.fcnn_hidden, args.fcnn_iters,
                                                      dev)
        # one instance alone (the first whose start is above the target): graph-replayed iterations
        e0 = net_run["err0"].cpu().numpy()
        i1 = int(np.argmax(e0 > TARGETS[-1]))
        R = args.recon_iters
        s1 = pdf.Solver(wl.M, wl.side, wl.freq_hz, tx, rx, wl.K, batch=1, device=dev)
        s1.set_data(torch.tensor(esca[i1:i1 + 1], dtype=s1.cdtype, device=dev))
        s1.reconstruct(50, n_check=50)
        one = s1.reconstruct(R, n_check=R)
        extra["single_instance"] = dict(instance=i1, iters_per_s=R / one["seconds"],
                                        note="direct Adam iterations of one instance from a replayed graph")
        s1.close()
        log(f"reconstructions: {extra}")
        if args.warm_pairs > 0:
            extra["warm_start"] = warm_start_leg(pdf, si, wl, s, eps_t, net_run, args, dev)
            log(f"warm start: {extra['warm_start']}")
    if args.fcnn_iters > 0:
        extra["coefficient_network"] = fcnn_leg(pdf, si, wl, s, eps, args.fcnn_hidden, args.fcnn_iters,
                                                args.steps, dev, r=net_run)
        log(f"coefficient network: {extra['coefficient_network']}")
    if args.csi:
        extra["csi_start"] = csi_leg(pdf, si, wl, s, eps, dev)
        log(f"CSI start: {extra['csi_start']}")
    if args.positions > 0:
        extra["position_uncertainty"] = positions_leg(pdf, si, wl, args.positions, dev)
        log(f"position uncertainty: {extra['position_uncertainty']}")
    if args.sweep_batch > 0:
        extra["parameter_sweep"] = sweep_leg(pdf, si, wl, args.sweep_batch, dev)
        log(f"parameter sweep: {extra['parameter_sweep']}")
    if args.uneven > 0:
        extra["uneven_batch"] = uneven_leg(pdf, si, wl, args.uneven, 200, dev)
        log(f"uneven batch: {extra['uneven_batch']}")
    if args.large > 0:
        extra["large_multifrequency"] = large_leg(pdf, si, args.large, dev, args.large_fields)
        log(f"large multi-frequency: {extra['large_multifrequency']}")
    s.close()

    out = {
        "metric": METRIC, "value": value, "unit": "instance-iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "cfg2: 64x64 grid over 2 wavelengths, 32 Tx / 32 Rx on a 3-wavelength circle, "
                               "K=15, FP32; fields from FP64 MoM on 128x128 with +-2 deg jitter and 10% AWGN",
                   "batch": B, "M": wl.M, "K": wl.K, "n_tx": wl.n_tx, "n_rx": wl.n_rx,
                   "freq_hz": wl.freq_hz, "parallelism": "none (one GPU, independent instances)"},
        "roofline": roof, "kernels": per_kernel,
        "effective_hbm": dict(
            floor_bytes_per_instance_iteration=floor_bytes(wl.M, wl.n_tx, wl.n_rx, wl.K),
            GBps=B * floor_bytes(wl.M, wl.n_tx, wl.n_rx, wl.K) / (dt / args.steps) / 1e9,
            frac=B * floor_bytes(wl.M, wl.n_tx, wl.n_rx, wl.K) / (dt / args.steps) / HBM_PEAK,
            basis="floor bytes (tables counted per instance) x batch / time per batched step / 8 TB/s"),
        "mfma_utilisation": dict(mfma_util, basis="MFMA flops of the kernel / its duration / 157.3 TFLOP/s "
                                                  "(dense FP32 matrix peak)"), "timed_kernel_steps": nrec, "synthesis_seconds": None if args.load_fields else synth_s,
        "tiles": dict(gemm_column_tiles=tuned[0], reduce_load_batch=tuned[1], fwd_plan=tuned[2],
                      adj_plan=tuned[3], source="given" if args.tiles else "autotuned"),
        "paper_context": {"seconds_per_reconstruction": 0.88, "hardware": "1x RTX 4090",
                          "note": "Table 1; 64x64, 36/36 antennas at 20 wavelengths, iteration count not stated"},
    }
    out.update(extra)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(si, wl, esca[0], args.cpu_seconds)
        rec = out.get("reconstructions")
        it = rec["network"][f"{TARGETS[-1]:.2f}"]["mean_iters"] if rec else None
        if it:
            # the network adds little to the physics step on the CPU: extrapolated from the direct rate
            out["cpu_baseline"]["seconds_per_reconstruction_extrapolated"] = it / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


def fcnn_cost(B, R, K, H):
    """Algorithmic HBM bytes and flops of the coefficient network's kernels in one step (FP32):
    forward (3 layers), pre-activation gradients (2 layers), weight gradients with Adam."""
    D = 2 * K * K
    layers = [(D, H), (H, H), (H, D)]
    P = sum((i + 1) * o for i, o in layers)
    fwd_b = 4 * B * sum((i + 1) * o + R * (i + o) for i, o in layers)
    fwd_f = 2 * B * R * sum(i * o for i, o in layers)
    bwd_b = 4 * B * sum(i * o + R * (o + 2 * i) for i, o in layers[1:])
    bwd_f = 2 * B * R * sum(i * o for i, o in layers[1:])
    adam_b = 4 * B * (6 * P + sum(R * (i + o) for i, o in layers))
    adam_f = B * (2 * R * P + 10 * P)
    return dict(fwd=(fwd_b, fwd_f), bwd=(bwd_b, bwd_f), adam=(adam_b, adam_f)), P


TARGETS = (0.40, 0.30)   # fixed relative image errors of the reconstruction counts


def network_errors(pdf, si, s, eps_t, H, iters, record_at=(), dev="cuda:0", a0=None, start=None):
    """Coefficient-network reconstructions of every instance of s (reading Z20 scales, output layer
    zero at the start): image error at the start, its minimum over checks every 10 steps, the error
    after each step count in record_at, and the first checked step at or below each of TARGETS
    (0 if the start is already there, -1 if never).  The networks' initial weights are an input
    (seeded draws, resident on the device before the clock starts, as the measured fields are); the
    clock starts before the start value is computed (start(), else the back-propagation start,
    unless a0 is given) and is read after every check (clock[t] = seconds until the check after
    step t)."""
    import torch
    B, K = s.B, s.K
    theta = torch.tensor(si.fcnn_theta(1, B, K, H, out_scale=0.0), dtype=s.rdtype, device=dev)
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    loss = torch.empty((B, pdf.LOSS_STRIDE), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    if a0 is None:
        a0 = start() if start is not None else s.init_alpha()
    sc = dict(s_in=1.0 / math.sqrt(pdf.mean_abs2(a0)), s_out=1.0 / H)
    ah = torch.empty_like(a0)
    _, _, err0 = s.image(a0, eps_t)
    best, at = err0.clone(), {}
    first = {tg: torch.where(err0 <= tg, 0, -1) for tg in TARGETS}
    torch.cuda.synchronize()
    clock = {0: time.perf_counter() - t_start}
    for t in range(1, iters + 1):
        s.fcnn_step(H, a0, theta, m, v, t, ah, loss, **sc)
        if t % 10 == 0 or t in record_at:
            _, _, err = s.image(s.fcnn_forward(H, a0, theta, **sc), eps_t)
            if t in record_at:
                at[t] = err
            if t % 10 == 0:
                best = torch.minimum(best, err)
                for tg in TARGETS:
                    first[tg] = torch.where((first[tg] < 0) & (err <= tg), t, first[tg])
                torch.cuda.synchronize()
                clock[t] = time.perf_counter() - t_start
    return dict(a0=a0, theta=theta, m=m, v=v, ah=ah, loss=loss, sc=sc, t=iters, err0=err0, best=best,
                at=at, first=first, clock=clock, seconds=time.perf_counter() - t_start)


def fixed_target_counts(first, clock, err0_bp):
    """Reconstructions to each fixed image error: only instances whose back-propagation start is
    worse than the target count (err0_bp > target), and one is reconstructed at the first check at
    or below the target.  seconds = the clock at the last check at which a counted instance first
    got there (the batch could stop there), per_s = reconstructions / seconds."""
    import numpy as np
    e0 = err0_bp.cpu().numpy() if hasattr(err0_bp, "cpu") else np.asarray(err0_bp)
    out = {}
    for tg in TARGETS:
        f = first[tg].cpu().numpy() if hasattr(first[tg], "cpu") else np.asarray(first[tg])
        elig = e0 > tg
        hit = elig & (f >= 0)
        n = int(hit.sum())
        secs = clock(int(f[hit].max())) if n else None
        out[f"{tg:.2f}"] = dict(n_counted=int(elig.sum()), n_reached=n,
                                frac_reached=n / max(int(elig.sum()), 1),
                                mean_iters=float(f[hit].mean()) if n else None,
                                seconds=secs, per_s=(n / secs) if n and secs > 0 else None)
    return out


def reconstruction_leg(pdf, s, eps_t, r, H, iters, dev):
    """Reconstructions/s of the benchmark batch to fixed image errors (TARGETS), through the solver
    of Sec. 3.1 (Adam on the coefficient network's weights, r = network_errors from the
    back-propagation start), with direct Adam on alpha from the same start as context (its time
    scaled to the last check at which a counted instance reached the target)."""
    import torch
    net = fixed_target_counts(r["first"], lambda t: r["clock"][t], r["err0"])
    direct = {}
    for tg in TARGETS:
        d = s.reconstruct(iters, n_check=10, eps_true=eps_t,
                          target=torch.full((s.B,), tg, dtype=torch.float64, device=dev))
        secs, run = d["seconds"], max(d["iters_run"], 1)
        counts = fixed_target_counts({t2: d["reached"] for t2 in TARGETS}, lambda t: secs * t / run, r["err0"])
        direct[f"{tg:.2f}"] = counts[f"{tg:.2f}"]
    head = net[f"{TARGETS[-1]:.2f}"]
    return dict(
        per_s=head["per_s"], target_image_error=TARGETS[-1], batch=s.B, iterations=iters, check_every=10,
        solver=f"Sec. 3.1: Adam (lr 1e-2) on the weights of the untrained coefficient network (hidden "
               f"width {H}), from the back-propagation start",
        network=net, direct_adam=direct,
        mean_start_image_error=float(r["err0"].mean()), mean_best_image_error=float(r["best"].mean()),
        definition="an instance counts if its back-propagation start error is above the target; it is "
                   "reconstructed at the first check (every 10 steps) at or below the target; the clock "
                   "runs from the start value to the last check at which a counted instance first got "
                   "there")


def fcnn_leg(pdf, si, wl, s, eps, H, iters, steps, dev, r=None):
    """The coefficient network (Sec. 3.1): Adam on per-instance network weights theta, the loss taken
    at alpha_hat = alpha_0 + f_theta(alpha_0), from the same back-propagation start as the direct
    optimisation.  Image error reached in `iters` steps (checked every 10; r: that run, if already
    made) next to the direct optimisation's, then `steps` timed steps split into network and
    physics kernels."""
    import numpy as np
    import torch
    B, K = s.B, s.K
    eps_t = torch.tensor(eps, dtype=s.cdtype, device=dev)
    if r is None:
        r = network_errors(pdf, si, s, eps_t, H, iters, dev=dev)
    a0, theta, m, v, ah, loss, sc, t = (r[k] for k in ("a0", "theta", "m", "v", "ah", "loss", "sc", "t"))
    err0, best = r["err0"], r["best"]
    if not np.all(np.isfinite(loss.cpu().numpy()[:, 5])):
        raise RuntimeError("non-finite loss in the coefficient-network steps")
    direct = s.reconstruct(iters, n_check=10, eps_true=eps_t)
    best_d = direct["best_err"].cpu().numpy()
    best_n = best.cpu().numpy()
    # timed steps, continuing from the trained weights, without instrumentation; then as many steps
    # with HIP events between the physics kernels for their durations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        t += 1
        s.fcnn_step(H, a0, theta, m, v, t, ah, loss, **sc)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.timing(True, steps)
    for _ in range(steps):
        t += 1
        s.fcnn_step(H, a0, theta, m, v, t, ah, loss, **sc)
    phys_ms, _ = s.timing_read()
    s.timing(False)
    t0 = time.perf_counter()
    for _ in range(steps):
        s.fcnn_forward(H, a0, theta, **sc)
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t0) / steps * 1e3
    step_ms = dt / steps * 1e3
    net_ms = step_ms - sum(phys_ms.values())
    cost, P = fcnn_cost(B, s.Ni, K, H)
    net_bytes = sum(c[0] for c in cost.values())
    net_flops = sum(c[1] for c in cost.values())
    return dict(
        hidden=H, params_per_instance=P, iterations=iters, s_in=sc["s_in"], s_out=sc["s_out"],
        mean_best_image_error=float(best_n.mean()), mean_best_image_error_direct=float(best_d.mean()),
        mean_start_image_error=float(err0.cpu().numpy().mean()),
        frac_better_than_direct=float(np.mean(best_n < best_d - 1e-6)),
        frac_improved_on_start=float(np.mean(best_n < err0.cpu().numpy() - 1e-6)),
        frac_improved_on_start_direct=float(np.mean(best_d < err0.cpu().numpy() - 1e-6)), check_every=10,
        instance_iters_per_s=B * steps / dt, ms_per_step=step_ms, physics_kernels_ms=sum(phys_ms.values()),
        network_ms=net_ms, network_forward_ms=fwd_ms,
        network_roofline=dict(bound="hbm", algorithmic_bytes=net_bytes, algorithmic_flops=net_flops,
                              achieved=net_bytes / (net_ms * 1e-3) / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s",
                              frac=net_bytes / (net_ms * 1e-3) / HBM_PEAK,
                              basis="network kernels' algorithmic bytes / (step time - physics kernels' "
                                    "event-timed durations)"),
        start="back-propagation alpha_0; output layer zero, so alpha_hat = alpha_0 at step 1",
        weights="U[-1/sqrt(in), 1/sqrt(in)] hidden layers, seed 1")


H_NET = 256   # hidden width of the coefficient network in the benchmark's legs


def csi_leg(pdf, si, wl, s, eps, dev):
    """The full CSI start (Sec. 3.1) against the one-step start on the benchmark batch: its time for
    n conjugate-gradient steps, L^CSI-driven start image error, and the best image error of 100
    direct Adam iterations and of 100 network steps from it."""
    import numpy as np
    import torch
    eps_t = torch.tensor(eps, dtype=s.cdtype, device=dev)
    out = {}
    for n in (1, 5, 20):
        s.init_alpha_csi(n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a = s.init_alpha_csi(n)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        _, _, e0 = s.image(a, eps_t)
        d = s.reconstruct(100, n_check=10, alpha=a.clone(), eps_true=eps_t)
        r = network_errors(pdf, si, s, eps_t, H_NET, 100, dev=dev, a0=a)
        out[f"cg_steps={n}"] = dict(ms=ms, start_image_error=float(e0.mean()),
                                    direct_best_100=float(d["best_err"].mean()),
                                    network_best_100=float(r["best"].mean()))
    return dict(batch=s.B, per_steps=out,
                note="start = n CG steps on L^CSI with R fixed at the back-propagation R_0; n = 1 is the "
                     "benchmark's start; best image error over checks every 10 iterations, start included")


def positions_leg(pdf, si, wl, n_real, dev):
    """Antenna-position uncertainty (Sec. 4): one cfg2 profile measured with every Tx and Rx displaced
    by N(0, sigma^2) in x and y, sigma in {1, 2, 3} mm, n_real realisations each, plus the exact
    positions; all reconstructed with the nominal positions as one batch (direct Adam, 100
    iterations, and the coefficient network, 100 steps).  Noise-free, so the spread of the image
    error is the position errors' alone."""
    import numpy as np
    import torch
    sigmas = (0.0, 1e-3, 2e-3, 3e-3)
    shapes = si.draw_profile(wl, 0)
    tx0 = si.antenna_positions(wl.n_tx, wl.radius)
    rx0 = si.antenna_positions(wl.n_rx, wl.radius)
    txs, rxs = [], []
    for si_idx, sg in enumerate(sigmas):
        for r in range(n_real if sg > 0 else 1):
            dt, dr = si.draw_position_errors(1000 * si_idx + r, wl.n_tx, wl.n_rx, sg)
            txs.append(tx0 + dt)
            rxs.append(rx0 + dr)
    B = len(txs)
    epsf = si.rasterize(shapes, wl.M_fine, wl.side)
    eps = si.rasterize(shapes, wl.M, wl.side)
    t0 = time.time()
    es = pdf.synthesize_batch(wl.M_fine, wl.side, wl.freq_hz, txs, rxs, np.repeat(epsf[None], B, 0), tol=1e-10,
                              device=dev)
    synth_s = time.time() - t0
    # what a position error does to the data: relative change of the measured field against the
    # exact positions' (about linear in sigma); and, to separate it from the solver's own sensitivity
    # to any data change, n_real data sets with exact positions and random noise of the same
    # relative size as the 1 mm position errors' mean change
    change = np.linalg.norm((es - es[0]).reshape(B, -1), axis=1) / np.linalg.norm(es[0])
    nu = float(change[1:1 + n_real].mean())
    extra = np.stack([si.add_noise(es[0], nu, *si.draw_noise(50000 + r, es[0].shape)) for r in range(n_real)])
    es = np.concatenate([es, extra])
    B = es.shape[0]
    s = pdf.Solver(wl.M, wl.side, wl.freq_hz, tx0, rx0, wl.K, batch=B, device=dev)
    s.set_data(torch.tensor(es, dtype=s.cdtype, device=dev))
    eps_t = torch.tensor(np.repeat(eps[None], B, 0), dtype=s.cdtype, device=dev)
    res = s.reconstruct(100, n_check=100)
    _, _, e_dir = s.image(res["alpha"], eps_t)
    e_net = network_errors(pdf, si, s, eps_t, H_NET, 100, record_at=(100,), dev=dev)["at"][100]
    e_dir, e_net = e_dir.cpu().numpy(), e_net.cpu().numpy()
    out, i = {}, 0
    for sg in sigmas:
        n = n_real if sg > 0 else 1
        out[f"sigma={sg * 1e3:g}mm"] = dict(
            realisations=n, data_change=dict(mean=float(change[i:i + n].mean()), std=float(change[i:i + n].std())),
            direct=dict(mean=float(e_dir[i:i + n].mean()), std=float(e_dir[i:i + n].std())),
            network=dict(mean=float(e_net[i:i + n].mean()), std=float(e_net[i:i + n].std())))
        i += n
    out["exact positions, noise of the 1 mm data change"] = dict(
        realisations=n_real, relative_noise=nu,
        direct=dict(mean=float(e_dir[i:].mean()), std=float(e_dir[i:].std())),
        network=dict(mean=float(e_net[i:].mean()), std=float(e_net[i:].std())))
    s.close()
    return dict(instances=B, per_sigma=out, synthesis_seconds=synth_s,
                recipe="cfg2 profile seed 0, FP64 MoM on 128x128 at displaced antennas, no noise; "
                       "inversion with the nominal positions; image error after 100 iterations; data_change "
                       "= ||E_sca - E_sca(exact positions)|| / ||E_sca(exact positions)||")


def sweep_leg(pdf, si, wl, Bs, dev):
    """The sensitivity study of Sec. 4.1-4.2.1 on synthetic cfg2 profiles: beta in {3, 6, 9} x M_F in
    {6, 7, 9} (K = 2 M_F, the corner blocks) x SNR in {20, 10, 5} dB, each combination a handle of Bs
    instances (the same profiles and noise draws throughout), all 27 in one shape class and so
    advanced by one grouped launch per kernel.  Mean image error after k = 10, 30 and 100 Adam
    iterations from each handle's back-propagation start, and the grouped rate against the same
    handles run one after another; then the same combinations through the coefficient network."""
    import numpy as np
    import torch
    betas, mfs, snrs, ks = (3.0, 6.0, 9.0), (6, 7, 9), (20.0, 10.0, 5.0), (10, 30, 100)
    clean, eps = synthesize_batch(pdf, si, wl, Bs, dev, noise=0.0)
    tx = si.antenna_positions(wl.n_tx, wl.radius)
    rx = si.antenna_positions(wl.n_rx, wl.radius)
    eps_t = None
    sol, keys = [], []
    for snr in snrs:
        nu = 10.0 ** (-snr / 20.0)
        es = np.stack([si.add_noise(clean[b], nu, *si.draw_noise(b, clean[b].shape)) for b in range(Bs)])
        for beta in betas:
            for mf in mfs:
                p = pdf.default_params("fp32", beta=beta)
                sv = pdf.Solver(wl.M, wl.side, wl.freq_hz, tx, rx, 2 * mf, batch=Bs, params=p, device=dev)
                sv.set_data(torch.tensor(es, dtype=sv.cdtype, device=dev))
                if eps_t is None:
                    eps_t = torch.tensor(eps, dtype=sv.cdtype, device=dev)
                sol.append(sv)
                keys.append((beta, mf, snr))
    errs, timing = {}, {}
    for k in ks:
        got, info = pdf.reconstruct_multi(sol, k, n_check=k)
        for (beta, mf, snr), sv, g in zip(keys, sol, got):
            _, _, err = sv.image(g["alpha"], eps_t)
            errs.setdefault(f"beta={beta:g} M_F={mf} SNR={snr:g}dB", {})[f"k={k}"] = float(err.mean())
        timing[k] = info["seconds"]
    t0 = time.perf_counter()
    for sv in sol:
        sv.reconstruct(ks[-1], n_check=ks[-1])
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    n_inst = len(sol) * Bs
    best = min(errs, key=lambda c: errs[c][f"k={ks[-1]}"])
    # the paper's solver is the coefficient network: the same combinations through it (handle by
    # handle; the network has no grouped launch)
    errs_net = {}
    t0 = time.perf_counter()
    for (beta, mf, snr), sv in zip(keys, sol):
        r = network_errors(pdf, si, sv, eps_t, H_NET, ks[-1], record_at=ks, dev=dev)
        errs_net[f"beta={beta:g} M_F={mf} SNR={snr:g}dB"] = {f"k={k}": float(r["at"][k].mean()) for k in ks}
    torch.cuda.synchronize()
    net_s = time.perf_counter() - t0
    best_net = min(errs_net, key=lambda c: errs_net[c][f"k={ks[-1]}"])
    for sv in sol:
        sv.close()
    return dict(handles=len(sol), instances=n_inst, batch_per_handle=Bs,
                mean_image_error=errs, lowest_at_k100=best,
                network_mean_image_error=errs_net, network_lowest_at_k100=best_net,
                network_hidden=H_NET, network_seconds=net_s,
                grouped_instance_iters_per_s=n_inst * ks[-1] / timing[ks[-1]],
                sequential_instance_iters_per_s=n_inst * ks[-1] / seq,
                speedup_over_sequential=seq / timing[ks[-1]],
                recipe="cfg2 profiles seeds 0.., clean FP64 MoM with +-2 deg jitter, AWGN at the SNR "
                       "(relative level 10^(-SNR/20)), same draws for every combination")


def warm_start_leg(pdf, si, wl, s, eps_t, r_bp, args, dev):
    """Train the warm-start network on fresh MoM pairs, then reconstruct the same instances from its
    start with the solver of Sec. 3.1 to the fixed image errors, timed from the start value (the
    network's prediction, the physics-loss selection, the iterations), against the same solver from
    the back-propagation start (r_bp); the instances counted are those whose back-propagation start
    is above the target, for both starts."""
    import numpy as np
    import torch
    from paper_2602_13805_amd import warmstart as ws
    B, H = s.B, args.fcnn_hidden
    t0 = time.time()
    data = ws.make_dataset(si, wl, ws.TRAIN_SEED0 + np.arange(args.warm_pairs), dev, log=log)
    data_s = time.time() - t0
    tr = ws.train(data, epochs=args.warm_epochs, batch=256, lr=1e-3, seed=0, device=dev, log=log)
    # forward throughput of the network on a full batch (bfloat16 MFMA)
    x = data.x[:256].contiguous()
    tr.net.forward(x, tr.s_in, tr.s_out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nf = 20
    for _ in range(nf):
        tr.net.forward(x, tr.s_in, tr.s_out)
    torch.cuda.synchronize()
    fwd_s = (time.perf_counter() - t1) / nf
    sizes = tr.net.sizes
    fwd_flops = 2.0 * 256 * sum(a * b for a, b in zip(sizes[:-1], sizes[1:]))
    del data
    chosen = {}

    def start():
        a, ch, _ = s.warm_start(tr.net, tr.s_in, tr.s_out)
        chosen["c"] = ch
        return a
    start()   # first use of the warm-start path outside the clock
    rw = network_errors(pdf, si, s, eps_t, H, args.fcnn_iters, dev=dev, start=start)
    warm = fixed_target_counts(rw["first"], lambda t: rw["clock"][t], r_bp["err0"])
    plain = fixed_target_counts(r_bp["first"], lambda t: r_bp["clock"][t], r_bp["err0"])
    tr.net.close()
    return dict(
        per_s=warm[f"{TARGETS[-1]:.2f}"]["per_s"], per_s_plain=plain[f"{TARGETS[-1]:.2f}"]["per_s"],
        target_image_error=TARGETS[-1], fixed_error_targets=dict(warm=warm, plain=plain),
        mean_start_image_error=float(rw["err0"].mean()), mean_start_image_error_plain=float(r_bp["err0"].mean()),
        mean_best_image_error=float(rw["best"].mean()), mean_best_image_error_plain=float(r_bp["best"].mean()),
        frac_network_start=float(chosen["c"].float().mean()), batch=B,
        solver="Sec. 3.1 coefficient network from either start, %d steps, checked every 10" % args.fcnn_iters,
        training=dict(pairs=args.warm_pairs, epochs=args.warm_epochs, steps=tr.steps, batch=256,
                      seconds=tr.seconds, data_seconds=data_s, first_epoch_mse=tr.history[0],
                      last_epoch_mse=tr.history[-1], widths=sizes,
                      data="cfg2 profiles, seeds 1000000 + i, FP64 MoM on 128x128 with jitter and noise; "
                           "targets F_T of the true induced currents on the 64x64 grid"),
        network_forward=dict(rows=256, ms=fwd_s * 1e3, tflops=fwd_flops / fwd_s / 1e12,
                             peak_tflops=2500.0, frac=fwd_flops / fwd_s / 2.5e15))


def uneven_leg(pdf, si, wl, n_inst, iters, dev):
    """Instances of uneven shapes (cfg3-style draws on the GPU-supported grids): one handle per
    shape, all advanced in one graph per 10 steps, against the same handles one after another."""
    import dataclasses
    import numpy as np
    import torch
    shapes = si.uneven_shapes(n_inst, seed=2026)
    groups = {}
    for i, key in enumerate(shapes):
        groups.setdefault(key, []).append(i)
    sols = []
    t0 = time.time()
    for (M, a, K), idx in sorted(groups.items()):
        # fields from the MoM on the 2M grid; the 128^2 instances on their own grid, since a 256^2
        # support of up to three cfg2 objects can exceed the dense support solve's 20000 pixels
        Mf = 2 * M if 2 * M <= 128 else M
        w = dataclasses.replace(wl, M=M, n_tx=a, n_rx=a, K=K, M_fine=Mf)
        txs, rxs, epsf = [], [], np.zeros((len(idx), Mf, Mf), np.complex128)
        for j, seed in enumerate(idx):
            jt, jr = si.draw_jitter(seed, a, a, w.jitter_deg)
            txs.append(si.antenna_positions(a, w.radius, angle_offsets=jt))
            rxs.append(si.antenna_positions(a, w.radius, angle_offsets=jr))
            epsf[j] = si.rasterize(si.draw_profile(w, seed), Mf, w.side)
        es = pdf.synthesize_batch(Mf, w.side, w.freq_hz, txs, rxs, epsf, tol=1e-10, device=dev)
        for j, seed in enumerate(idx):
            n1, n2 = si.draw_noise(seed, es[j].shape)
            es[j] = si.add_noise(es[j], w.noise, n1, n2)
        s = pdf.Solver(M, w.side, w.freq_hz, si.antenna_positions(a, w.radius), si.antenna_positions(a, w.radius),
                       K, batch=len(idx), device=dev)
        s.set_data(torch.tensor(es, dtype=s.cdtype, device=dev))
        sols.append(s)
    setup_s = time.time() - t0
    pdf.reconstruct_multi(sols, 10, n_check=10)   # tunes every handle, warms the graph path
    torch.cuda.synchronize()
    _, info = pdf.reconstruct_multi(sols, iters, n_check=10)
    multi_s = info["seconds"]
    seq_s = 0.0
    for s in sols:
        seq_s += s.reconstruct(iters, n_check=10)["seconds"]
    tiles = {}
    for s in sols:
        ch, _ = s.autotune(3)
        tiles[str(ch)] = tiles.get(str(ch), 0) + s.B
    for s in sols:
        s.close()
    work = n_inst * iters
    floor = sum(floor_bytes(M, a, a, K) for (M, a, K) in shapes)
    return dict(instances=n_inst, handles=len(sols), iterations=iters,
                floor_bytes_per_batched_iteration=floor,
                effective_hbm=dict(GBps=floor * iters / multi_s / 1e9, frac=floor * iters / multi_s / HBM_PEAK,
                                   basis="per instance 8 B x [N_i N + 2 N_s N + 2 (2M)^2 + N_s N_i + 6 N_i K^2] "
                                         "(E_inc once, G_S and the G_D spectrum twice, data, alpha/m/v read "
                                         "and written), summed over the instances, per batched iteration"),
                shapes="M from {32, 48, 64, 96, 128}, N_i = N_s from {16, 24, 32, 48, 64}, K odd 7..21 (K <= M), "
                       "cfg2 profiles; fields from MoM on the 2M grid (128^2: on the 128^2 grid)",
                instance_iters_per_s=work / multi_s, seconds=multi_s,
                sequential_instance_iters_per_s=work / seq_s, sequential_seconds=seq_s,
                speedup_over_sequential=seq_s / multi_s, setup_seconds=setup_s,
                tile_choices_by_instances=tiles)


def large_fields(pdf, si, dev, path=None):
    """Measured fields of the large multi-frequency leg [F][Ni][Ns] and the true permittivity:
    from `path` if it exists, else synthesised (and written to `path` if given)."""
    import numpy as np
    wl = si.WORKLOADS["cfg5"]
    shapes = si.draw_profile(wl, 0)
    eps = si.rasterize(shapes, wl.M, wl.side)
    if path and os.path.exists(path):
        with np.load(path) as f:
            return f["esca"], eps, 0.0
    freqs = [wl.freq_hz * m for m in wl.freq_mult]
    tx = si.antenna_positions(wl.n_tx, wl.radius)
    rx = si.antenna_positions(wl.n_rx, wl.radius)
    t0 = time.time()
    es = []
    for f, fr in enumerate(freqs):
        # an iterative-solve tolerance far below the 5 % noise: at 2.5 x 400 MHz over 8 wavelengths
        # BiCGSTAB stalls near 1e-5
        e = pdf.synthesize_batch(wl.M, wl.side, fr, [tx], [rx], eps[None], tol=1e-4, device=dev)[0]
        es.append(si.add_noise(e, wl.noise, *si.draw_noise(f, e.shape)))
    es = np.stack(es)
    if path:
        np.savez(path, esca=es)
    return es, eps, time.time() - t0


def large_leg(pdf, si, iters, dev, fields=None):
    """The large multi-frequency reconstruction: 256x256 over 8 wavelengths, 64 Tx / 64 Rx on a
    10-wavelength circle, frequencies 1, 1.5, 2 and 2.5 x 400 MHz, K = 41 per incidence and frequency,
    5-10 discs and rings with eps_r in [1.5, 3.5], 5 % noise, FP32; one contrast for all frequencies.
    Measured fields: the library's FP64 MoM on the 256x256 grid itself (a 512x512 support has too many
    pixels for the dense support solve), iterated to a relative residual of 1e-4.  Timed: `iters` Adam steps (loss, adjoint, update), after
    the start value and a warm-up."""
    import numpy as np
    import torch
    wl = si.WORKLOADS["cfg5"]
    freqs = [wl.freq_hz * m for m in wl.freq_mult]
    F, Ni, Ns, M, K = len(freqs), wl.n_tx, wl.n_rx, wl.M, wl.K
    tx = si.antenna_positions(Ni, wl.radius)
    rx = si.antenna_positions(Ns, wl.radius)
    es, eps, synth_s = large_fields(pdf, si, dev, fields)
    s = pdf.Solver(M, wl.side, freqs, tx, rx, K, batch=1, device=dev)
    s.set_data(torch.tensor(es.reshape(1, F * Ni, Ns), dtype=s.cdtype, device=dev))
    tuned, _ = s.autotune(3)
    eps_t = torch.tensor(eps[None], dtype=s.cdtype, device=dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    a = s.init_alpha()
    torch.cuda.synchronize()
    init_ms = (time.perf_counter() - t1) * 1e3
    _, _, e0 = s.image(a, eps_t)
    m, v, t = s.new_state()
    loss = torch.empty((1, pdf.LOSS_STRIDE), dtype=torch.float64, device=dev)
    for _ in range(5):
        s.step(a, m, v, t, loss)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(iters):
        s.step(a, m, v, t, loss)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    _, _, e1 = s.image(a, eps_t)
    lo = loss.cpu().numpy()[0]
    if not np.isfinite(lo[5]):
        raise RuntimeError("non-finite loss in the large multi-frequency leg")
    floor = F * floor_bytes(M, Ni, Ns, K)
    # flops per iteration: per frequency and incidence the forward and adjoint convolutions
    # (2 x (row, column, row) length-2M transforms over the padded half), synthesis and analysis,
    # plus the receiver GEMMs (8 N_s real flops per pixel and incidence, forward and adjoint)
    P = 2 * M
    conv = 2 * (2 * M * 5 * P * np.log2(P) + 2 * P * 5 * P * np.log2(P))
    flops = F * Ni * (conv + 2 * (M + K) * 5 * M * np.log2(M) + 2 * 8 * Ns * M * M)
    s.close()
    return dict(grid=M, frequencies=freqs, n_tx=Ni, n_rx=Ns, K=K, precision="fp32", iterations=iters,
                ms_per_iteration=dt / iters * 1e3, iters_per_s=iters / dt, start_ms=init_ms,
                start_image_error=float(e0.item()), image_error_after=float(e1.item()),
                loss_after=float(lo[5]), tiles=list(tuned), synthesis_seconds=synth_s,
                effective_hbm=dict(floor_bytes=floor, GBps=floor / (dt / iters) / 1e9,
                                   frac=floor / (dt / iters) / HBM_PEAK),
                flops_per_iteration=float(flops), tflops=float(flops / (dt / iters) / 1e12),
                adjoint="recompute mode: the adjoint keeps no FFT intermediates of the forward pass (only J "
                        "and E) and recomputes its transforms",
                data="FP64 MoM on the 256x256 inversion grid per frequency, 5 % noise; cfg5 profile seed 0")


def mlp_forward_only(pdf, si, calls, dev):
    """Forward passes of 256 rows through the warm-start network at its trained widths (the
    flattened 32 x 32 complex field in, 32 x 15 x 15 complex coefficients out), with seeded weights
    and inputs: its kernels without the data synthesis the trained network needs."""
    import torch
    from paper_2602_13805_amd import warmstart
    wl = si.WORKLOADS["cfg2"]
    sizes = [2 * wl.n_tx * wl.n_rx, *warmstart.HIDDEN, 2 * wl.n_tx * wl.K * wl.K]
    net = pdf.Mlp(sizes, 256, device=dev)
    net.init_weights(1)
    g = torch.Generator().manual_seed(5)
    x = torch.randn(256, sizes[0], generator=g).to(dev)
    for _ in range(5):
        net.forward(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        net.forward(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / calls
    flops = 2.0 * 256 * sum(a * b for a, b in zip(sizes[:-1], sizes[1:]))
    net.close()
    return dict(widths=sizes, rows=256, calls=calls, us_per_call=dt * 1e6, tflops_per_call=flops / dt / 1e12,
                note="per call, host marshalling included; the kernels' own durations come from a kernel trace")


def floor_bytes(M, n_tx, n_rx, K, csz=8):
    """Algorithmic HBM bytes of one instance-iteration when every per-incidence intermediate stays on
    chip: E_inc read once, G_S and the padded G_D spectrum twice (forward and adjoint), the data, and
    alpha, m, v read and written."""
    N, P = M * M, 2 * M
    return csz * (n_tx * N + 2 * n_rx * N + 2 * P * P + n_rx * n_tx + 6 * n_tx * K * K)


def si_start_error(s, eps_t):
    """Image error of each instance at the start value."""
    _, _, err = s.image(s.init_alpha(), eps_t)
    return err.cpu().numpy()


def s_ntiles(M):
    N = M * M
    return (N + 255) // 256


if __name__ == "__main__":
    main()
