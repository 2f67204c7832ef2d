"""Learned warm start for the PDF iteration (an addition to the method).

A fully connected network (library: pdf_mlp_*) maps the measured fields of
one instance to start coefficients alpha_0.  Its training pairs come from the
method's own FP64 MoM forward solver: random profiles of the workload, fields
at jittered antennas plus noise as input, and as target the kept Fourier
coefficients F_T(J) of the true induced currents J = chi E_tot (averaged onto
the inversion grid).  At use, pdf_warm_start keeps the network's start only
where its physics loss is below the back-propagation start's, so the plain
method remains the fallback.

Every arithmetic step runs in the library; this module draws the seeded
inputs, moves arrays and loops over batches.
"""
from __future__ import annotations

import dataclasses
import math
import time
from concurrent.futures import ThreadPoolExecutor
from typing import Optional, Sequence

import numpy as np
import torch

from . import binding as _b

# widths: 2 Ni Ns inputs, three hidden layers of 1024, 2 Ni K^2 outputs
HIDDEN = (1024, 1024, 1024)
TRAIN_SEED0 = 1_000_000   # training profiles use seeds TRAIN_SEED0 + i, disjoint from evaluation seeds


@dataclasses.dataclass
class Dataset:
    x: torch.Tensor          # [n, 2 Ni Ns] float32: measured fields, interleaved (Re, Im)
    t: torch.Tensor          # [n, 2 Ni K^2] float32: target coefficients, interleaved (Re, Im)
    eps: np.ndarray          # [n, M, M] complex128: permittivity on the inversion grid
    seeds: np.ndarray


def make_dataset(si, wl, seeds: Sequence[int], device: str = "cuda:0", chunk: int = 512,
                 log=None) -> Dataset:
    """Training / evaluation pairs of workload `wl` (a seeded_inputs.Workload) for the given seeds."""
    Ni, Ns, M, K = wl.n_tx, wl.n_rx, wl.M, wl.K
    d = wl.M_fine // M
    if d * M != wl.M_fine:
        raise ValueError("the fine grid must be a multiple of the inversion grid")
    tx = si.antenna_positions(Ni, wl.radius)
    rx = si.antenna_positions(Ns, wl.radius)
    sv = _b.Solver(M, wl.side, wl.freq_hz, tx, rx, K, batch=1, device=device)
    xs, ts, eps_all = [], [], []
    seeds = np.asarray(seeds, dtype=np.int64)
    t0 = time.time()
    def draw(s):
        shapes = si.draw_profile(wl, int(s))
        jt, jr = si.draw_jitter(int(s), Ni, Ns, wl.jitter_deg)
        return (si.antenna_positions(Ni, wl.radius, angle_offsets=jt),
                si.antenna_positions(Ns, wl.radius, angle_offsets=jr),
                si.rasterize(shapes, wl.M_fine, wl.side), si.rasterize(shapes, M, wl.side))

    pool = ThreadPoolExecutor(max_workers=8)
    for c0 in range(0, len(seeds), chunk):
        cs = seeds[c0:c0 + chunk]
        drawn = list(pool.map(draw, cs))   # seeded per instance: the order of completion does not matter
        txs = [d[0] for d in drawn]
        rxs = [d[1] for d in drawn]
        epsf = np.stack([d[2] for d in drawn])
        eps_all.extend(d[3] for d in drawn)
        es, jc = _b.synthesize_batch(wl.M_fine, wl.side, wl.freq_hz, txs, rxs, epsf, tol=1e-10, coarse=d,
                                     device=device)
        for i, s in enumerate(cs):
            n1, n2 = si.draw_noise(int(s), es[i].shape)
            es[i] = si.add_noise(es[i], wl.noise, n1, n2)
        x = torch.tensor(es.astype(np.complex64), device=device)
        alpha = sv.analyze(torch.tensor(jc, dtype=torch.complex64, device=device))
        xs.append(torch.view_as_real(x).reshape(len(cs), -1).contiguous())
        ts.append(torch.view_as_real(alpha).reshape(len(cs), -1).contiguous())
        if log:
            log(f"  warm-start data {c0 + len(cs)}/{len(seeds)} ({time.time() - t0:.1f} s)")
    pool.shutdown()
    sv.close()
    return Dataset(torch.cat(xs), torch.cat(ts), np.stack(eps_all), seeds)


@dataclasses.dataclass
class Trained:
    net: "_b.Mlp"
    s_in: float
    s_out: float
    history: list
    seconds: float
    steps: int


def train(data: Dataset, epochs: int = 40, batch: int = 256, lr: float = 1e-3, seed: int = 0,
          device: str = "cuda:0", hidden: Sequence[int] = HIDDEN, log=None) -> Trained:
    """Trains a new network on `data` (inputs and targets scaled to unit RMS)."""
    n, n_in = data.x.shape
    n_out = data.t.shape[1]
    s_in = 1.0 / math.sqrt(_b.mean_abs2(data.x))
    s_out = math.sqrt(_b.mean_abs2(data.t))
    tn = (data.t / s_out).contiguous()
    net = _b.Mlp([n_in, *hidden, n_out], batch_max=batch, device=device)
    net.init_weights(seed)
    rng = np.random.Generator(np.random.PCG64(seed))
    loss = torch.zeros(1, dtype=torch.float64, device=device)
    history, steps = [], 0
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(n).astype(np.int32), device=device)
        acc, cnt = torch.zeros((), dtype=torch.float64, device=device), 0
        for b0 in range(0, n - batch + 1 if n >= batch else 1, batch):
            idx = perm[b0:b0 + min(batch, n)]
            net.train_step(data.x, tn, idx, s_in, lr, loss)
            acc += loss[0]
            cnt += 1
            steps += 1
        history.append(float(acc) / max(cnt, 1))
        if log and (ep % 10 == 0 or ep == epochs - 1):
            log(f"  warm-start epoch {ep}: mse {history[-1]:.4f}")
    torch.cuda.synchronize(device)
    return Trained(net, s_in, s_out, history, time.perf_counter() - t0, steps)


def predict(tr: Trained, x: torch.Tensor) -> torch.Tensor:
    """Network start coefficients [n, 2 Ni K^2] (interleaved) for fields x [n, 2 Ni Ns]."""
    out = []
    for b0 in range(0, x.shape[0], tr.net.batch_max):
        out.append(tr.net.forward(x[b0:b0 + tr.net.batch_max].contiguous(), tr.s_in, tr.s_out))
    return torch.cat(out)
