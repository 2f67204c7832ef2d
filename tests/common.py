"""Shared problem builders for the parity tests: seeded inputs -> oracle problem
and the matching GPU inputs."""
import numpy as np

import seeded_inputs as si
from oracle import forward, loss as oloss, operators as ops


def geometry(n_tx, n_rx, radius_wl=3.0, freq=400e6):
    lam = si.C0 / freq
    tx = si.antenna_positions(n_tx, radius_wl * lam)
    rx = si.antenna_positions(n_rx, radius_wl * lam)
    return tx, rx


def make_case(M, K, n_tx, n_rx, seeds=(0,), workload="cfg1", noise=0.05, params=None, fine=2):
    """Per seed: oracle Problem, eps_true on the inversion grid, measured data."""
    wl = si.WORKLOADS[workload]
    tx, rx = geometry(n_tx, n_rx)
    k0 = ops.wavenumber(wl.freq_hz)
    cases = []
    for s in seeds:
        shapes = si.draw_profile(wl, s)
        epsf = si.rasterize(shapes, fine * M, wl.side)
        es, _ = forward.mom_solve(epsf, wl.side, k0, tx, rx)
        n1, n2 = si.draw_noise(s, es.shape)
        es = forward.add_noise(es, noise, n1, n2)
        prob = oloss.build_problem(M, K, wl.side, [wl.freq_hz], tx, rx, es, params)
        cases.append(dict(prob=prob, esca=es, eps=si.rasterize(shapes, M, wl.side), seed=s))
    return dict(wl=wl, tx=tx, rx=rx, cases=cases, M=M, K=K)


def rand_alpha(shape, scale=0.05, seed=1):
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))
