"""The paper's convergence claim as a property of the oracle at the benchmark size (Sec. 4.1: the
reconstructed image improves with the iteration count, and the solver ends better than its
start).  It is stated for the solver of Sec. 3.1, Adam on the weights of the untrained network
that maps alpha_0 to a correction; 64x64 grid, 32/32 antennas, K = 15, eps_r in [2, 4], 10 %
noise, jittered antennas, FP64.  Parity is unpinned by the paper for individual trajectories
(it prints none), so the property is checked on the mean over seeds."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import cco, fcnn, forward, init, loss, operators as ops

WL = si.WORKLOADS["cfg2"]
H = 256


def _instance(seed):
    shapes = si.draw_profile(WL, seed)
    jt, jr = si.draw_jitter(seed, WL.n_tx, WL.n_rx, WL.jitter_deg)
    txj = si.antenna_positions(WL.n_tx, WL.radius, angle_offsets=jt)
    rxj = si.antenna_positions(WL.n_rx, WL.radius, angle_offsets=jr)
    es, _ = forward.mom_solve(si.rasterize(shapes, WL.M_fine, WL.side), WL.side, ops.wavenumber(WL.freq_hz),
                              txj, rxj)
    n1, n2 = si.draw_noise(seed, es.shape)
    es = si.add_noise(es, WL.noise, n1, n2)
    tx = si.antenna_positions(WL.n_tx, WL.radius)
    rx = si.antenna_positions(WL.n_rx, WL.radius)
    prob = loss.build_problem(WL.M, WL.K, WL.side, [WL.freq_hz], tx, rx, es)
    return prob, si.rasterize(shapes, WL.M, WL.side)


def _err(prob, a, et):
    return cco.image_error(cco.cco(loss.evaluate(a[None], prob, grad=False)["chi"]), et)


@pytest.mark.slow
def test_network_solver_image_improves_with_iterations_at_benchmark_size():
    start, at10, at100 = [], [], []
    for seed in range(4):
        prob, et = _instance(seed)
        a0 = init.alpha0(prob)[0][0]
        theta = si.fcnn_theta(1, 1, WL.K, H)[0]
        m, v = np.zeros_like(theta), np.zeros_like(theta)
        s_in, s_out = 1.0 / np.sqrt(np.mean(np.abs(a0) ** 2)), 1.0 / H
        start.append(_err(prob, a0, et))
        for t in range(1, 101):
            theta, m, v, _, out = fcnn.step(theta, m, v, t, a0, prob, WL.K, H, s_in=s_in, s_out=s_out)
            if t in (10, 100):
                ah, _ = fcnn.forward(theta, a0, WL.K, H, s_in, s_out)
                (at10 if t == 10 else at100).append(_err(prob, ah, et))
        print(f"seed {seed}: start {start[-1]:.3f}, k=10 {at10[-1]:.3f}, k=100 {at100[-1]:.3f}", flush=True)
    assert np.mean(at100) < np.mean(at10)
    assert np.mean(at100) < np.mean(start)
