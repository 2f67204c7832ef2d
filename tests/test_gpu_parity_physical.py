"""FP32 parity on physical inputs held to a flat 1e-4: measured fields from the FP64 MoM of
random cfg2-style profiles (eps_r in [2, 4], jitter, 10 % noise), at the start value and along the
solver's own trajectory (after 10 and 100 steps of the coefficient network of Sec. 3.1 and after
10 direct Adam steps), on the benchmark grid (64^2, 32/32, K = 15), on 48^2 (radix-3 passes) and on
96^2.  At each point the device's alpha is taken as the input of both sides; every loss term
(Eqs. 15-19) and every gradient entry must be within 1e-4 of the oracle (terms relative to
themselves, with an absolute floor of 1e-8 of the total for terms that vanish; gradient entries
relative to the largest).  The conditioning of chi(R) (Eq. 7) stays small on these inputs, which
is printed."""
import dataclasses

import numpy as np
import pytest
import torch

import seeded_inputs as si
from oracle import forward, init as oinit, loss as oloss, operators as ops
from tests.test_gpu_parity import DEV, chi_condition, oracle_terms

pytestmark = pytest.mark.gpu

pdf = pytest.importorskip("paper_2602_13805_amd")

H = 64


def _case(M, n_ant, K, seeds):
    wl = dataclasses.replace(si.WORKLOADS["cfg2"], M=M, n_tx=n_ant, n_rx=n_ant, K=K, M_fine=2 * M)
    tx = si.antenna_positions(n_ant, wl.radius)
    rx = si.antenna_positions(n_ant, wl.radius)
    es, probs = [], []
    for sd in seeds:
        jt, jr = si.draw_jitter(sd, n_ant, n_ant, wl.jitter_deg)
        e, _ = forward.mom_solve(si.rasterize(si.draw_profile(wl, sd), 2 * M, wl.side), wl.side,
                                 ops.wavenumber(wl.freq_hz), si.antenna_positions(n_ant, wl.radius, angle_offsets=jt),
                                 si.antenna_positions(n_ant, wl.radius, angle_offsets=jr))
        e = forward.add_noise(e, wl.noise, *si.draw_noise(sd, e.shape))
        es.append(e)
        probs.append(oloss.build_problem(M, K, wl.side, [wl.freq_hz], tx, rx, e))
    s = pdf.Solver(M, wl.side, wl.freq_hz, tx, rx, K, batch=len(seeds), device=DEV)
    s.set_data(torch.tensor(np.stack(es), dtype=s.cdtype, device=DEV))
    return s, probs


def _check_at(s, probs, alpha, label):
    loss, g = s.loss_grad(alpha.contiguous())
    loss, g = loss.cpu().numpy(), g.cpu().numpy()
    a = alpha.cpu().numpy().astype(np.complex128)
    for b, prob in enumerate(probs):
        ref = oloss.evaluate(a[b], prob)
        want, got = oracle_terms(ref), loss[b, :6]
        err_t = np.abs(got - want) / np.maximum(np.abs(want), 1e-8 * abs(want[5]))
        gr = ref["g_alpha"]
        err_g = np.max(np.abs(g[b] - gr)) / np.max(np.abs(gr))
        print(f"  {label} b={b}: kappa {chi_condition(ref):.1f}, terms {np.array2string(err_t, precision=1)}, "
              f"gradient {err_g:.1e}", flush=True)
        assert np.all(err_t <= 1e-4), (label, b, err_t)
        assert err_g <= 1e-4, (label, b, err_g)


@pytest.mark.parametrize("M,n_ant,K,B", [(64, 32, 15, 2), (48, 24, 13, 2), (96, 16, 21, 1)])
def test_fp32_parity_along_the_trajectory(M, n_ant, K, B):
    print(f"case physical M={M} Ni=Ns={n_ant} K={K} B={B}", flush=True)
    s, probs = _case(M, n_ant, K, tuple(range(B)))
    a0 = s.init_alpha()
    _check_at(s, probs, a0, "start")
    # the solver of Sec. 3.1: network steps from the start
    sc = dict(s_in=1.0 / float(np.sqrt(pdf.mean_abs2(a0))), s_out=1.0 / H)
    theta = torch.tensor(si.fcnn_theta(1, B, K, H, out_scale=0.0), dtype=s.rdtype, device=DEV)
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    for t in range(1, 101):
        s.fcnn_step(H, a0, theta, m, v, t, **sc)
        if t in (10, 100):
            _check_at(s, probs, s.fcnn_forward(H, a0, theta, **sc), f"network step {t}")
    # direct Adam on alpha
    a = a0.clone()
    mm, vv, tt = s.new_state()
    for _ in range(10):
        s.step(a, mm, vv, tt)
    _check_at(s, probs, a, "direct step 10")
    s.close()


def test_fp32_gradient_by_finite_differences_at_steps_0_500_1000():
    """The benchmark configuration's gradient check: along 1000 steps of the solver (Sec. 3.1 network)
    on one cfg2 instance, the device's FP32 gradient at steps 0, 500 and 1000 against central
    differences of the FP64 oracle's loss at the same alpha, on 64 random real coordinates (Re or Im
    of a coefficient); step 1e-5 times the largest |alpha|, within 1e-4 of the largest gradient
    entry."""
    print("case cfg2 finite differences at steps 0, 500, 1000", flush=True)
    s, probs = _case(64, 32, 15, (5,))
    prob = probs[0]
    a0 = s.init_alpha()
    sc = dict(s_in=1.0 / float(np.sqrt(pdf.mean_abs2(a0))), s_out=1.0 / H)
    theta = torch.tensor(si.fcnn_theta(1, 1, 15, H, out_scale=0.0), dtype=s.rdtype, device=DEV)
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    rng = np.random.default_rng(7)
    for t in range(0, 1001):
        if t > 0:
            s.fcnn_step(H, a0, theta, m, v, t, **sc)
        if t not in (0, 500, 1000):
            continue
        ah = s.fcnn_forward(H, a0, theta, **sc)
        _, g = s.loss_grad(ah)
        g = g.cpu().numpy()[0]
        a = ah.cpu().numpy().astype(np.complex128)[0]
        h = 1e-5 * np.max(np.abs(a))
        worst = 0.0
        for _ in range(64):
            idx = tuple(int(rng.integers(0, n)) for n in a.shape)
            d = 1.0 if rng.random() < 0.5 else 1j
            ap, am = a.copy(), a.copy()
            ap[idx] += h * d
            am[idx] -= h * d
            fd = (oloss.loss_total(ap[None], prob) - oloss.loss_total(am[None], prob)) / (2 * h)
            an = g[idx].real if d == 1.0 else g[idx].imag
            worst = max(worst, abs(fd - an) / np.max(np.abs(g)))
        print(f"  step {t}: max |FD - device| / max |g| = {worst:.1e}", flush=True)
        assert worst <= 1e-4, (t, worst)
    s.close()
