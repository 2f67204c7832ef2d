"""Pins of the composite loss and its hand adjoint (Sec. 3.2, Eqs. 13-19).

The loss is pinned by its zero at the true currents (inverse-crime setting),
by hand-computed regulariser values, by the paper's printed constants and by
ablation / frequency reductions; the gradient by central finite differences,
by torch float64 autograd of an independently written forward, by the
variable-projection identity and by adjoint dot products.
"""
import json
import os

import numpy as np
import pytest
import torch

import seeded_inputs as si
from oracle import fourier, forward, loss, operators as ops

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
WL = si.WORKLOADS["cfg1"]
LAM = WL.wavelength
K0 = ops.wavenumber(WL.freq_hz)


def small_problem(M=16, K=7, n_tx=6, n_rx=8, seed=0, noise=0.05, params=None, eps_fine=None):
    tx = si.antenna_positions(n_tx, WL.radius)
    rx = si.antenna_positions(n_rx, WL.radius)
    shapes = si.draw_profile(WL, seed)
    epsf = si.rasterize(shapes, 2 * M, WL.side) if eps_fine is None else eps_fine
    es, _ = forward.mom_solve(epsf, WL.side, K0, tx, rx)
    n1, n2 = si.draw_noise(seed, es.shape)
    es = forward.add_noise(es, noise, n1, n2)
    return loss.build_problem(M, K, WL.side, [WL.freq_hz], tx, rx, es, params)


def rand_alpha(prob, scale=0.05, seed=1):
    rng = np.random.default_rng(seed)
    shp = (prob.Ni, prob.K, prob.K)
    return scale * (rng.standard_normal(shp) + 1j * rng.standard_normal(shp))


def test_default_constants_are_the_papers():
    p = loss.Params()
    assert p.beta == GOLD["beta"]["value"]
    assert p.lam_bound == GOLD["lam_bound"]["value"]
    assert p.lam_tv == GOLD["lam_tv"]["value"]
    assert p.lam_bridge == GOLD["lam_bridge"]["value"]
    assert p.tau_b == GOLD["tau_b"]["value"]


def test_truth_is_a_global_zero():
    # Same grid for data and inversion, full basis (even K = M: every mode),
    # no noise, no regularisers, alpha = F_T(J_true): L = 0 and grad = 0.
    M = 16
    tx = si.antenna_positions(6, WL.radius)
    rx = si.antenna_positions(8, WL.radius)
    eps = si.rasterize(si.draw_profile(WL, 5), M, WL.side)
    es, etot = forward.mom_solve(eps, WL.side, K0, tx, rx)
    prob = loss.build_problem(M, M, WL.side, [WL.freq_hz], tx, rx, es,
                              loss.Params(lam_bound=0, lam_tv=0, lam_bridge=0))
    Jt = ((eps - 1).reshape(-1)[None] * etot).reshape(-1, M, M)
    out = loss.evaluate(fourier.analyze(Jt, M), prob)
    assert out["L_state"] < 1e-24 and out["L_data"] < 1e-24
    assert np.max(np.abs(out["g_alpha"])) < 1e-11
    beta = prob.params.beta
    chi = eps - 1
    assert np.max(np.abs(out["R"] - beta * chi / (beta * chi + 1))) < 1e-12
    assert np.max(np.abs(out["chi"] - chi)) < 1e-12


def test_regularisers_constant_image():
    M, N = 5, 25
    for c in (0.7 + 0.2j, -0.3 + 0.0j, 0.0):
        chi = np.full((M, M), c, complex)
        assert abs(loss.reg_tv(chi, 1e-12)[0] - N * 1e-6) < 1e-15
        a = np.sqrt(abs(c) ** 2 + 1e-12)
        assert abs(loss.reg_bridge(chi, 0.5, 1e-12)[0] - N / (1 + np.exp(-(a - 0.5) / 0.5))) < 1e-12
        assert abs(loss.reg_bound(chi)[0] - N * max(-c.real, 0) ** 2) < 1e-15


def test_regularisers_hand_2x2():
    chi = np.array([[0.0, 1.0], [2.0, 4.0]], complex)
    e = 1e-12
    tv = np.sqrt(1 + 4 + e) + np.sqrt(9 + e) + np.sqrt(4 + e) + np.sqrt(e)
    assert abs(loss.reg_tv(chi, e)[0] - tv) < 1e-12

    def sg(x):
        return 1 / (1 + np.exp(-(x - 0.5) / 0.5))
    a = np.sqrt(np.abs(chi) ** 2 + e)
    br = sg(a[0, 0]) * np.exp(-(a[0, 1] - a[0, 0]) ** 2 - (a[1, 0] - a[0, 0]) ** 2) \
        + sg(a[0, 1]) * np.exp(-(a[1, 1] - a[0, 1]) ** 2) \
        + sg(a[1, 0]) * np.exp(-(a[1, 1] - a[1, 0]) ** 2) + sg(a[1, 1])
    assert abs(loss.reg_bridge(chi, 0.5, e)[0] - br) < 1e-12
    chi2 = np.array([[-1.0, 2.0], [-0.5 + 3j, 0.1]], complex)
    assert abs(loss.reg_bound(chi2)[0] - 1.25) < 1e-15


def test_regulariser_gradients_fd():
    rng = np.random.default_rng(0)
    chi = rng.standard_normal((6, 5)) * 0.8 + 1j * rng.standard_normal((6, 5)) * 0.3
    for fn in (lambda z: loss.reg_tv(z, 1e-12), lambda z: loss.reg_bridge(z, 0.5, 1e-12),
               loss.reg_bound):
        _, g = fn(chi)
        for idx in [(0, 0), (2, 3), (5, 4), (3, 4)]:
            for d in (1.0, 1j):
                h = 1e-7
                zp, zm = chi.copy(), chi.copy()
                zp[idx] += h * d
                zm[idx] -= h * d
                fd = (fn(zp)[0] - fn(zm)[0]) / (2 * h)
                an = g[idx].real if d == 1.0 else g[idx].imag
                assert abs(fd - an) < 1e-6 * max(1, abs(an))


def test_ablation_switches():
    prob = small_problem()
    a = rand_alpha(prob)
    full = loss.evaluate(a, prob, grad=False)
    prob.params = loss.Params(lam_bridge=0.0)
    nob = loss.evaluate(a, prob, grad=False)
    assert nob["L"] == pytest.approx(full["L"] - 1e-5 * full["L_bridge"], rel=1e-14)
    prob.params = loss.Params(lam_bound=0, lam_tv=0, lam_bridge=0)
    phys = loss.evaluate(a, prob, grad=False)
    assert phys["L"] == phys["L_state"] + phys["L_data"]


def test_gradient_central_fd():
    prob = small_problem()
    a = rand_alpha(prob)
    g = loss.evaluate(a, prob)["g_alpha"]
    rng = np.random.default_rng(9)
    for _ in range(10):
        idx = tuple(rng.integers(0, s) for s in a.shape)
        for d in (1.0, 1j):
            h = 1e-6 * 0.05
            ap, am = a.copy(), a.copy()
            ap[idx] += h * d
            am[idx] -= h * d
            fd = (loss.loss_total(ap, prob) - loss.loss_total(am, prob)) / (2 * h)
            an = g[idx].real if d == 1.0 else g[idx].imag
            assert abs(fd - an) <= 1e-6 * np.max(np.abs(g)), (idx, d, fd, an)


def _torch_loss(alpha_t, prob):
    """Independent torch float64 forward of Eqs. 6-7, 9, 13-19 for F = 1."""
    p = prob.params
    M, K = prob.M, prob.K
    k = torch.tensor(fourier.modes(K), dtype=torch.float64)
    i = torch.arange(M, dtype=torch.float64)
    Ey = torch.exp(2j * torch.pi * i[:, None] * k[None, :] / M)
    J = Ey @ alpha_t @ Ey.T
    P = 2 * M
    pad = torch.zeros((alpha_t.shape[0], P, P), dtype=torch.complex128)
    pad[:, :M, :M] = J
    GJ = torch.fft.ifft2(torch.fft.fft2(pad) * torch.from_numpy(prob.ghat[0]))[:, :M, :M]
    E = torch.from_numpy(prob.einc[0]).reshape(-1, M, M) + GJ + p.beta * J
    num = (J * E.conj()).sum(0)
    den = (E.abs() ** 2).sum(0)
    R = p.beta * num / den
    chi = R / (p.beta * (1 - R))
    s = R * E - p.beta * J
    Ls = (s.abs() ** 2).sum() / (torch.from_numpy(prob.einc[0]).abs() ** 2).sum()
    D = J.reshape(J.shape[0], -1) @ torch.from_numpy(prob.gs[0]).T
    es = torch.from_numpy(prob.esca[0])
    Ld = ((D - es).abs() ** 2).sum() / (es.abs() ** 2).sum()
    Lb = (torch.relu(-chi.real) ** 2).sum()

    def dx(z):
        return torch.nn.functional.pad(z[:, 1:] - z[:, :-1], (0, 1))

    def dy(z):
        return torch.nn.functional.pad((z[1:, :] - z[:-1, :]).T, (0, 1)).T
    Lt = torch.sqrt(dx(chi).abs() ** 2 + dy(chi).abs() ** 2 + p.eps_tv).sum()
    a = torch.sqrt(chi.abs() ** 2 + p.eps_abs)
    Lr = (torch.sigmoid((a - p.tau_b) / p.tau_b) * torch.exp(-dx(a) ** 2 - dy(a) ** 2)).sum()
    return Ls + Ld + p.lam_bound * Lb + p.lam_tv * Lt + p.lam_bridge * Lr


def test_gradient_matches_torch_autograd():
    prob = small_problem(n_tx=5)
    a = rand_alpha(prob, seed=4)
    out = loss.evaluate(a, prob)
    at = torch.tensor(a, requires_grad=True)
    L = _torch_loss(at, prob)
    L.backward()
    assert abs(L.item() - out["L"]) < 1e-12 * out["L"]
    g = at.grad.numpy()
    assert np.max(np.abs(g - out["g_alpha"])) < 1e-10 * np.max(np.abs(g))


def test_variable_projection():
    # R is the least-squares optimum, so the state loss has zero derivative in R;
    # with the regularisers off, freezing R changes nothing.
    prob = small_problem(params=loss.Params(lam_bound=0, lam_tv=0, lam_bridge=0))
    a = rand_alpha(prob, seed=2)
    full = loss.evaluate(a, prob)
    frozen = loss.evaluate(a, prob, r_stopgrad=True)
    assert np.max(np.abs(full["g_R"])) < 1e-12 * np.max(np.abs(full["num"]))
    assert np.max(np.abs(full["g_alpha"] - frozen["g_alpha"])) < 1e-10 * np.max(np.abs(full["g_alpha"]))


def test_multi_frequency_reductions():
    prob = small_problem()
    a = rand_alpha(prob)
    one = loss.evaluate(a, prob)
    dup = loss.Problem(prob.M, prob.K, np.concatenate([prob.ghat] * 2), np.concatenate([prob.gs] * 2),
                       np.concatenate([prob.einc] * 2), np.concatenate([prob.esca] * 2), prob.params)
    two = loss.evaluate(np.stack([a, a]), dup)
    assert two["L_state"] == pytest.approx(2 * one["L_state"], rel=1e-13)
    assert two["L_data"] == pytest.approx(2 * one["L_data"], rel=1e-13)
    assert np.max(np.abs(two["R"] - one["R"])) < 1e-13
    assert np.max(np.abs(two["g_alpha"][0] - two["g_alpha"][1])) < 1e-12
