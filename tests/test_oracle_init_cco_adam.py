"""Pins of the start value (Sec. 3.1, Eq. 12), the CCO (Sec. 2.4, Eqs. 10-11),
the image error and Adam (Sec. 3.3)."""
import json
import os

import numpy as np
import pytest
import torch

import seeded_inputs as si
from oracle import adam, cco, fourier, forward, init, loss, operators as ops, solver

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
WL = si.WORKLOADS["cfg1"]
K0 = ops.wavenumber(WL.freq_hz)


def problem(M=16, K=7, seed=0):
    tx = si.antenna_positions(6, WL.radius)
    rx = si.antenna_positions(8, WL.radius)
    shapes = si.draw_profile(WL, seed)
    es, _ = forward.mom_solve(si.rasterize(shapes, 2 * M, WL.side), WL.side, K0, tx, rx)
    return loss.build_problem(M, K, WL.side, [WL.freq_hz], tx, rx, es), shapes


def test_bp_scalar_is_least_squares():
    prob, _ = problem()
    e = prob.esca[0][2]
    u = np.conj(prob.gs[0]).T @ e
    v = prob.gs[0] @ u
    gamma = np.vdot(v, e) / np.vdot(v, v)
    f0 = np.linalg.norm(gamma * v - e)
    for dr in np.linspace(-0.2, 0.2, 9):
        for di in np.linspace(-0.2, 0.2, 9):
            g = gamma * (1 + dr + 1j * di)
            assert np.linalg.norm(g * v - e) >= f0 - 1e-15


def test_ls_contrast_recovers_a_known_contrast():
    # currents J = chi E_tot of a lossy profile solved on the inversion grid itself: E_inc + G_D J
    # is then E_tot (the state equation, Eq. 3), and the per-pixel least squares over the
    # incidences must return chi exactly (a complex chi, so a conjugate on the wrong factor fails)
    M = 16
    prob, shapes = problem(M=M, K=7, seed=3)
    eps = 1.0 + (si.rasterize(shapes, M, WL.side) - 1.0) * (1.0 + 0.4j)
    tx = si.antenna_positions(6, WL.radius)
    rx = si.antenna_positions(8, WL.radius)
    _, etot = forward.mom_solve(eps, WL.side, K0, tx, rx)
    chi = (eps - 1.0).reshape(-1)
    J = (chi[None, :] * etot).reshape(1, 6, M, M)
    chi0, R0 = init.ls_contrast(prob, J)
    support = np.abs(chi) > 0
    assert support.sum() > 10
    assert np.max(np.abs(chi0.reshape(-1) - chi)) < 1e-9 * np.max(np.abs(chi))
    beta = prob.params.beta
    assert np.max(np.abs(R0 - beta * chi0 / (beta * chi0 + 1.0))) < 1e-15
    # Eq. 6-7: R_0 is the contraction of the CIE, beta J = R (E + beta J) pixel by pixel
    Ecie = etot.reshape(1, 6, M, M) + beta * J
    assert np.max(np.abs(beta * J - R0[None, None] * Ecie)) < 1e-9 * np.max(np.abs(beta * J))


def test_bp_currents_are_the_best_scaled_back_projection():
    prob, _ = problem(seed=1)
    J = init.bp_currents(prob)[0]
    for p in range(prob.Ni):
        e = prob.esca[0][p]
        u = (np.conj(prob.gs[0]).T @ e)
        j = J[p].reshape(-1)
        # parallel to G_S^H e_p
        assert abs(abs(np.vdot(u, j)) - np.linalg.norm(u) * np.linalg.norm(j)) < 1e-12 * np.linalg.norm(u) * \
            np.linalg.norm(j)
        # and the scale that fits the data best (scan of complex factors)
        f0 = np.linalg.norm(prob.gs[0] @ j - e)
        for dr in np.linspace(-0.3, 0.3, 7):
            for di in np.linspace(-0.3, 0.3, 7):
                assert np.linalg.norm(prob.gs[0] @ (j * (1 + dr + 1j * di)) - e) >= f0 - 1e-14


def test_alpha0_is_exact_line_search_of_csi():
    prob, _ = problem()
    a0, info = init.alpha0(prob)
    R0, g, t = info["R0"], info["g"], info["t"]
    f = lambda tt: init.csi_loss(prob, R0, -tt * g)
    ft = f(t)
    for s in np.linspace(0.0, 3.0 * t, 61):
        assert ft <= f(s) + 1e-13
    assert ft < f(0.0)


def test_csi_gradient_fd():
    prob, _ = problem()
    _, info = init.alpha0(prob)
    R0, g = info["R0"], info["g"]
    z = np.zeros_like(g)
    rng = np.random.default_rng(0)
    for _ in range(6):
        idx = tuple(rng.integers(0, s) for s in g.shape)
        for d in (1.0, 1j):
            h = 1e-6
            zp, zm = z.copy(), z.copy()
            zp[idx] += h * d
            zm[idx] -= h * d
            fd = (init.csi_loss(prob, R0, zp) - init.csi_loss(prob, R0, zm)) / (2 * h)
            an = g[idx].real if d == 1.0 else g[idx].imag
            assert abs(fd - an) < 1e-6 * np.max(np.abs(g))


def test_cco_constants_are_the_papers():
    import inspect
    sig = inspect.signature(cco.cco)
    assert sig.parameters["tau"].default == GOLD["cco_tau"]["value"]
    assert sig.parameters["eta_max"].default == GOLD["cco_eta_max"]["value"]
    assert sig.parameters["delta"].default == GOLD["cco_delta"]["value"]


def test_cco_special_cases():
    c = 1.3 + 0.4j
    chi = np.full((6, 7), c)
    assert np.allclose(cco.guided_self(chi.real), c.real, rtol=0, atol=1e-15)
    eta = 0.1 / (1 + np.exp(-(abs(c) - 3) / 0.5))
    assert np.allclose(cco.cco(chi), (1 + 2 * eta) * c, rtol=1e-14)
    # eta at |chi| = tau is exactly eta_max / 2
    chi3 = np.full((3, 3), 3.0 + 0j)
    assert np.allclose(cco.cco(chi3), 3.0 * (1 + 2 * 0.05), rtol=1e-15)
    rng = np.random.default_rng(0)
    p = rng.standard_normal((8, 9))
    # eps -> 0: the filter is the identity (where windows are not constant)
    assert np.max(np.abs(cco.guided_self(p, 1, 1e-14) - p)) < 1e-9
    # eps -> infinity: the filter is a box mean of the box mean
    assert np.max(np.abs(cco.guided_self(p, 1, 1e14) - cco.box_mean(cco.box_mean(p, 1), 1))) < 1e-12
    # count-normalised box mean at a corner: mean of the 2 x 2 in-grid window
    assert abs(cco.box_mean(p, 1)[0, 0] - p[:2, :2].mean()) < 1e-15
    # with G = identity the peak |chi| never decreases
    z = rng.standard_normal((8, 8)) * 2 + 1j * rng.standard_normal((8, 8))
    eta = 0.1 / (1 + np.exp(-(np.abs(z) - 3) / 0.5))
    assert np.max(np.abs((1 + 2 * eta) * z)) >= np.max(np.abs(z))


def test_image_error_zero_at_truth():
    eps = si.rasterize(si.draw_profile(WL, 1), 16, WL.side)
    assert cco.image_error(eps - 1.0, eps) == 0.0


def test_adam_first_step_and_torch():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((3, 5, 5)) + 1j * rng.standard_normal((3, 5, 5))
    m = np.zeros(a.shape + (2,))
    v = np.zeros(a.shape + (2,))
    g = rng.standard_normal(a.shape) + 1j * rng.standard_normal(a.shape)
    a1, m1, v1 = adam.adam_step(a, g, m, v, 1)
    ref = a - 1e-2 * (g.real / (np.abs(g.real) + 1e-8) + 1j * g.imag / (np.abs(g.imag) + 1e-8))
    assert np.max(np.abs(a1 - ref)) < 1e-15
    # multi-step sequence against torch.optim.Adam on view_as_real(alpha)
    p = torch.tensor(a.copy())
    p.requires_grad_(True)
    opt = torch.optim.Adam([p], lr=GOLD["adam_lr"]["value"])
    x, mm, vv = a.copy(), m, v
    for t in range(1, 8):
        gt = rng.standard_normal(a.shape) + 1j * rng.standard_normal(a.shape)
        opt.zero_grad()
        p.grad = torch.tensor(gt)
        opt.step()
        x, mm, vv = adam.adam_step(x, gt, mm, vv, t)
    assert np.max(np.abs(p.detach().numpy() - x)) < 1e-14


@pytest.mark.slow
def test_reconstruction_improves_on_the_start():
    prob, shapes = problem(M=16, K=7, seed=2)
    et = si.rasterize(shapes, 16, WL.side)
    a0, info = init.alpha0(prob)
    res = solver.reconstruct(prob, 60, a0, eps_true=et)
    start = cco.image_error(cco.cco(loss.evaluate(a0, prob, grad=False)["chi"]), et)
    assert res["loss"][-1] < res["loss"][0]
    assert res["err"] < start


def test_csi_gradient_at_any_alpha_fd():
    prob, _ = problem()
    _, info = init.alpha0(prob)
    R0 = info["R0"]
    rng = np.random.default_rng(3)
    a = 0.05 * (rng.standard_normal(info["g"].shape) + 1j * rng.standard_normal(info["g"].shape))
    g = init.csi_gradient(prob, R0, a)
    assert np.max(np.abs(init.csi_gradient(prob, R0, np.zeros_like(a)) - info["g"])) < 1e-13 * np.max(np.abs(g))
    for _ in range(8):
        idx = tuple(rng.integers(0, s) for s in a.shape)
        for d in (1.0, 1j):
            h = 1e-6
            ap, am = a.copy(), a.copy()
            ap[idx] += h * d
            am[idx] -= h * d
            fd = (init.csi_loss(prob, R0, ap) - init.csi_loss(prob, R0, am)) / (2 * h)
            an = g[idx].real if d == 1.0 else g[idx].imag
            assert abs(fd - an) < 1e-6 * np.max(np.abs(g))


def test_csi_cg_reaches_the_least_squares_minimiser():
    """On a tiny case (36 real unknowns) CG ends at the minimiser of the quadratic, found here
    independently by numpy's least squares on the explicit real matrix of the affine map
    alpha -> weighted residuals; one CG step is the one-step start; the loss never increases."""
    tx = si.antenna_positions(2, WL.radius)
    rx = si.antenna_positions(3, WL.radius)
    es, _ = forward.mom_solve(si.rasterize(si.draw_profile(WL, 1), 16, WL.side), WL.side, K0, tx, rx)
    prob = loss.build_problem(8, 3, WL.side, [WL.freq_hz], tx, rx, es)
    _, R0, _ = init.bp_contrast(prob)
    shape = (1, prob.Ni, 3, 3)
    n = 2 * int(np.prod(shape))

    def resid(alpha):   # weighted residual vector whose squared norm is L^CSI
        M, beta = prob.M, prob.params.beta
        J = fourier.synthesize(alpha[0], M)
        D = J.reshape(prob.Ni, M * M) @ prob.gs[0].T - prob.esca[0]
        s = R0[None] * (prob.einc[0].reshape(prob.Ni, M, M) + ops.gd_apply(J, prob.ghat[0]) + beta * J) - beta * J
        r = np.concatenate([D.ravel() / np.sqrt(prob.S_d[0]), s.ravel() / np.sqrt(prob.S_s[0])])
        return np.concatenate([r.real, r.imag])

    def unflat(x):
        return (x[:n // 2] + 1j * x[n // 2:]).reshape(shape)
    b = resid(np.zeros(shape, np.complex128))
    A = np.stack([resid(unflat(np.eye(n)[i])) - b for i in range(n)], axis=1)
    x, *_ = np.linalg.lstsq(A, -b, rcond=None)
    a_ls = unflat(x)
    L_ls = init.csi_loss(prob, R0, a_ls)
    a_cg, info = init.csi_cg(prob, 60)
    assert abs(info["losses"][-1] - L_ls) < 1e-10 * L_ls
    assert np.max(np.abs(a_cg - a_ls)) < 1e-6 * np.max(np.abs(a_ls))
    assert all(l1 <= l0 * (1 + 1e-12) for l0, l1 in zip(info["losses"], info["losses"][1:]))
    a1, _ = init.csi_cg(prob, 1)
    assert np.max(np.abs(a1 - init.alpha0(prob)[0])) < 1e-14 * np.max(np.abs(a1))
    # what defines CG: after k steps the loss is the minimum over the Krylov subspace
    # span{g0, N g0, ..., N^(k-1) g0}, N = A^T A, g0 = A^T b (steepest descent misses it from k = 2)
    N, g0 = A.T @ A, A.T @ b
    for k in (2, 3, 5):
        V = np.linalg.qr(np.stack([np.linalg.matrix_power(N, j) @ g0 for j in range(k)], axis=1))[0]
        y, *_ = np.linalg.lstsq(A @ V, -b, rcond=None)
        L_kry = float(np.sum((A @ (V @ y) + b) ** 2))
        L_cg = init.csi_cg(prob, k)[1]["losses"][-1]
        assert abs(L_cg - L_kry) < 1e-8 * L_kry, (k, L_cg, L_kry)
