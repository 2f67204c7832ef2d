"""Pins of the loss evaluated on the CCO image (the cco_in_loss option; Sec. 2.4, Eqs. 10-11
inside the loss of Sec. 3.2, Eqs. 13-19).

The option replaces chi by chi_c = CCO(chi) in every chi-dependent term: the regularisers are
evaluated on chi_c and the state residual takes R_c = beta chi_c / (1 + beta chi_c).  Pinned by
central finite differences of the CCO's vector-Jacobian product and of the whole loss, by torch
float64 autograd of a forward written with torch's own windowed mean (average pooling that
excludes the padding), by the transpose identity of the box mean, by the closed form of the state
term (L_State(R_c) = L_State(R) + sum den |R_c - R|^2 / ||E_inc||^2, R being the per-pixel
least-squares optimum), and by the reduction to the plain loss when the CCO is the identity.
"""
import dataclasses

import numpy as np
import torch

from oracle import cco, fourier, loss
from test_oracle_loss import _torch_loss, rand_alpha, small_problem


def cco_params(**kw):
    return loss.Params(cco_in_loss=True, **kw)


def test_box_mean_transpose():
    rng = np.random.default_rng(3)
    for shape, r in (((7, 5), 1), ((9, 9), 2), ((4, 6), 1)):
        x, y = rng.standard_normal(shape), rng.standard_normal(shape)
        assert abs(np.sum(cco.box_mean(x, r) * y) - np.sum(x * cco.box_mean_t(y, r))) < 1e-13


def test_cco_vjp_central_fd():
    rng = np.random.default_rng(1)
    # moduli around tau = 3, where eta(|chi|) changes fastest
    chi = 3.0 + 0.8 * rng.standard_normal((7, 6)) + 1j * 0.8 * rng.standard_normal((7, 6))
    g = rng.standard_normal((7, 6)) + 1j * rng.standard_normal((7, 6))
    gv = cco.cco_vjp(chi, g)

    def f(c):
        return np.sum(np.real(np.conj(g) * cco.cco(c)))
    h = 1e-6
    for (i, j) in ((0, 0), (3, 2), (6, 5), (2, 5), (6, 0)):
        for d in (1.0, 1j):
            e = np.zeros_like(chi)
            e[i, j] = h * d
            fd = (f(chi + e) - f(chi - e)) / (2 * h)
            an = np.real(np.conj(gv[i, j]) * d)
            assert abs(fd - an) < 1e-7 * max(1.0, abs(an)), (i, j, d, fd, an)


def test_cco_in_loss_gradient_central_fd():
    prob = small_problem(params=cco_params())
    a = rand_alpha(prob, seed=3)
    out = loss.evaluate(a, prob)
    g = out["g_alpha"]
    assert np.max(np.abs(out["chi_c"] - out["chi"])) > 1e-3  # the CCO does change the image
    rng = np.random.default_rng(11)
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


def _torch_cco(chi, p):
    """CCO of Eqs. 10-11 with torch's average pooling (padding excluded from the count) as the
    window mean of the self-guided filter."""
    def mean(x):
        k = 2 * p.gf_radius + 1
        return torch.nn.functional.avg_pool2d(x[None, None], k, stride=1, padding=p.gf_radius,
                                              count_include_pad=False)[0, 0]

    def guided(x):
        mu = mean(x)
        var = mean(x * x) - mu * mu
        A = var / (var + p.gf_eps)
        return mean(A) * x + mean((1 - A) * mu)
    G = torch.complex(guided(chi.real), guided(chi.imag))
    eta = p.cco_eta_max * torch.sigmoid((chi.abs() - p.cco_tau) / p.cco_delta)
    return (1 + eta) * G + eta * chi


def test_cco_in_loss_matches_torch_autograd():
    prob = small_problem(n_tx=5, params=cco_params())
    a = rand_alpha(prob, seed=4)
    out = loss.evaluate(a, prob)
    p = prob.params

    def torch_loss_cco(at):
        # Eqs. 6-7, 9, 13-19 with chi -> CCO(chi) and R -> R_c in the chi-dependent terms
        M, K = prob.M, prob.K
        k = torch.tensor(fourier.modes(K), dtype=torch.float64)
        i = torch.arange(M, dtype=torch.float64)
        Ey = torch.exp(2j * torch.pi * i[:, None] * k[None, :] / M)
        J = Ey @ at @ Ey.T
        P = 2 * M
        pad = torch.zeros((at.shape[0], P, P), dtype=torch.complex128)
        pad[:, :M, :M] = J
        GJ = torch.fft.ifft2(torch.fft.fft2(pad) * torch.from_numpy(prob.ghat[0]))[:, :M, :M]
        einc = torch.from_numpy(prob.einc[0]).reshape(-1, M, M)
        E = einc + GJ + p.beta * J
        R = p.beta * (J * E.conj()).sum(0) / (E.abs() ** 2).sum(0)
        chi_c = _torch_cco(R / (p.beta * (1 - R)), p)
        R_c = p.beta * chi_c / (1 + p.beta * chi_c)
        Ls = ((R_c * E - p.beta * J).abs() ** 2).sum() / (einc.abs() ** 2).sum()
        D = J.reshape(J.shape[0], -1) @ torch.from_numpy(prob.gs[0]).T
        es = torch.from_numpy(prob.esca[0])
        Ld = ((D - es).abs() ** 2).sum() / (es.abs() ** 2).sum()
        Lb = (torch.relu(-chi_c.real) ** 2).sum()

        def dx(z):
            return torch.nn.functional.pad(z[:, 1:] - z[:, :-1], (0, 1))

        def dy(z):
            return torch.nn.functional.pad((z[1:, :] - z[:-1, :]).T, (0, 1)).T
        Lt = torch.sqrt(dx(chi_c).abs() ** 2 + dy(chi_c).abs() ** 2 + p.eps_tv).sum()
        am = torch.sqrt(chi_c.abs() ** 2 + p.eps_abs)
        Lr = (torch.sigmoid((am - p.tau_b) / p.tau_b) * torch.exp(-dx(am) ** 2 - dy(am) ** 2)).sum()
        return Ls + Ld + p.lam_bound * Lb + p.lam_tv * Lt + p.lam_bridge * Lr

    at = torch.tensor(a, requires_grad=True)
    L = torch_loss_cco(at)
    L.backward()
    assert abs(L.item() - out["L"]) < 1e-12 * out["L"]
    g = at.grad.numpy()
    assert np.max(np.abs(g - out["g_alpha"])) < 1e-10 * np.max(np.abs(g))
    # and the same forward without the CCO is the plain loss
    plain = loss.evaluate(a, dataclasses.replace(prob, params=dataclasses.replace(p, cco_in_loss=False)))
    assert abs(_torch_loss(torch.tensor(a), prob).item() - plain["L"]) < 1e-12 * plain["L"]


def test_cco_in_loss_state_term_closed_form():
    prob = small_problem(params=cco_params())
    a = rand_alpha(prob, seed=5)
    on = loss.evaluate(a, prob, grad=False)
    off = loss.evaluate(a, dataclasses.replace(prob, params=dataclasses.replace(prob.params, cco_in_loss=False)),
                        grad=False)
    e2 = np.sum(np.abs(on["E"][0]) ** 2, axis=0)  # sum over incidences of |E|^2, per pixel
    extra = np.sum(e2 * np.abs(on["R_c"] - on["R"]) ** 2) / prob.S_s[0]
    assert abs(on["L_state"] - (off["L_state"] + extra)) < 1e-12 * on["L_state"]
    assert extra > 1e-6 * on["L_state"]
    # the data term does not see the CCO
    assert on["L_data"] == off["L_data"]


def test_cco_in_loss_with_an_identity_cco_is_the_plain_loss():
    # eta_max = 0 and a vanishing filter regulariser: G(p) -> p, so chi_c -> chi and R_c -> R
    ident = cco_params(cco_eta_max=0.0, gf_eps=1e-13)
    prob = small_problem(params=ident)
    a = rand_alpha(prob, seed=6)
    on = loss.evaluate(a, prob)
    off = loss.evaluate(a, dataclasses.replace(prob, params=dataclasses.replace(ident, cco_in_loss=False)))
    assert np.max(np.abs(on["chi_c"] - on["chi"])) < 1e-9 * np.max(np.abs(on["chi"]))
    assert abs(on["L"] - off["L"]) < 1e-9 * off["L"]
    assert np.max(np.abs(on["g_alpha"] - off["g_alpha"])) < 1e-7 * np.max(np.abs(off["g_alpha"]))
