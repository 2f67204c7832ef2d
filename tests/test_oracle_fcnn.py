"""Pins of the FP64 coefficient-network reference (Sec. 3.1, Fig. 4; layer sizes are a reading):
the hand backward against central differences and torch float64 autograd, the composition
with the physics loss against central differences of that loss, a torch re-implementation of
three Adam steps end to end, and the structural facts of the reading (row-wise network,
zero output layer = start coefficients)."""
import numpy as np
import torch

import seeded_inputs as si
from oracle import fcnn, loss as oloss
from tests.test_oracle_loss import _torch_loss, rand_alpha, small_problem


def _alpha(Ni, K, scale, seed):
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal((Ni, K, K)) + 1j * rng.standard_normal((Ni, K, K)))


def _torch_forward(theta_t, alpha0_t, K, H, s_in=1.0, s_out=1.0):
    """alpha_hat by torch ops, written from the layer description alone."""
    D = 2 * K * K
    off = 0
    x = alpha0_t.reshape(alpha0_t.shape[0], -1) * s_in
    z = torch.cat([x.real, x.imag], 1)
    for li, (i, o) in enumerate([(D, H), (H, H), (H, D)]):
        blk = theta_t[off:off + (i + 1) * o].reshape(i + 1, o)
        off += (i + 1) * o
        z = torch.nn.functional.linear(z, blk[:i].T.contiguous(), blk[i])
        if li < 2:
            z = torch.tanh(z)
    q = K * K
    return alpha0_t + s_out * torch.complex(z[:, :q], z[:, q:]).reshape(alpha0_t.shape)


def test_backward_matches_central_differences_of_a_linear_functional():
    K, H, Ni = 3, 5, 4
    theta = si.fcnn_theta(3, 1, K, H, out_scale=1.0)[0]
    a0 = _alpha(Ni, K, 0.7, 2)
    rng = np.random.default_rng(5)
    c = rng.standard_normal((Ni, K, K)) + 1j * rng.standard_normal((Ni, K, K))

    s_in, s_out = 3.0, 0.25

    def L(th):   # sum Re(conj(c) alpha_hat): its gradient dL/dRe + i dL/dIm is c
        return float(np.sum(np.real(np.conj(c) * fcnn.forward(th, a0, K, H, s_in, s_out)[0])))
    _, cache = fcnn.forward(theta, a0, K, H, s_in, s_out)
    g = fcnn.backward(theta, cache, c, K, H, s_out)
    assert g.shape == (fcnn.n_params(K, H),) == theta.shape
    h = 1e-6
    fd = np.empty_like(theta)
    for p in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        fd[p] = (L(tp) - L(tm)) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-7 * np.max(np.abs(g))


def test_forward_and_backward_match_torch_autograd():
    K, H, Ni = 5, 16, 6
    theta = si.fcnn_theta(4, 1, K, H, out_scale=0.5)[0]
    a0 = _alpha(Ni, K, 0.5, 3)
    rng = np.random.default_rng(6)
    c = rng.standard_normal((Ni, K, K)) + 1j * rng.standard_normal((Ni, K, K))
    for s_in, s_out in ((1.0, 1.0), (7.0, 1.0 / H)):
        ah, cache = fcnn.forward(theta, a0, K, H, s_in, s_out)
        tt = torch.tensor(theta, requires_grad=True)
        aht = _torch_forward(tt, torch.tensor(a0), K, H, s_in, s_out)
        assert np.max(np.abs(aht.detach().numpy() - ah)) < 1e-14
        (aht.conj() * torch.tensor(c)).real.sum().backward()
        g = fcnn.backward(theta, cache, c, K, H, s_out)
        assert np.max(np.abs(tt.grad.numpy() - g)) < 1e-12 * np.max(np.abs(g))


def test_composition_with_the_physics_loss_central_differences():
    prob = small_problem(M=16, K=5, n_tx=4, n_rx=6)
    K, H = prob.K, 8
    theta = si.fcnn_theta(5, 1, K, H, out_scale=0.05)[0]
    a0 = rand_alpha(prob, scale=0.05, seed=7)
    ah, cache = fcnn.forward(theta, a0, K, H)
    out = oloss.evaluate(ah, prob)
    g = fcnn.backward(theta, cache, out["g_alpha"], K, H)
    rng = np.random.default_rng(8)
    h = 1e-6
    for p in rng.choice(theta.size, 24, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        fd = (oloss.loss_total(fcnn.forward(tp, a0, K, H)[0], prob)
              - oloss.loss_total(fcnn.forward(tm, a0, K, H)[0], prob)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 * np.max(np.abs(g)), (p, fd, g[p])


def test_three_adam_steps_match_torch_end_to_end():
    """Forward by torch ops, the physics loss by an independent torch implementation,
    autograd, torch.optim.Adam (lr 1e-2): the oracle's steps give the same weights."""
    prob = small_problem(M=16, K=5, n_tx=5, n_rx=6)
    K, H = prob.K, 12
    theta = si.fcnn_theta(6, 1, K, H, out_scale=0.1)[0]
    a0 = rand_alpha(prob, scale=0.05, seed=9)
    m, v = np.zeros_like(theta), np.zeros_like(theta)
    tt = torch.tensor(theta, requires_grad=True)
    opt = torch.optim.Adam([tt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    a0t = torch.tensor(a0)
    th = theta
    for t in range(1, 4):
        th, m, v, ah, out = fcnn.step(th, m, v, t, a0, prob, K, H, s_in=20.0, s_out=1.0 / H)
        opt.zero_grad()
        L = _torch_loss(_torch_forward(tt, a0t, K, H, 20.0, 1.0 / H), prob)
        assert abs(L.item() - out["L"]) < 1e-11 * out["L"]
        L.backward()
        opt.step()
        assert np.max(np.abs(tt.detach().numpy() - th)) < 1e-11


def test_rows_are_one_network_applied_per_incidence():
    K, H, Ni = 3, 7, 5
    theta = si.fcnn_theta(7, 1, K, H, out_scale=1.0)[0]
    a0 = _alpha(Ni, K, 0.6, 4)
    perm = np.array([3, 0, 4, 1, 2])
    ah = fcnn.forward(theta, a0, K, H)[0]
    ahp = fcnn.forward(theta, a0[perm], K, H)[0]
    assert np.array_equal(ahp, ah[perm])
    one = fcnn.forward(theta, a0[2:3], K, H)[0]
    assert np.max(np.abs(one[0] - ah[2])) < 1e-14   # one row alone: BLAS may round differently


def test_zero_output_layer_starts_at_alpha0():
    """With the output block zero, alpha_hat = alpha_0 exactly, the hidden layers get no
    gradient, and the output bias gradient is the incidence sum of [Re g, Im g]."""
    K, H, Ni = 3, 6, 4
    theta = si.fcnn_theta(8, 1, K, H, out_scale=0.0)[0]
    a0 = _alpha(Ni, K, 0.6, 5)
    ah, cache = fcnn.forward(theta, a0, K, H)
    assert np.array_equal(ah, a0)
    rng = np.random.default_rng(3)
    c = rng.standard_normal((Ni, K, K)) + 1j * rng.standard_normal((Ni, K, K))
    g = fcnn.backward(theta, cache, c, K, H)
    D = 2 * K * K
    n12 = (D + 1) * H + (H + 1) * H
    assert np.all(g[:n12] == 0.0)
    gout = g[n12:].reshape(H + 1, D)
    assert np.allclose(gout[H, :K * K], c.real.sum(0).ravel(), rtol=0, atol=1e-14)
    assert np.allclose(gout[H, K * K:], c.imag.sum(0).ravel(), rtol=0, atol=1e-14)


def test_parameter_count_and_layout():
    assert fcnn.n_params(15, 256) == (450 + 1) * 256 + (256 + 1) * 256 + (256 + 1) * 450
    th = np.arange(fcnn.n_params(2, 3), dtype=float)
    (W1, b1), (W2, b2), (W3, b3) = fcnn.unpack(th, 2, 3)
    assert W1.shape == (8, 3) and b1[0] == 24 and W2[0, 0] == 27 and W3.shape == (3, 8) and b3[-1] == th[-1]
