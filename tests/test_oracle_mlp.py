"""Pins of the FP64 warm-start network reference (an addition; the paper has no such network):
bfloat16 rounding against torch's conversion, GELU against torch, the hand backward against
torch float64 autograd and central differences, Adam against torch.optim.Adam."""
import numpy as np
import torch

from oracle import mlp


def make_params(sizes, seed=0):
    rng = np.random.default_rng(seed)
    return [(rng.normal(size=(o, i)) / np.sqrt(i), 0.1 * rng.normal(size=o)) for i, o in zip(sizes[:-1], sizes[1:])]


def test_bf16_round_is_torch_conversion():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-30, 30, size=4000),
                        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, 1.0 + 2.0 ** -7 + 2.0 ** -8,
                         3.0e38, -3.0e38, 1e-40, np.inf, -np.inf]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = mlp.bf16_round(x)
    assert np.array_equal(got, ref)
    # ties go to the even neighbour, values above a tie round up
    assert mlp.bf16_round(np.float32(1.0 + 2.0 ** -8)) == 1.0
    assert mlp.bf16_round(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6
    assert mlp.bf16_round(np.float32(1.0 + 2.0 ** -8 + 2.0 ** -20)) == 1.0 + 2.0 ** -7
    assert np.isnan(mlp.bf16_round(np.float32(np.nan)))


def test_gelu_and_its_derivative():
    z = np.linspace(-8, 8, 1601)
    ref = torch.nn.functional.gelu(torch.from_numpy(z)).numpy()
    assert np.max(np.abs(mlp.gelu(z) - ref)) < 1e-15
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(mlp.gelu_grad(z) - fd)) < 1e-8
    assert mlp.gelu(0.0) == 0.0 and abs(mlp.gelu_grad(0.0) - 0.5) < 1e-15


def test_backward_matches_torch_autograd():
    sizes = [12, 9, 7, 8, 10]
    params = make_params(sizes)
    rng = np.random.default_rng(2)
    x, t = rng.normal(size=(5, 12)), rng.normal(size=(5, 10))
    y, cache = mlp.forward(params, x, s_in=0.7)
    loss, dy = mlp.mse(y, t)
    grads = mlp.backward(params, cache, dy)
    tp = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in params]
    h = 0.7 * torch.from_numpy(x)
    for l, (W, b) in enumerate(tp):
        h = h @ W.T + b
        if l < len(tp) - 1:
            h = torch.nn.functional.gelu(h)
    tl = torch.mean((h - torch.from_numpy(t)) ** 2)
    tl.backward()
    assert abs(loss - tl.item()) < 1e-14 * max(1.0, abs(loss))
    assert np.max(np.abs(y - h.detach().numpy())) < 1e-13
    for (gW, gb), (W, b) in zip(grads, tp):
        assert np.max(np.abs(gW - W.grad.numpy())) < 1e-13
        assert np.max(np.abs(gb - b.grad.numpy())) < 1e-13


def test_backward_central_differences():
    sizes = [6, 5, 5, 4]
    params = make_params(sizes, seed=3)
    rng = np.random.default_rng(4)
    x, t = rng.normal(size=(3, 6)), rng.normal(size=(3, 4))

    def f(ps):
        return mlp.mse(mlp.forward(ps, x)[0], t)[0]

    y, cache = mlp.forward(params, x)
    grads = mlp.backward(params, cache, mlp.mse(y, t)[1])
    h = 1e-6
    for l in range(len(params)):
        for (i, j) in [(0, 0), (1, 2), (params[l][0].shape[0] - 1, params[l][0].shape[1] - 1)]:
            Wp = [(W.copy(), b.copy()) for W, b in params]
            Wm = [(W.copy(), b.copy()) for W, b in params]
            Wp[l][0][i, j] += h
            Wm[l][0][i, j] -= h
            fd = (f(Wp) - f(Wm)) / (2 * h)
            assert abs(fd - grads[l][0][i, j]) < 1e-8 * max(1.0, abs(fd)), (l, i, j)
        Bp = [(W.copy(), b.copy()) for W, b in params]
        Bm = [(W.copy(), b.copy()) for W, b in params]
        Bp[l][1][1] += h
        Bm[l][1][1] -= h
        assert abs((f(Bp) - f(Bm)) / (2 * h) - grads[l][1][1]) < 1e-8


def test_quantised_network_stays_within_bf16_bound():
    sizes = [64, 48, 48, 32]
    params = make_params(sizes, seed=5)
    x = np.random.default_rng(6).normal(size=(8, 64))
    y, _ = mlp.forward(params, x)
    yq, _ = mlp.forward(params, x, quant=True)
    # each rounding is within 2^-9 relative; three layers of length <= 64 sums
    assert np.linalg.norm(yq - y) / np.linalg.norm(y) < 2e-2
    assert np.linalg.norm(yq - y) > 0


def test_adam_update_is_torch_adam():
    rng = np.random.default_rng(7)
    w = rng.normal(size=20)
    tw = torch.tensor(w.copy(), requires_grad=True)
    opt = torch.optim.Adam([tw], lr=3e-3)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for t in range(1, 6):
        g = rng.normal(size=20)
        w, m, v = mlp.adam_update(w, g, m, v, t, 3e-3)
        opt.zero_grad()
        tw.grad = torch.from_numpy(g.copy())
        opt.step()
    assert np.max(np.abs(w - tw.detach().numpy())) < 1e-15


def test_training_fits_a_linear_map():
    rng = np.random.default_rng(8)
    sizes = [8, 16, 16, 4]
    params = make_params(sizes, seed=9)
    state = [(np.zeros_like(W), np.zeros_like(W), np.zeros_like(b), np.zeros_like(b)) for W, b in params]
    A = rng.normal(size=(4, 8))
    x = rng.normal(size=(64, 8))
    t = x @ A.T
    first = None
    for step in range(1, 301):
        params, state, loss = mlp.train_step(params, state, x, t, step, 1e-2)
        first = loss if first is None else first
    assert loss < 0.05 * first
