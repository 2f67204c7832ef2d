"""GPU parity of the warm-start network (an addition; the paper has none), of the Fourier
analysis used for its targets, and of the start selection.  The network is held to the plain FP64
oracle (oracle.mlp, quant=False) within a first-order bound derived from bfloat16's unit
round-off and the layer products (test_bf16_network_within_the_rounding_bound_of_fp64); a second
test checks where the device rounds, against the oracle evaluated with the same rounding points
(quant=True)."""
import numpy as np
import pytest
import torch

import paper_2602_13805_amd as pdf
from oracle import fourier, mlp as omlp
from tests.common import make_case, rel

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def host_params(net):
    return [tuple(np.asarray(a, np.float64) for a in net.get_layer(l)) for l in range(net.L)]


# ragged widths: partial 128-wide tiles in every dimension, batch not a multiple of 32
SIZES = [72, 130, 100, 44]


def test_mlp_forward_gradients_adam_match_oracle():
    print(f"mlp sizes={SIZES}", flush=True)
    B = 37
    net = pdf.Mlp(SIZES, batch_max=64, device=DEV)
    net.init_weights(11)
    rng = np.random.default_rng(12)
    x = rng.normal(size=(B, SIZES[0])).astype(np.float32)
    t = rng.normal(size=(B, SIZES[-1])).astype(np.float32)
    xd, td = torch.tensor(x, device=DEV), torch.tensor(t, device=DEV)
    s_in = 0.8
    params = host_params(net)
    y = net.forward(xd, s_in=s_in, s_out=1.0).cpu().numpy()
    yo, cache = omlp.forward(params, x, s_in=s_in, quant=True)
    assert rel(y, yo) < 1e-4, rel(y, yo)
    y2 = net.forward(xd, s_in=s_in, s_out=2.5).cpu().numpy()
    assert rel(y2, 2.5 * yo) < 1e-4
    # one training step: loss, gradients, Adam
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    lr = 1e-3
    net.train_step(xd, td, None, s_in, lr, loss)
    lo, dy = omlp.mse(yo, t)
    assert abs(loss.item() - lo) < 1e-4 * lo
    go = omlp.backward(params, cache, dy, quant=True)
    new = host_params(net)
    for l in range(net.L):
        gW, gb = net.get_layer(l, grad=True)
        assert rel(gW, go[l][0]) < 2e-3, (l, rel(gW, go[l][0]))
        assert rel(gb, go[l][1]) < 2e-3, (l, rel(gb, go[l][1]))
        # Adam from the device's own gradients: first step of the bias-corrected form
        W1, _, _ = omlp.adam_update(params[l][0], gW.astype(np.float64), 0.0, 0.0, 1, lr)
        b1, _, _ = omlp.adam_update(params[l][1], gb.astype(np.float64), 0.0, 0.0, 1, lr)
        assert np.max(np.abs(new[l][0] - W1)) < 1e-6, l
        assert np.max(np.abs(new[l][1] - b1)) < 1e-6, l
    net.close()


U_BF16 = 2.0 ** -8       # unit round-off of bfloat16 (8 significant bits, round to nearest even)
# RMS relative error of rounding to 8 significant bits, for log-uniformly spread mantissas m in
# [1, 2): the absolute error is uniform in +-u (variance u^2 / 3) and E[1/m^2] = 3 / (8 ln 2)
R_BF16 = U_BF16 * np.sqrt(3.0 / (8.0 * np.log(2.0)) / 3.0)
C_CONF = 3.0             # standard deviations allowed


def _rounding_sd(A, B):
    """RMS Frobenius norm of the error of A @ B when both operands are rounded to bfloat16,
    errors independent across elements: (A B)_ij's error has variance
    2 R^2 sum_k A_ik^2 B_kj^2 (FP32 accumulation adds 2^-24 per term: negligible)."""
    return R_BF16 * np.sqrt(2.0 * np.sum((A * A) @ (B * B)))


def _gain(W, axis):
    """RMS gain of a layer product on an error of random direction: ||W||_F / sqrt(reduction width)."""
    return np.linalg.norm(W) / np.sqrt(W.shape[axis])


def _rms(v):
    return float(np.sqrt(np.mean(np.asarray(v) ** 2)))


def bf16_bounds(params, x, t, s_in):
    """Error bounds of the device's output and weight gradients against the plain FP64 network:
    C_CONF times the RMS error of a random-rounding model in which every layer product rounds
    both operands to bfloat16 once, and errors made earlier pass through later layers with the
    RMS gain of the layer product and of GELU's derivative at the FP64 pre-activations
    (independent errors add in quadrature), forward and then backward."""
    y, cache = omlp.forward(params, x, s_in=s_in)
    L = len(params)
    ez = [0.0] * L                     # RMS error of z_l
    for l, (W, _) in enumerate(params):
        a = cache[l][0]
        ea = _rms(omlp.gelu_grad(cache[l - 1][1])) * ez[l - 1] if l > 0 else 0.0
        ez[l] = np.hypot(_rounding_sd(a, W.T), _gain(W, 1) * ea)
    _, dy = omlp.mse(y, t)
    dz = dy
    edz = 2.0 * ez[L - 1] / y.size     # error of dL/dy = 2 (y - t) / size
    gW = [None] * L
    for l in range(L - 1, -1, -1):
        W, _ = params[l]
        a = cache[l][0]
        ea = _rms(omlp.gelu_grad(cache[l - 1][1])) * ez[l - 1] if l > 0 else 0.0
        # dW = dz^T a: fresh rounding of both operands, then the errors carried by dz and by a
        carried = np.hypot(edz * np.linalg.norm(a), np.linalg.norm(dz) * ea) / np.sqrt(a.shape[0])
        gW[l] = C_CONF * np.hypot(_rounding_sd(dz.T, a), carried)
        if l > 0:
            gp = omlp.gelu_grad(cache[l - 1][1])
            dh = dz @ W
            edh = np.hypot(_rounding_sd(dz, W), _gain(W, 0) * edz)
            # dz_{l-1} = dh * gelu'(z_{l-1}): error of dh, and of gelu' at the perturbed z
            gpp = np.exp(-0.5 * cache[l - 1][1] ** 2) / np.sqrt(2.0 * np.pi) * (2.0 - cache[l - 1][1] ** 2)
            edz = np.hypot(_rms(gp) * edh, _rms(dh * gpp) * ez[l - 1] / np.sqrt(dh.size))
            dz = dh * gp
    return y, C_CONF * ez[L - 1], gW


def test_bf16_network_within_the_rounding_bound_of_fp64():
    print(f"mlp bf16 vs fp64 sizes={SIZES}", flush=True)
    B = 37
    net = pdf.Mlp(SIZES, batch_max=64, device=DEV)
    net.init_weights(21)
    rng = np.random.default_rng(22)
    x = rng.normal(size=(B, SIZES[0])).astype(np.float32)
    t = rng.normal(size=(B, SIZES[-1])).astype(np.float32)
    s_in = 0.8
    params = host_params(net)
    y_ref, ey, gW_bound = bf16_bounds(params, x.astype(np.float64), t.astype(np.float64), s_in)
    y = net.forward(torch.tensor(x, device=DEV), s_in=s_in, s_out=1.0).cpu().numpy()
    err_y = np.linalg.norm(y - y_ref)
    print(f"output error {err_y / np.linalg.norm(y_ref):.2e} relative, bound {ey / np.linalg.norm(y_ref):.2e}",
          flush=True)
    assert err_y <= ey
    net.train_step(torch.tensor(x, device=DEV), torch.tensor(t, device=DEV), None, s_in, 1e-3)
    _, cache = omlp.forward(params, x.astype(np.float64), s_in=s_in)
    _, dy = omlp.mse(y_ref, t.astype(np.float64))
    go = omlp.backward(params, cache, dy)
    for l in range(net.L):
        gW, _ = net.get_layer(l, grad=True)
        err = np.linalg.norm(gW - go[l][0])
        print(f"layer {l}: weight-gradient error {err / np.linalg.norm(go[l][0]):.2e} relative, bound "
              f"{gW_bound[l] / np.linalg.norm(go[l][0]):.2e}", flush=True)
        assert err <= gW_bound[l], l
    net.close()


def test_mlp_row_gather_equals_gathered_rows():
    B = 24
    rng = np.random.default_rng(13)
    x = torch.tensor(rng.normal(size=(50, SIZES[0])).astype(np.float32), device=DEV)
    t = torch.tensor(rng.normal(size=(50, SIZES[-1])).astype(np.float32), device=DEV)
    idx = torch.tensor(rng.permutation(50)[:B].astype(np.int32), device=DEV)
    grads = []
    for gathered in (False, True):
        net = pdf.Mlp(SIZES, batch_max=32, device=DEV)
        net.init_weights(14)
        if gathered:
            net.train_step(x[idx.long()].contiguous(), t[idx.long()].contiguous(), None, 1.0, 1e-3)
        else:
            net.train_step(x, t, idx, 1.0, 1e-3)
        grads.append([net.get_layer(l, grad=True) for l in range(net.L)])
        net.close()
    for (a, b), (c, d) in zip(grads[0], grads[1]):
        assert np.array_equal(a, c) and np.array_equal(b, d)


def test_mlp_training_fits_a_linear_map():
    sizes = [64, 128, 128, 32]
    rng = np.random.default_rng(15)
    A = rng.normal(size=(32, 64)) / 8.0
    x = rng.normal(size=(256, 64)).astype(np.float32)
    t = (x @ A.T).astype(np.float32)
    xd, td = torch.tensor(x, device=DEV), torch.tensor(t, device=DEV)
    net = pdf.Mlp(sizes, batch_max=256, device=DEV)
    net.init_weights(16)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    hist = []
    for step in range(300):
        net.train_step(xd, td, None, 1.0, 3e-3, loss)
        hist.append(loss.item())
    assert np.all(np.isfinite(hist))
    assert hist[-1] < 0.05 * hist[0], (hist[0], hist[-1])
    net.close()


def test_analyze_matches_oracle():
    for M, K, prec, tol in [(32, 9, "fp32", 1e-5), (64, 15, "fp32", 1e-5), (16, 7, "fp64", 1e-12),
                            (16, 16, "fp32", 1e-5), (48, 13, "fp32", 1e-5), (48, 11, "fp64", 1e-12)]:
        case = make_case(M, K, 3, 4, seeds=(0,))
        wl = case["wl"]
        s = pdf.Solver(M, wl.side, wl.freq_hz, case["tx"], case["rx"], K, batch=1,
                       params=pdf.default_params(prec), device=DEV)
        rng = np.random.default_rng(M + K)
        J = rng.normal(size=(5, 3, M, M)) + 1j * rng.normal(size=(5, 3, M, M))
        got = s.analyze(torch.tensor(J, dtype=s.cdtype, device=DEV)).cpu().numpy()
        ref = fourier.analyze(J, K)
        assert rel(got, ref) < tol, (M, K, prec, rel(got, ref))
        s.close()


def test_warm_start_keeps_the_lower_loss_start():
    M, K, Ni, Ns, B = 32, 9, 6, 8, 4
    case = make_case(M, K, Ni, Ns, seeds=tuple(range(B)))
    wl = case["wl"]
    s = pdf.Solver(M, wl.side, wl.freq_hz, case["tx"], case["rx"], K, batch=B, device=DEV)
    esca = np.stack([c["esca"] for c in case["cases"]])
    s.set_data(torch.tensor(esca, dtype=s.cdtype, device=DEV))
    bp = s.init_alpha()
    nin, nout = 2 * Ni * Ns, 2 * Ni * K * K
    net = pdf.Mlp([nin, 16, nout], batch_max=3, device=DEV)  # batch_max < B: predictions in chunks
    net.init_weights(17)
    # a network whose output ignores its input: zero last weights, bias = a chosen alpha
    target = (bp[1] * 0.5).cpu().numpy()
    bias = np.stack([target.real, target.imag], axis=-1).reshape(-1).astype(np.float32)
    net.set_layer(1, np.zeros((nout, 16), np.float32), bias)
    alpha, chosen, losses = s.warm_start(net, 1.0, 1.0)
    l_bp = s.loss_grad(bp, grad=False)[0][:, 5].cpu().numpy()
    pred = torch.tensor(np.broadcast_to(target, (B, Ni, K, K)).copy(), dtype=s.cdtype, device=DEV)
    l_net = s.loss_grad(pred, grad=False)[0][:, 5].cpu().numpy()
    lo = losses.cpu().numpy()
    assert np.allclose(lo[:, 0], l_bp, rtol=1e-12) and np.allclose(lo[:, 1], l_net, rtol=1e-12)
    want = l_net < l_bp
    assert np.array_equal(chosen.cpu().numpy() == 1, want)
    for b in range(B):
        ref = pred[b] if want[b] else bp[b]
        assert torch.equal(alpha[b], ref), b
    # widths that do not fit the handle are refused
    bad = pdf.Mlp([nin + 2, 8, nout], batch_max=4, device=DEV)
    with pytest.raises(pdf.PdfError):
        s.warm_start(bad, 1.0, 1.0)
    bad.close()
    net.close()
    s.close()


def test_trained_warm_start_gains_over_the_plain_start():
    """What the trained network adds: on held-out cfg2 instances its start (kept only where its loss
    is lower) has a lower image error than the back-propagation start, and so has the best image
    along 100 Adam iterations from it."""
    import seeded_inputs as si
    from paper_2602_13805_amd import warmstart as ws
    wl = si.WORKLOADS["cfg2"]
    print("warm-start gain: 768 training pairs, 32 held-out instances", flush=True)
    tr_data = ws.make_dataset(si, wl, ws.TRAIN_SEED0 + np.arange(768), DEV)
    ev = ws.make_dataset(si, wl, np.arange(32), DEV)
    tr = ws.train(tr_data, epochs=40, batch=128, lr=1e-3, seed=3, device=DEV)
    assert tr.history[-1] < 0.5 * tr.history[0]
    B = 32
    tx = si.antenna_positions(wl.n_tx, wl.radius)
    rx = si.antenna_positions(wl.n_rx, wl.radius)
    s = pdf.Solver(wl.M, wl.side, wl.freq_hz, tx, rx, wl.K, batch=B, device=DEV)
    s.set_data(torch.view_as_complex(ev.x.reshape(B, wl.n_tx, wl.n_rx, 2)).contiguous())
    eps_t = torch.tensor(ev.eps, dtype=torch.complex64, device=DEV)
    a_bp = s.init_alpha()
    a_w, chosen, losses = s.warm_start(tr.net, tr.s_in, tr.s_out)
    lo = losses.cpu().numpy()
    assert np.all(lo[:, 1][chosen.cpu().numpy() == 1] < lo[:, 0][chosen.cpu().numpy() == 1])
    e_bp = s.image(a_bp, eps_t)[2].cpu().numpy()
    e_w = s.image(a_w, eps_t)[2].cpu().numpy()
    r_bp = s.reconstruct(100, n_check=10, alpha=a_bp.clone(), eps_true=eps_t)["best_err"].cpu().numpy()
    r_w = s.reconstruct(100, n_check=10, alpha=a_w.clone(), eps_true=eps_t)["best_err"].cpu().numpy()
    print(f"start error bp {e_bp.mean():.4f} warm {e_w.mean():.4f}; best within 100 its bp {r_bp.mean():.4f} "
          f"warm {r_w.mean():.4f}; network start kept on {int(chosen.sum())} of {B}", flush=True)
    assert int(chosen.sum()) > 0
    assert e_w.mean() < e_bp.mean()
    assert r_w.mean() < r_bp.mean()
    # image-error bound of the bfloat16 network path: the start predicted by the device network and
    # the start the plain FP64 network (same weights) predicts give image errors within 0.01 of
    # each other on every held-out instance (both images from the same FP32 physics and CCO)
    params = host_params(tr.net)
    y64, _ = omlp.forward(params, ev.x.double().cpu().numpy(), s_in=tr.s_in)
    a64 = torch.view_as_complex(torch.tensor(tr.s_out * y64, dtype=torch.float32).reshape(B, -1, 2)).reshape(
        a_bp.shape).to(DEV).contiguous()
    a16 = torch.view_as_complex(ws.predict(tr, ev.x).reshape(B, -1, 2)).reshape(a_bp.shape).contiguous()
    d = np.abs(s.image(a16, eps_t)[2].cpu().numpy() - s.image(a64, eps_t)[2].cpu().numpy())
    print(f"bfloat16 vs FP64 network start: image errors differ by at most {d.max():.2e} (mean {d.mean():.2e})",
          flush=True)
    assert d.max() <= 0.01
    tr.net.close()
    s.close()
