"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances: FP32 arithmetic on the device against FP64 on the host: loss terms
and gradients within 1e-4 relative (norm-wise, and every gradient entry within
1e-4 of the largest), or, for the terms that depend on chi = R / (beta (1 - R))
and the gradient, 1e-6 times that map's condition number where it is larger;
the FP64 instantiation within 1e-9.
"""
import numpy as np
import pytest
import torch

import seeded_inputs as si
from oracle import adam as oadam, cco as occo, forward, init as oinit, loss as oloss, solver as osolver
from oracle import operators as ops
from tests.common import geometry, make_case, rand_alpha, rel

pytestmark = pytest.mark.gpu

pdf = pytest.importorskip("paper_2602_13805_amd")
DEV = "cuda:0"


def solver_for(case, precision, batch=None, **kw):
    wl = case["wl"]
    B = batch or len(case["cases"])
    params = pdf.default_params(precision, **kw)
    s = pdf.Solver(case["M"], wl.side, wl.freq_hz, case["tx"], case["rx"], case["K"], batch=B, params=params,
                   precision=precision, device=DEV)
    es = np.stack([c["esca"] for c in case["cases"]])[:B]
    s.set_data(torch.tensor(es, dtype=s.cdtype, device=DEV))
    return s


def oracle_terms(out):
    return np.array([out["L_state"], out["L_data"], out["L_bound"], out["L_tv"], out["L_bridge"], out["L"]])


def chi_condition(ref):
    """max |R| / |1 - R| over the pixels: the factor by which chi = R / (beta (1 - R)) amplifies a
    relative error in R."""
    R = np.asarray(ref["R"])
    return float(np.max(np.abs(R) / np.abs(1.0 - R)))


def term_tolerances(ref, prec, tol):
    """Per-term tolerance of (state, data, bound, TV, bridge, total) and of the gradient.  In FP32
    the device's R carries a relative error of about 1e-6 (two FFT convolutions and the incidence
    sums); the chi-dependent terms see it times the condition number of chi(R)."""
    tc = max(tol, 1e-6 * chi_condition(ref)) if prec == "fp32" else tol
    return np.array([tol, tol, tc, tc, tc, tc]), tc


def check_grad(g_dev, g_ref, tol):
    g_dev = np.asarray(g_dev)
    assert rel(g_dev, g_ref) < tol, rel(g_dev, g_ref)
    assert np.max(np.abs(g_dev - g_ref)) < tol * np.max(np.abs(g_ref))


CASES = [
    # (M, K, Ni, Ns, batch, precision, tol)
    (8, 5, 4, 6, 2, "fp32", 1e-4),
    (16, 7, 6, 8, 2, "fp32", 1e-4),
    (32, 9, 16, 32, 3, "fp32", 1e-4),
    (64, 15, 32, 32, 1, "fp32", 1e-4),
    (16, 7, 6, 8, 2, "fp64", 1e-9),
    (32, 9, 16, 32, 2, "fp64", 1e-9),
    (16, 16, 3, 5, 1, "fp32", 1e-4),   # full basis, even K (corner blocks)
    (32, 14, 5, 7, 1, "fp64", 1e-9),   # paper's corner set M_F = 7
    (16, 1, 1, 1, 1, "fp32", 1e-4),    # degenerate: one mode, one antenna each
    (32, 9, 36, 36, 2, "fp32", 1e-4),  # the paper's 36 / 36 antennas: ragged 2nd incidence / receiver tiles
    (16, 7, 64, 64, 1, "fp32", 1e-4),  # largest antenna counts of the FP32 path
    (8, 5, 33, 17, 2, "fp32", 1e-4),   # ragged tiles on a grid smaller than one pixel sub-tile
    (48, 13, 12, 20, 2, "fp32", 1e-4),  # P = 96: radix-12 / radix-3 passes; chi(R) condition ~1400
    (48, 13, 12, 20, 2, "fp64", 1e-9),  # the same instances in FP64: the arithmetic itself, strictly
    (48, 11, 6, 9, 2, "fp64", 1e-9),
    (48, 48, 3, 5, 1, "fp32", 1e-4),    # full basis on the radix-3 grid, even K (mapped wrap past 0)
    (48, 21, 36, 36, 1, "fp32", 1e-4),  # largest truncation of the uneven draws, the paper's antenna count
    (64, 15, 8, 12, 1, "fp64", 1e-9),   # the benchmark grid in FP64
    (96, 15, 12, 16, 1, "fp32", 1e-4),  # P = 192: 12-, 8- and 2-point row passes, 96-point column chains
    (64, 32, 8, 12, 1, "fp32", 1e-4),   # the compact tile at its largest K (even: corner blocks)
    (64, 33, 8, 12, 1, "fp32", 1e-4),   # one mode more: the full tile
    (64, 1, 4, 6, 2, "fp32", 1e-4),     # the compact tile with a single mode
    (64, 16, 8, 12, 1, "fp32", 1e-4),   # the compact tile's largest K with beta U and g_J's kept columns in
                                        # its spare columns, and the adjoint's odd-part product (even K)
    (64, 17, 8, 12, 1, "fp32", 1e-4),   # one mode more: both wait elsewhere, the odd part by row transforms
    (32, 16, 6, 8, 1, "fp64", 1e-9),    # 2K = M: the last K at which the full tile's forward folds beta J
]


@pytest.mark.parametrize("M,K,Ni,Ns,B,prec,tol", CASES)
def test_loss_grad_parity(M, K, Ni, Ns, B, prec, tol):
    print(f"case M={M} K={K} Ni={Ni} Ns={Ns} B={B} {prec}", flush=True)
    case = make_case(M, K, Ni, Ns, seeds=tuple(range(B)))
    s = solver_for(case, prec)
    alpha = np.stack([rand_alpha((Ni, K, K), seed=10 + b) for b in range(B)])
    loss, g = s.loss_grad(torch.tensor(alpha, dtype=s.cdtype, device=DEV))
    loss = loss.cpu().numpy()
    g = g.cpu().numpy()
    for b, c in enumerate(case["cases"]):
        ref = oloss.evaluate(alpha[b], c["prob"])
        want = oracle_terms(ref)
        got = loss[b, :6]
        tt, tg = term_tolerances(ref, prec, tol)
        assert np.all(np.abs(got - want) <= tt * np.abs(want) + tol * 1e-3 * abs(want[5])), (b, got, want, tt)
        assert loss[b, 7] == 0.0
        check_grad(g[b], ref["g_alpha"], tg)
    s.close()


def test_cfg2_full_size_parity():
    # 64 x 64, 32 Tx / 32 Rx, K = 15, data from a 128 x 128 MoM with noise and jitter
    wl = si.WORKLOADS["cfg2"]
    print("case cfg2 full size", flush=True)
    jt, jr = si.draw_jitter(0, wl.n_tx, wl.n_rx, wl.jitter_deg)
    txj = si.antenna_positions(wl.n_tx, wl.radius, angle_offsets=jt)
    rxj = si.antenna_positions(wl.n_rx, wl.radius, angle_offsets=jr)
    shapes = si.draw_profile(wl, 0)
    es, _ = forward.mom_solve(si.rasterize(shapes, wl.M_fine, wl.side), wl.side, ops.wavenumber(wl.freq_hz),
                              txj, rxj)
    n1, n2 = si.draw_noise(0, es.shape)
    es = forward.add_noise(es, wl.noise, n1, n2)
    tx, rx = geometry(wl.n_tx, wl.n_rx)
    prob = oloss.build_problem(wl.M, wl.K, wl.side, [wl.freq_hz], tx, rx, es)
    a0 = oinit.alpha0(prob)[0][0]
    s = pdf.Solver(wl.M, wl.side, wl.freq_hz, tx, rx, wl.K, batch=1, device=DEV)
    s.set_data(torch.tensor(es[None], dtype=s.cdtype, device=DEV))
    for alpha in (a0, a0 + rand_alpha(a0.shape, 0.02, 3)):
        loss, g = s.loss_grad(torch.tensor(alpha[None], dtype=s.cdtype, device=DEV))
        ref = oloss.evaluate(alpha, prob)
        want = oracle_terms(ref)
        got = loss.cpu().numpy()[0, :6]
        assert np.all(np.abs(got - want) <= 1e-4 * np.abs(want) + 1e-7 * abs(want[5])), (got, want)
        check_grad(g.cpu().numpy()[0], ref["g_alpha"], 1e-4)
    # start value on the device against the oracle's
    a_dev = s.init_alpha().cpu().numpy()[0]
    assert rel(a_dev, a0) < 1e-4
    s.close()


# FP32: the start is one exact line-search step, its inputs the back-propagation image and R_0;
# FP32's unit round-off 6e-8 times a few dozen operations in sequence (two FFT convolutions, the
# incidence sums, the receiver GEMMs; the step size from FP64-accumulated sums) leaves ~1e-6
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp64", 1e-9)])
def test_init_alpha_parity(prec, tol):
    case = make_case(32, 9, 8, 12, seeds=(0, 1))
    s = solver_for(case, prec)
    a = s.init_alpha().cpu().numpy()
    for b, c in enumerate(case["cases"]):
        ref, info = oinit.alpha0(c["prob"])
        print(f"init alpha {prec} b={b}: rel {rel(a[b], ref[0]):.2e}", flush=True)
        assert rel(a[b], ref[0]) < tol, rel(a[b], ref[0])
    s.close()


@pytest.mark.parametrize("M,K,prec,tol", [(32, 9, "fp32", 1e-4), (32, 9, "fp64", 1e-10), (64, 15, "fp64", 1e-10),
                                           (96, 15, "fp32", 1e-4)])
def test_image_and_cco_parity(M, K, prec, tol):
    print(f"image / CCO M={M} K={K} {prec}", flush=True)
    case = make_case(M, K, 8, 12, seeds=(0, 1))
    s = solver_for(case, prec)
    alpha = np.stack([oinit.alpha0(c["prob"])[0][0] for c in case["cases"]])
    eps = np.stack([c["eps"] for c in case["cases"]])
    chi, cco, err = s.image(torch.tensor(alpha, dtype=s.cdtype, device=DEV),
                            torch.tensor(eps, dtype=s.cdtype, device=DEV))
    for b, c in enumerate(case["cases"]):
        ref = oloss.evaluate(alpha[b], c["prob"], grad=False)
        assert rel(chi[b].cpu().numpy(), ref["chi"]) < tol
        ref_cco = occo.cco(ref["chi"])
        assert rel(cco[b].cpu().numpy(), ref_cco) < tol
        assert abs(err[b].item() - occo.image_error(ref_cco, c["eps"])) < tol
    s.close()


def test_adam_steps_fp64_match_oracle():
    case = make_case(16, 7, 6, 8, seeds=(0, 1))
    s = solver_for(case, "fp64")
    alpha0 = np.stack([rand_alpha((6, 7, 7), seed=20 + b) for b in range(2)])
    a = torch.tensor(alpha0, dtype=s.cdtype, device=DEV)
    m, v, t = s.new_state()
    loss = torch.empty((2, 8), dtype=torch.float64, device=DEV)
    for _ in range(12):
        s.step(a, m, v, t, loss)
    assert t.cpu().tolist() == [12, 12]
    for b, c in enumerate(case["cases"]):
        x = alpha0[b].copy()
        mm = np.zeros(x.shape + (2,))
        vv = np.zeros(x.shape + (2,))
        for k in range(1, 13):
            last = oloss.evaluate(x, c["prob"])
            x, mm, vv = oadam.adam_step(x, last["g_alpha"], mm, vv, k)
        assert rel(a[b].cpu().numpy(), x) < 1e-9
        assert abs(loss[b, 5].item() - last["L"]) < 1e-9 * last["L"]
    s.close()


def test_reconstruct_fp64_matches_oracle_and_graph_replay():
    # cfg1-shaped FP64 reconstruction: 32 x 32, 16 Tx / 32 Rx, K = 9, 100 Adam steps
    print("case cfg1 reconstruct", flush=True)
    wl = si.WORKLOADS["cfg1"]
    case = make_case(wl.M, wl.K, wl.n_tx, wl.n_rx, seeds=(0, 1))
    s = solver_for(case, "fp64")
    res = s.reconstruct(100, n_check=25)
    assert res["iters_run"] == 100
    a_dev = res["alpha"].cpu().numpy()
    for b, c in enumerate(case["cases"]):
        ref = osolver.reconstruct(c["prob"], 100)
        assert rel(a_dev[b], ref["alpha"][0]) < 1e-8, rel(a_dev[b], ref["alpha"][0])
        assert rel(res["chi_cco"][b].cpu().numpy(), ref["chi_cco"]) < 1e-8
    # the same steps issued one by one (no graph) give the same bits
    a = s.init_alpha()
    m, v, t = s.new_state()
    for _ in range(100):
        s.step(a, m, v, t)
    assert torch.equal(a, res["alpha"])
    s.close()


def test_batched_equals_single_and_deterministic():
    case = make_case(32, 9, 8, 12, seeds=(0, 1, 2))
    sb = solver_for(case, "fp32")
    alpha = np.stack([rand_alpha((8, 9, 9), seed=30 + b) for b in range(3)])
    at = torch.tensor(alpha, dtype=sb.cdtype, device=DEV)
    l1, g1 = sb.loss_grad(at)
    l2, g2 = sb.loss_grad(at)
    assert torch.equal(l1, l2) and torch.equal(g1, g2)
    for b in range(3):
        one = dict(case)
        one["cases"] = [case["cases"][b]]
        s1 = solver_for(one, "fp32")
        l, g = s1.loss_grad(at[b:b + 1].contiguous())
        assert torch.equal(l[0], l1[b]) and torch.equal(g[0], g1[b])
        s1.close()
    sb.close()


def test_gradient_fd_on_device_fp64():
    # the device adjoint against central differences of the device loss
    case = make_case(16, 7, 4, 6, seeds=(3,))
    s = solver_for(case, "fp64")
    alpha = rand_alpha((1, 4, 7, 7), seed=5)
    at = torch.tensor(alpha, dtype=s.cdtype, device=DEV)
    _, g = s.loss_grad(at)
    g = g.cpu().numpy()
    rng = np.random.default_rng(0)
    for _ in range(8):
        idx = tuple(int(rng.integers(0, n)) for n in alpha.shape)
        for d in (1.0, 1j):
            h = 1e-7
            ap, am = alpha.copy(), alpha.copy()
            ap[idx] += h * d
            am[idx] -= h * d
            lp = s.loss_grad(torch.tensor(ap, dtype=s.cdtype, device=DEV), grad=False)[0][0, 5].item()
            lm = s.loss_grad(torch.tensor(am, dtype=s.cdtype, device=DEV), grad=False)[0][0, 5].item()
            fd = (lp - lm) / (2 * h)
            an = g[idx].real if d == 1.0 else g[idx].imag
            assert abs(fd - an) < 1e-6 * np.max(np.abs(g)), (idx, d, fd, an)
    s.close()


def test_autograd_function_and_checkpoint():
    case = make_case(16, 7, 4, 6, seeds=(0, 1))
    s = solver_for(case, "fp32")
    alpha = torch.tensor(np.stack([rand_alpha((4, 7, 7), seed=b) for b in range(2)]), dtype=s.cdtype,
                         device=DEV, requires_grad=True)
    w = torch.tensor([1.0, 0.5], dtype=torch.float64, device=DEV)
    (pdf.PdfLoss.apply(alpha, s, False) * w).sum().backward()
    g1 = alpha.grad.clone()
    alpha.grad = None
    l_ck = pdf.PdfLoss.apply(alpha, s, True)
    (l_ck * w).sum().backward()
    assert torch.equal(alpha.grad, g1)
    lo, g = s.loss_grad(alpha.detach().contiguous())
    assert torch.allclose(g1[1], 0.5 * g[1])
    # the loss-only pass (no gradient output: no adjoint kernels) gives the same loss bit for bit
    lo_only, none = s.loss_grad(alpha.detach().contiguous(), grad=False)
    assert none is None and torch.equal(lo_only, lo) and torch.equal(l_ck.detach(), lo[:, 5])
    s.close()


def test_mean_square_of_device_arrays():
    rng = np.random.default_rng(5)
    for dt in (torch.float32, torch.float64, torch.complex64, torch.complex128):
        for n in (1, 1000, 300001):
            x = torch.tensor(rng.standard_normal(n) * 3.0, device=DEV).to(dt if not dt.is_complex else
                                                                              torch.float64)
            if dt.is_complex:
                x = torch.complex(x, 0.5 * x.flip(0)).to(dt)
            ref = float(np.mean(np.abs(x.cpu().numpy().astype(np.complex128)) ** 2))
            got = pdf.mean_abs2(x)
            tol = 1e-6 if dt in (torch.float32, torch.complex64) else 1e-13
            assert abs(got - ref) <= tol * ref, (dt, n, got, ref)


def test_synthesize_matches_oracle_mom():
    wl = si.WORKLOADS["cfg1"]
    tx, rx = geometry(8, 12)
    shapes = si.draw_profile(wl, 4)
    eps = si.rasterize(shapes, 64, wl.side)
    got = pdf.synthesize(64, wl.side, wl.freq_hz, tx, rx, eps, tol=1e-11, device=DEV)
    ref, _ = forward.mom_solve(eps, wl.side, ops.wavenumber(wl.freq_hz), tx, rx)
    assert rel(got, ref) < 1e-9, rel(got, ref)
    # antennas 1.5 wavelengths from the centre of a 2-wavelength domain: too close for the
    # interpolated Hankel samples, so the host evaluates the antenna fields
    txn, rxn = geometry(6, 7, radius_wl=1.5)
    got = pdf.synthesize(64, wl.side, wl.freq_hz, txn, rxn, eps, tol=1e-11, device=DEV)
    ref, _ = forward.mom_solve(eps, wl.side, ops.wavenumber(wl.freq_hz), txn, rxn)
    assert rel(got, ref) < 1e-9, rel(got, ref)
    # a 96 x 96 grid (the fine grid of the 48 x 48 inversion grid)
    eps96 = si.rasterize(shapes, 96, wl.side)
    got = pdf.synthesize(96, wl.side, wl.freq_hz, tx, rx, eps96, tol=1e-11, device=DEV)
    ref, _ = forward.mom_solve(eps96, wl.side, ops.wavenumber(wl.freq_hz), tx, rx)
    assert rel(got, ref) < 1e-9, rel(got, ref)
    # empty support: zero field
    z = pdf.synthesize(16, wl.side, wl.freq_hz, tx, rx, np.ones((16, 16)), device=DEV)
    assert np.all(z == 0)


def test_synthesize_batch_matches_single_and_oracle_currents():
    wl = si.WORKLOADS["cfg1"]
    n, Ni, Ns, M = 5, 8, 12, 32
    txs, rxs, eps = [], [], np.zeros((n, M, M), np.complex128)
    for b in range(n):
        jt, jr = si.draw_jitter(b, Ni, Ns, 2.0)
        txs.append(si.antenna_positions(Ni, 3 * wl.wavelength, angle_offsets=jt))
        rxs.append(si.antenna_positions(Ns, 3 * wl.wavelength, angle_offsets=jr))
        eps[b] = si.rasterize(si.draw_profile(wl, b), M, wl.side)
    eps[3] = 1.0  # an empty instance in the middle of the batch
    print(f"synthesize_batch n={n} M={M}", flush=True)
    es, jc = pdf.synthesize_batch(M, wl.side, wl.freq_hz, txs, rxs, eps, tol=1e-11, coarse=2, workers=3,
                                  device=DEV)
    assert jc.shape == (n, Ni, M // 2, M // 2)
    k0 = ops.wavenumber(wl.freq_hz)
    for b in range(n):
        one = pdf.synthesize(M, wl.side, wl.freq_hz, txs[b], rxs[b], eps[b], tol=1e-11, device=DEV)
        assert np.array_equal(one, es[b]), b          # same solve, whichever thread ran it
        ref, etot = forward.mom_solve(eps[b], wl.side, k0, txs[b], rxs[b])
        if b == 3:
            assert np.all(es[b] == 0) and np.all(jc[b] == 0)
            continue
        assert rel(es[b], ref) < 1e-9, (b, rel(es[b], ref))
        jref = ((eps[b].reshape(-1) - 1.0)[None, :] * etot).reshape(Ni, M // 2, 2, M // 2, 2).mean(axis=(2, 4))
        assert rel(jc[b], jref) < 1e-9, (b, rel(jc[b], jref))


def test_synthesis_at_displaced_antennas():
    """The antenna-position study's data (Sec. 4): one batched synthesis of the same object seen
    from displaced antennas.  Each member within 1e-9 of the oracle's MoM at those positions; and
    on the device too, antennas moved by one pixel width see the object shifted back by one pixel
    (once the sources' unit-at-centre amplitudes are divided out)."""
    from scipy import special
    wl = si.WORKLOADS["cfg1"]
    M, Ni, Ns = 32, 8, 12
    h = wl.side / M
    k0 = ops.wavenumber(wl.freq_hz)
    tx, rx = geometry(Ni, Ns)
    eps = si.rasterize([si.Shape("ellipse", 0.05 * wl.wavelength, -0.1 * wl.wavelength, 0.3 * wl.wavelength,
                                 0.3 * wl.wavelength, 0.0, 2.5 + 0j)], M, wl.side)
    assert np.all(eps[:, 0] == 1) and np.all(eps[:, -1] == 1) and np.all(eps[0] == 1) and np.all(eps[-1] == 1)
    dx = np.array([h, 0.0])
    dt, dr = si.draw_position_errors(3, Ni, Ns, 1e-3)
    txs = [tx, tx + dx, tx, tx + dt]
    rxs = [rx, rx + dx, rx, rx + dr]
    epss = np.stack([eps, eps, np.roll(eps, -1, axis=1), eps])
    print(f"synthesize_batch at displaced antennas M={M}", flush=True)
    es = pdf.synthesize_batch(M, wl.side, wl.freq_hz, txs, rxs, epss, tol=1e-12, device=DEV)
    for b in range(4):
        ref, _ = forward.mom_solve(epss[b], wl.side, k0, txs[b], rxs[b])
        assert rel(es[b], ref) < 1e-9, (b, rel(es[b], ref))
    amp = lambda t: 1.0 / np.abs(special.hankel1(0, k0 * np.hypot(t[:, 0], t[:, 1])))[:, None]
    assert rel(es[1] / amp(tx + dx), es[2] / amp(tx)) < 1e-9
    assert rel(es[1], es[0]) > 1e-3 and rel(es[3], es[0]) > 1e-5


def test_tile_choices_do_not_change_results_and_autotune_picks_one():
    for (M, K, Ni, Ns, B) in [(32, 9, 16, 32, 3), (8, 5, 33, 17, 2), (64, 15, 32, 32, 1), (48, 13, 24, 24, 2),
                              (96, 11, 8, 12, 1)]:
        case = make_case(M, K, Ni, Ns, seeds=tuple(range(B)))
        s = solver_for(case, "fp32")
        alpha = torch.tensor(rand_alpha(s.alpha_shape, seed=M), dtype=s.cdtype, device=DEV)
        outs = []
        for ct in (1, 2, 4):
            for pb in (4, 8):
                for fpp, app in ((0, 0), (1, 1), (0, 1)):
                    s.set_tiles(ct, pb, fpp, app)
                    loss, g = s.loss_grad(alpha)
                    outs.append((loss.clone(), g.clone()))
        for loss, g in outs[1:]:
            assert torch.equal(loss, outs[0][0]) and torch.equal(g, outs[0][1]), (M, Ni, Ns)
        (ct, pb, fpp, app), ms = s.autotune(3)
        print(f"autotune M={M} Ni={Ni} Ns={Ns} B={B}: ct={ct} pb={pb} fwd_plan={fpp} adj_plan={app} "
              f"ms={np.round(ms, 4).tolist()}", flush=True)
        assert ct in (1, 2, 4) and pb in (4, 8) and fpp in (0, 1) and app in (0, 1) and np.all(ms > 0)
        if M == 96:  # the full tile does not fit: plan 0 only
            assert (fpp, app) == (0, 0) and np.all(ms[5:] == ms[5])
        loss, g = s.loss_grad(alpha)
        assert torch.equal(loss, outs[0][0]) and torch.equal(g, outs[0][1])
        with pytest.raises(pdf.PdfError):
            s.set_tiles(3, 4)
        s.close()


def test_reconstruct_multi_equals_separate_reconstructions():
    """Uneven batching: handles of different grids, antenna counts, truncations, batches and
    precisions advanced in one graph give exactly what each handle gives alone."""
    # same-class pairs (one grid, the same receiver / incidence tile counts) run as grouped launches:
    # M = 16 with N_s <= 16, N_i <= 16, M = 32 with 16 < N_s <= 32, N_i <= 16, and M = 48 with
    # N_s <= 16, N_i <= 16
    shapes = [(16, 7, 6, 8, 2, "fp32"), (32, 9, 16, 32, 3, "fp32"), (16, 5, 4, 6, 2, "fp64"), (8, 5, 3, 5, 1, "fp32"),
              (16, 5, 5, 7, 3, "fp32"), (32, 11, 12, 20, 2, "fp32"), (16, 9, 9, 13, 1, "fp32"),
              (48, 9, 16, 16, 2, "fp32"), (48, 13, 12, 14, 1, "fp32")]
    sol, eps, datas = [], [], []
    for (M, K, Ni, Ns, B, prec) in shapes:
        case = make_case(M, K, Ni, Ns, seeds=tuple(range(B)))
        s = solver_for(case, prec)
        sol.append(s)
        eps.append(torch.tensor(np.stack([c["eps"] for c in case["cases"]]), dtype=s.cdtype, device=DEV))
    print("reconstruct_multi shapes", shapes, flush=True)
    for with_target in (False, True):
        targets = None
        ref = []
        for s, et in zip(sol, eps):
            tg = None
            if with_target:  # stop some instances early: the error after the first check
                r0 = s.reconstruct(10, n_check=10, eps_true=et)
                tg = (r0["best_err"] * 1.02).contiguous()
            ref.append((s.reconstruct(40, n_check=10, eps_true=et, target=tg), tg))
        if with_target:
            targets = [tg for _, tg in ref]
        got, info = pdf.reconstruct_multi(sol, 40, n_check=10, eps_trues=eps, targets=targets)
        for (r, _), g in zip(ref, got):
            assert torch.equal(r["alpha"], g["alpha"])
            assert torch.equal(r["chi_cco"], g["chi_cco"])
            assert torch.equal(r["best_err"], g["best_err"]) and torch.equal(r["best_iter"], g["best_iter"])
            assert torch.equal(r["reached"], g["reached"])
        if with_target:
            assert info["n_reached"] == sum(int((r["reached"] >= 0).sum()) for r, _ in ref)
    # a handle listed twice is refused
    with pytest.raises(pdf.PdfError):
        pdf.reconstruct_multi([sol[0], sol[0]], 10)
    for s in sol:
        s.close()


def test_error_paths_on_device():
    case = make_case(16, 7, 4, 6, seeds=(0,))
    wl = case["wl"]
    s = pdf.Solver(16, wl.side, wl.freq_hz, case["tx"], case["rx"], 7, device=DEV)
    with pytest.raises(pdf.PdfError) as e:
        s.loss_grad(s.zeros_alpha())   # no data yet
    assert e.value.code == -1
    with pytest.raises(pdf.PdfError) as e:
        s.set_data(torch.zeros((1, 4, 6), dtype=s.cdtype, device=DEV))  # ||E_sca|| = 0
    assert e.value.code == -4
    s.close()


def test_cfg2_batch_of_256_in_the_benchmark_configuration():
    """The benchmark's launch configuration (cfg2, 256 instances, autotuned tiles and FFT plans):
    loss terms, gradient and one Adam step of sampled instances against the oracle, one by one.
    Measured fields and coefficients are seeded random draws (any field is a valid input of the
    loss), so no input comes from the device."""
    wl = si.WORKLOADS["cfg2"]
    B, sample = 256, (0, 97, 181, 255)
    print("case cfg2 B=256 autotuned, sampled instances", sample, flush=True)
    tx, rx = geometry(wl.n_tx, wl.n_rx)
    rng = np.random.default_rng(256)
    es = 0.1 * (rng.standard_normal((B, wl.n_tx, wl.n_rx)) + 1j * rng.standard_normal((B, wl.n_tx, wl.n_rx)))
    alpha = np.stack([rand_alpha((wl.n_tx, wl.K, wl.K), 0.02, 1000 + b) for b in range(B)])
    s = pdf.Solver(wl.M, wl.side, wl.freq_hz, tx, rx, wl.K, batch=B, device=DEV)
    s.set_data(torch.tensor(es, dtype=s.cdtype, device=DEV))
    tiles, _ = s.autotune(3)
    print("tiles", tiles, flush=True)
    ad = torch.tensor(alpha, dtype=s.cdtype, device=DEV)
    loss, g = s.loss_grad(ad)
    loss, g = loss.cpu().numpy(), g.cpu().numpy()
    m, v, t = s.new_state()
    s.step(ad, m, v, t)
    stepped = ad.cpu().numpy()
    for b in sample:
        prob = oloss.build_problem(wl.M, wl.K, wl.side, [wl.freq_hz], tx, rx, es[b])
        ref = oloss.evaluate(alpha[b], prob)
        want = oracle_terms(ref)
        tt, tg = term_tolerances(ref, "fp32", 1e-4)
        assert np.all(np.abs(loss[b, :6] - want) <= tt * np.abs(want) + 1e-7 * abs(want[5])), (b, loss[b], want)
        check_grad(g[b], ref["g_alpha"], tg)
        a1, _, _ = oadam.adam_step(alpha[b], ref["g_alpha"], np.zeros(alpha[b].shape + (2,)),
                                   np.zeros(alpha[b].shape + (2,)), 1)
        # first Adam step: lr sign(g) wherever |g| >> eps; near-zero gradients may take either sign
        gmax = np.max(np.abs(ref["g_alpha"]))
        for part in (np.real, np.imag):
            strong = np.abs(part(ref["g_alpha"])) > 1e-2 * gmax
            assert np.max(np.abs(part(stepped[b] - a1)[strong])) < 1e-6
        assert np.max(np.abs(stepped[b] - a1)) <= 2 * np.sqrt(2) * 1e-2
    s.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_resume_100_plus_100_equals_200_steps(prec):
    """Checkpoint and resume: the step state (alpha, Adam moments, step counters) is caller-visible
    device memory, so 100 steps, a copy to the host, a new handle and 100 more steps equal 200 steps
    on one handle bit for bit."""
    case = make_case(16, 7, 6, 8, seeds=(0, 1))
    s = solver_for(case, prec)
    a = s.init_alpha()
    m, v, t = s.new_state()
    for _ in range(100):
        s.step(a, m, v, t)
    saved = [x.cpu().clone() for x in (a, m, v, t)]
    for _ in range(100):
        s.step(a, m, v, t)
    s.close()
    s2 = solver_for(case, prec)
    a2, m2, v2, t2 = [x.to(DEV) for x in saved]
    for _ in range(100):
        s2.step(a2, m2, v2, t2)
    assert torch.equal(a2, a) and torch.equal(m2, m) and torch.equal(v2, v) and torch.equal(t2, t)
    assert int(t2[0]) == 200
    s2.close()


def test_step_multi_equals_separate_steps():
    """A grouped step over handles of uneven shapes (three classes of several FP32 handles, an FP64
    handle, lone class members) equals separate steps bit for bit, and so do three steps in a row."""
    # the 64 x 64 handles with K <= 32 form a class on the compact tile; K = 33 stands alone
    specs = [(32, 9, 16, 24, "fp32", 2), (32, 7, 12, 20, "fp32", 1), (32, 11, 16, 24, "fp32", 3),
             (16, 7, 6, 8, "fp32", 2), (16, 5, 6, 8, "fp32", 1), (16, 7, 6, 8, "fp64", 2), (48, 9, 8, 12, "fp32", 1),
             (64, 15, 8, 12, "fp32", 1), (64, 9, 6, 10, "fp32", 2), (64, 33, 8, 12, "fp32", 1)]
    solvers, states = [], []
    for M, K, Ni, Ns, prec, B in specs:
        case = make_case(M, K, Ni, Ns, seeds=tuple(range(B)))
        s = solver_for(case, prec)
        solvers.append(s)
        a = s.init_alpha()
        states.append([a, *s.new_state()])
    ref = [[x.clone() for x in st] for st in states]
    for _ in range(3):
        pdf.step_multi(solvers, *[[st[k] for st in states] for k in range(4)])
        for s, st in zip(solvers, ref):
            s.step(*st)
    torch.cuda.synchronize()
    for st, rf in zip(states, ref):
        for x, y in zip(st, rf):
            assert torch.equal(x, y)
    with pytest.raises(pdf.PdfError):
        pdf.step_multi([solvers[0], solvers[0]], *[[st[k] for st in states[:1] * 2] for k in range(4)])
    for s in solvers:
        s.close()
