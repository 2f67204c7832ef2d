"""GPU parity of reconstructions measured at several frequencies (one contrast, per-frequency
coefficients, currents and operators; R the least-squares contrast over all frequencies with each
weighted by 1/||E_inc,f||^2; L^State and L^Data summed over frequencies), against the oracle's
multi-frequency loss, start value and Adam steps: FP64 within 1e-9, FP32 within 1e-4 (the
chi-dependent terms within the conditioning-scaled bound).  The LDS-resident convolution (32^2)
and the multi-pass one (96^2 FP64, 128^2 FP32), two to four frequencies."""
import numpy as np
import pytest
import torch

import seeded_inputs as si
from oracle import adam, forward, init as oinit, loss as oloss, operators as ops
from tests.common import geometry, rand_alpha, rel
from tests.test_gpu_parity import DEV, check_grad, oracle_terms, term_tolerances

pytestmark = pytest.mark.gpu

pdf = pytest.importorskip("paper_2602_13805_amd")


def _mf_case(M, K, Ni, Ns, mults, seed=0, fine=2):
    wl = si.WORKLOADS["cfg1"]
    freqs = [wl.freq_hz * m for m in mults]
    tx, rx = geometry(Ni, Ns)
    shapes = si.draw_profile(wl, seed)
    epsf = si.rasterize(shapes, fine * M, wl.side)
    es = []
    for f, fr in enumerate(freqs):
        e, _ = forward.mom_solve(epsf, wl.side, ops.wavenumber(fr), tx, rx)
        n1, n2 = si.draw_noise(seed + 17 * f, e.shape)
        es.append(forward.add_noise(e, 0.05, n1, n2))
    es = np.array(es)
    prob = oloss.build_problem(M, K, wl.side, freqs, tx, rx, es)
    return wl, freqs, tx, rx, es, prob


MF = [  # M, K, Ni, Ns, frequency multiples, precision, tol
    (32, 9, 8, 12, (1.0, 1.5, 2.0), "fp64", 1e-9),
    (32, 9, 8, 12, (1.0, 1.5), "fp32", 1e-4),
    (16, 7, 5, 6, (1.0, 1.25, 1.5, 2.0), "fp64", 1e-9),
    (96, 13, 4, 6, (1.0, 2.0), "fp64", 1e-9),
    (128, 21, 6, 8, (1.0, 1.5), "fp32", 1e-4),
]


@pytest.mark.parametrize("M,K,Ni,Ns,mults,prec,tol", MF)
def test_multifrequency_loss_grad_start_and_steps(M, K, Ni, Ns, mults, prec, tol):
    print(f"case multi-frequency M={M} K={K} Ni={Ni} Ns={Ns} F={len(mults)} {prec}", flush=True)
    wl, freqs, tx, rx, es, prob = _mf_case(M, K, Ni, Ns, mults, fine=1 if M > 64 else 2)
    F = len(freqs)
    s = pdf.Solver(M, wl.side, freqs, tx, rx, K, batch=1, params=pdf.default_params(prec), device=DEV)
    assert s.F == F and s.Ni == F * Ni
    s.set_data(torch.tensor(es.reshape(1, F * Ni, Ns), dtype=s.cdtype, device=DEV))
    # loss and gradient at random coefficients
    alpha = rand_alpha((F, Ni, K, K), scale=0.05 * 32.0 / M, seed=4)
    lo, g = s.loss_grad(torch.tensor(alpha.reshape(1, F * Ni, K, K), dtype=s.cdtype, device=DEV))
    ref = oloss.evaluate(alpha, prob)
    want, got = oracle_terms(ref), lo.cpu().numpy()[0, :6]
    tt, tg = term_tolerances(ref, prec, tol)
    print(f"  terms rel {np.abs(got - want) / np.abs(want)}", flush=True)
    assert np.all(np.abs(got - want) <= tt * np.abs(want) + tol * 1e-3 * abs(want[5])), (got, want)
    check_grad(g.cpu().numpy()[0].reshape(F, Ni, K, K), ref["g_alpha"], tg)
    # the start value: joint back-propagation contrast, one line-search step on the summed L^CSI
    a0 = s.init_alpha()
    r0, _ = oinit.alpha0(prob)
    e0 = rel(a0.cpu().numpy()[0].reshape(F, Ni, K, K), r0)
    print(f"  start rel {e0:.1e}", flush=True)
    assert e0 < (1e-9 if prec == "fp64" else 1e-5)
    # Adam steps from the device's start: FP64 against the oracle's trajectory (5 steps); FP32 the
    # first step against the bias-corrected update of the device's own gradient (the first step
    # takes the sign of every gradient entry, which FP32 rounding may flip where an entry is ~0)
    a = a0.clone()
    m, v, t = s.new_state()
    x = a0.cpu().numpy()[0].reshape(F, Ni, K, K).astype(np.complex128)
    mm, vv = np.zeros(x.shape + (2,)), np.zeros(x.shape + (2,))
    nsteps = 5 if prec == "fp64" else 1
    g_dev = s.loss_grad(a0)[1].cpu().numpy()[0].reshape(F, Ni, K, K).astype(np.complex128)
    for k in range(1, nsteps + 1):
        s.step(a, m, v, t)
        gk = oloss.evaluate(x, prob)["g_alpha"] if prec == "fp64" else g_dev
        x, mm, vv = adam.adam_step(x, gk, mm, vv, k)
    e = np.max(np.abs(a.cpu().numpy()[0].reshape(F, Ni, K, K) - x)) / np.max(np.abs(x))
    print(f"  after {nsteps} Adam steps rel {e:.1e}", flush=True)
    assert e < (1e-8 if prec == "fp64" else 1e-5)
    assert int(t[0]) == nsteps
    s.close()


def test_multifrequency_duplicate_frequency_doubles_the_physics_terms():
    """Two copies of one frequency with the same data: R and chi are those of one frequency, so
    the state and data terms double and the regularisers stay."""
    wl, freqs, tx, rx, es, prob = _mf_case(32, 9, 8, 12, (1.0,))
    one = pdf.Solver(32, wl.side, freqs[0], tx, rx, 9, batch=1, params=pdf.default_params("fp64"), device=DEV)
    two = pdf.Solver(32, wl.side, [freqs[0], freqs[0]], tx, rx, 9, batch=1, params=pdf.default_params("fp64"),
                     device=DEV)
    one.set_data(torch.tensor(es.reshape(1, 8, 12), dtype=one.cdtype, device=DEV))
    two.set_data(torch.tensor(np.concatenate([es, es]).reshape(1, 16, 12), dtype=two.cdtype, device=DEV))
    alpha = rand_alpha((8, 9, 9), 0.05, seed=2)
    l1, _ = one.loss_grad(torch.tensor(alpha[None], dtype=one.cdtype, device=DEV), grad=False)
    l2, _ = two.loss_grad(torch.tensor(np.concatenate([alpha, alpha])[None], dtype=two.cdtype, device=DEV),
                          grad=False)
    l1, l2 = l1.cpu().numpy()[0], l2.cpu().numpy()[0]
    assert np.allclose(l2[:2], 2 * l1[:2], rtol=1e-12) and np.allclose(l2[2:5], l1[2:5], rtol=1e-10)
    # the entry points that cover one frequency refuse the container
    with pytest.raises(pdf.PdfError):
        two.init_alpha_csi(2)
    one.close()
    two.close()


def test_multifrequency_reconstruction_runs_from_a_graph():
    wl, freqs, tx, rx, es, prob = _mf_case(32, 9, 8, 12, (1.0, 1.5))
    s = pdf.Solver(32, wl.side, freqs, tx, rx, 9, batch=1, params=pdf.default_params("fp32"), device=DEV)
    s.set_data(torch.tensor(es.reshape(1, 16, 12), dtype=s.cdtype, device=DEV))
    eps = si.rasterize(si.draw_profile(wl, 0), 32, wl.side)
    r = s.reconstruct(40, n_check=10, eps_true=torch.tensor(eps[None], dtype=s.cdtype, device=DEV))
    # the same 40 steps eagerly from the same start give the same coefficients
    a = s.init_alpha()
    m, v, t = s.new_state()
    for _ in range(40):
        s.step(a, m, v, t)
    assert torch.equal(a, r["alpha"])
    assert np.isfinite(r["best_err"].item())
    s.close()
