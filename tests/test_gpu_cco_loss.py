"""GPU parity of the loss evaluated on the CCO image (pdf_params.cco_in_loss = 1; Sec. 2.4,
Eqs. 10-11 inside the loss of Sec. 3.2, Eqs. 13-19) against the FP64 oracle, through the C ABI.

FP64: every loss term and the gradient within 1e-9 of the oracle at random coefficients on 16^2 to
64^2 grids, twelve Adam steps along the oracle's trajectory, R held fixed (r_stopgrad), and the
loss-only pass equal to the full pass bit for bit.  FP32: physical inputs (cfg2-style profiles, MoM
fields with jitter and noise) at the device's start value and after ten of its Adam steps, every
term and gradient entry within a flat 1e-4 (the same bar as the plain loss on such inputs)."""
import dataclasses

import numpy as np
import pytest
import torch

import seeded_inputs as si
from oracle import adam as oadam, forward, loss as oloss, operators as ops
from tests.common import make_case, rand_alpha, rel
from tests.test_gpu_parity import DEV, chi_condition, oracle_terms, solver_for

pytestmark = pytest.mark.gpu

pdf = pytest.importorskip("paper_2602_13805_amd")

CCO = oloss.Params(cco_in_loss=True)


def _check(loss, g, a, probs, tol, label, r_stopgrad=False):
    for b, prob in enumerate(probs):
        ref = oloss.evaluate(a[b], prob, r_stopgrad=r_stopgrad)
        want, got = oracle_terms(ref), loss[b, :6]
        err_t = np.abs(got - want) / np.maximum(np.abs(want), 1e-8 * abs(want[5]))
        gr = ref["g_alpha"]
        err_g = np.max(np.abs(g[b] - gr)) / np.max(np.abs(gr))
        print(f"  {label} b={b}: kappa {chi_condition(ref):.1f}, |chi_c - chi| {np.max(np.abs(ref['chi_c'] - ref['chi'])):.2e}, "
              f"terms {np.array2string(err_t, precision=1)}, gradient {err_g:.1e} (rel {rel(g[b], gr):.1e})", flush=True)
        assert loss[b, 7] == 0.0
        assert np.all(err_t <= tol), (label, b, err_t)
        assert err_g <= tol, (label, b, err_g)


@pytest.mark.parametrize("M,K,Ni,Ns,B", [(16, 7, 6, 8, 2), (32, 9, 16, 20, 2), (48, 13, 8, 12, 1), (64, 15, 8, 12, 1)])
def test_cco_loss_grad_fp64(M, K, Ni, Ns, B):
    print(f"case cco_in_loss M={M} K={K} Ni={Ni} Ns={Ns} B={B} fp64", flush=True)
    case = make_case(M, K, Ni, Ns, seeds=tuple(range(B)), params=CCO)
    s = solver_for(case, "fp64", cco_in_loss=1)
    alpha = np.stack([rand_alpha((Ni, K, K), seed=40 + b) for b in range(B)])
    loss, g = s.loss_grad(torch.tensor(alpha, dtype=s.cdtype, device=DEV))
    probs = [c["prob"] for c in case["cases"]]
    _check(loss.cpu().numpy(), g.cpu().numpy(), alpha, probs, 1e-9, f"M={M}")
    # the loss-only pass (no adjoint) gives the same loss bit for bit
    l2, _ = s.loss_grad(torch.tensor(alpha, dtype=s.cdtype, device=DEV), grad=False)
    assert torch.equal(l2, loss)
    s.close()


def test_cco_loss_r_stopgrad_fp64():
    print("case cco_in_loss with R held fixed, 32x32 fp64", flush=True)
    case = make_case(32, 9, 12, 16, seeds=(0, 1), params=CCO)
    s = solver_for(case, "fp64", cco_in_loss=1, r_stopgrad=1)
    alpha = np.stack([rand_alpha((12, 9, 9), seed=50 + b) for b in range(2)])
    loss, g = s.loss_grad(torch.tensor(alpha, dtype=s.cdtype, device=DEV))
    _check(loss.cpu().numpy(), g.cpu().numpy(), alpha, [c["prob"] for c in case["cases"]], 1e-9, "r_stopgrad",
           r_stopgrad=True)
    s.close()


def test_cco_loss_adam_steps_fp64():
    print("case cco_in_loss 12 Adam steps, 32x32 fp64", flush=True)
    case = make_case(32, 9, 8, 12, seeds=(2, 3), params=CCO)
    s = solver_for(case, "fp64", cco_in_loss=1)
    a = s.init_alpha()
    alpha0 = a.cpu().numpy().copy()
    m, v, t = s.new_state()
    loss = torch.zeros((2, 8), dtype=torch.float64, device=DEV)
    for _ in range(12):
        s.step(a, m, v, t, loss)
    for b, c in enumerate(case["cases"]):
        x = alpha0[b].copy()
        mm = np.zeros(x.shape + (2,))
        vv = np.zeros(x.shape + (2,))
        for k in range(1, 13):
            last = oloss.evaluate(x, c["prob"])
            x, mm, vv = oadam.adam_step(x, last["g_alpha"], mm, vv, k)
        assert rel(a[b].cpu().numpy(), x) < 1e-9, rel(a[b].cpu().numpy(), x)
        assert abs(loss[b, 5].item() - last["L"]) < 1e-9 * last["L"]
    s.close()


def _physical(M, n_ant, K, seeds):
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
        probs.append(oloss.build_problem(M, K, wl.side, [wl.freq_hz], tx, rx, e, CCO))
    params = pdf.default_params("fp32", cco_in_loss=1)
    s = pdf.Solver(M, wl.side, wl.freq_hz, tx, rx, K, batch=len(seeds), params=params, device=DEV)
    s.set_data(torch.tensor(np.stack(es), dtype=s.cdtype, device=DEV))
    return s, probs


@pytest.mark.parametrize("M,n_ant,K", [(32, 16, 9), (64, 32, 15)])
def test_cco_loss_fp32_physical(M, n_ant, K):
    print(f"case cco_in_loss fp32 physical M={M} antennas={n_ant} K={K}", flush=True)
    s, probs = _physical(M, n_ant, K, seeds=(0, 1))
    a = s.init_alpha()
    for label, n in (("start", 0), ("after 10 Adam steps", 10)):
        if n:
            m, v, t = s.new_state()
            for _ in range(n):
                s.step(a, m, v, t)
        loss, g = s.loss_grad(a.contiguous())
        _check(loss.cpu().numpy(), g.cpu().numpy(), a.cpu().numpy().astype(np.complex128), probs, 1e-4,
               f"M={M} {label}")
    s.close()
