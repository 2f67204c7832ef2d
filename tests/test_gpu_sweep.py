"""The hyper-parameter sweep of Sec. 4.1-4.2.1 (beta, M_F, noise) as one grouped launch: the
contraction parameter beta = 3 and 9 against the oracle (every other parity case runs the paper's
beta = 6), and handles that differ only in beta and the truncation K, advanced together by the
grouped kernels, bit for bit equal to each handle alone."""
import numpy as np
import pytest
import torch

from oracle import loss as oloss
from tests.common import make_case, rand_alpha
from tests.test_gpu_parity import DEV, check_grad, oracle_terms, solver_for, term_tolerances

pytestmark = pytest.mark.gpu

pdf = pytest.importorskip("paper_2602_13805_amd")


@pytest.mark.parametrize("beta", [3.0, 9.0])
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("fp64", 1e-9)])
def test_loss_grad_parity_other_beta(beta, prec, tol):
    M, K, Ni, Ns, B = 32, 14, 8, 12, 2   # K = 2 M_F with M_F = 7: the paper's corner blocks
    print(f"case beta={beta} {prec}", flush=True)
    case = make_case(M, K, Ni, Ns, seeds=(0, 1), params=oloss.Params(beta=beta))
    s = solver_for(case, prec, beta=beta)
    alpha = np.stack([rand_alpha((Ni, K, K), seed=20 + b) for b in range(B)])
    loss, g = s.loss_grad(torch.tensor(alpha, dtype=s.cdtype, device=DEV))
    loss, g = loss.cpu().numpy(), g.cpu().numpy()
    for b, c in enumerate(case["cases"]):
        ref = oloss.evaluate(alpha[b], c["prob"])
        want = oracle_terms(ref)
        tt, tg = term_tolerances(ref, prec, tol)
        assert np.all(np.abs(loss[b, :6] - want) <= tt * np.abs(want) + tol * 1e-3 * abs(want[5])), (b, loss[b], want)
        check_grad(g[b], ref["g_alpha"], tg)
    s.close()


def test_grouped_sweep_equals_separate_runs():
    """beta in {3, 6, 9} x K in {10, 13} (even K: corner blocks) on one geometry: one shape class,
    so one grouped launch per kernel; each handle's trajectory equals its own run bit for bit."""
    M, Ni, Ns, B = 32, 16, 16, 2
    sol, eps = [], []
    for beta in (3.0, 6.0, 9.0):
        for K in (10, 13):
            case = make_case(M, K, Ni, Ns, seeds=(int(beta), int(beta) + 1), params=oloss.Params(beta=beta))
            s = solver_for(case, "fp32", beta=beta)
            sol.append(s)
            eps.append(torch.tensor(np.stack([c["eps"] for c in case["cases"]]), dtype=s.cdtype, device=DEV))
    print("grouped sweep: 6 handles, one class", flush=True)
    ref = [s.reconstruct(30, n_check=10, eps_true=e) for s, e in zip(sol, eps)]
    got, _ = pdf.reconstruct_multi(sol, 30, n_check=10, eps_trues=eps)
    for r, g in zip(ref, got):
        assert torch.equal(r["alpha"], g["alpha"])
        assert torch.equal(r["best_err"], g["best_err"]) and torch.equal(r["best_iter"], g["best_iter"])
        assert torch.equal(r["chi_cco"], g["chi_cco"])
    for s in sol:
        s.close()
