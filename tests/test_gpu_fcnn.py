"""GPU parity of the coefficient network (Sec. 3.1, Fig. 4; layer sizes are a reading): the
forward alpha_hat, loss, weight gradient and Adam steps of the HIP path against the FP64 oracle,
through the C ABI; ragged widths, one and 64 incidences, and the argument checks."""
import numpy as np
import pytest
import torch

import seeded_inputs as si
from oracle import fcnn as ofcnn, loss as oloss
from tests.common import make_case, rand_alpha
from tests.test_gpu_parity import DEV, oracle_terms, solver_for, term_tolerances

pytestmark = pytest.mark.gpu

pdf = pytest.importorskip("paper_2602_13805_amd")

CASES = [
    # (M, K, Ni, Ns, batch, hidden, precision, scaled): scaled = s_in 1 / rms(alpha_0), s_out 1 / H
    (16, 5, 6, 8, 2, 16, "fp64", False),      # widths below one column tile
    (32, 7, 12, 16, 2, 80, "fp64", True),     # D = 98, H = 80: ragged column and reduction tiles
    (16, 3, 1, 4, 3, 8, "fp64", True),        # one incidence per instance
    (32, 9, 33, 16, 1, 64, "fp32", False),    # 33 rows: the 16-rows-per-wave variant with a ragged last wave
    (16, 5, 64, 64, 1, 32, "fp32", True),     # largest incidence count
    (64, 15, 32, 32, 2, 256, "fp32", True),   # the benchmark shape (D = 450)
    (32, 7, 12, 16, 2, 80, "fp32", True),     # ragged hidden width on the matrix-core path
    (16, 5, 40, 24, 2, 48, "fp32", False),    # two 32-row MFMA tiles, the second ragged
]


def _rel_max(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(np.asarray(b))), 1e-300))


def _inputs(case, B, K, H, Ni, seed):
    a0 = np.stack([rand_alpha((Ni, K, K), scale=0.05, seed=40 + b) for b in range(B)])
    theta = si.fcnn_theta(seed, B, K, H, out_scale=0.2)
    return a0, theta


@pytest.mark.parametrize("M,K,Ni,Ns,B,H,prec,scaled", CASES)
def test_fcnn_steps_match_the_oracle(M, K, Ni, Ns, B, H, prec, scaled):
    print(f"case fcnn M={M} K={K} Ni={Ni} Ns={Ns} B={B} H={H} {prec} scaled={scaled}", flush=True)
    case = make_case(M, K, Ni, Ns, seeds=tuple(range(B)))
    s = solver_for(case, prec)
    P = s.fcnn_size(H)
    assert P == ofcnn.n_params(K, H)
    a0, theta = _inputs(case, B, K, H, Ni, seed=M + K + H)
    s_in, s_out = (1.0 / float(np.sqrt(np.mean(np.abs(a0) ** 2))), 1.0 / H) if scaled else (1.0, 1.0)
    a0d = torch.tensor(a0, dtype=s.cdtype, device=DEV)
    th = torch.tensor(theta, dtype=s.rdtype, device=DEV)
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    loss = torch.zeros((B, pdf.binding.LOSS_STRIDE), dtype=torch.float64, device=DEV)
    ref = [dict(theta=theta[b].copy(), m=np.zeros(P), v=np.zeros(P), th_err=0.0) for b in range(B)]
    n_steps = 3 if prec == "fp64" else 1
    for t in range(1, n_steps + 1):
        ah = s.fcnn_step(H, a0d, th, m, v, t, loss=loss, s_in=s_in, s_out=s_out).cpu().numpy()
        got_loss = loss.cpu().numpy()
        for b, c in enumerate(case["cases"]):
            r = ref[b]
            th_n, m_n, v_n, ah_ref, out = ofcnn.step(r["theta"], r["m"], r["v"], t, a0[b], c["prob"], K, H,
                                                     s_in=s_in, s_out=s_out)
            if prec == "fp64":
                e_ah = _rel_max(ah[b], ah_ref)
                assert e_ah < 1e-9, (t, b, e_ah)
                want = oracle_terms(out)   # (a term that is exactly zero, e.g. the state term of one incidence,
                #                            carries rounding relative to the total)
                assert np.all(np.abs(got_loss[b, :6] - want) <= 1e-9 * np.abs(want) + 1e-12 * abs(want[5])), t
                assert _rel_max(m.cpu().numpy()[b], m_n) < 1e-9, (t, b)
                assert _rel_max(v.cpu().numpy()[b], v_n) < 1e-9, (t, b)
                # the update lr1 m / (sqrt(v ic2) + eps) moves by about lr1 dm / (sqrt(v ic2) + eps) for an
                # error dm in m: near-zero gradients (|g| ~ eps) amplify a 1e-17 difference ~1e6 times
                lr1, ic2 = 1e-2 / (1 - 0.9 ** t), 1 / (1 - 0.999 ** t)
                tol_th = r["th_err"] + 1e-13 + 2 * lr1 * 1e-9 * np.max(np.abs(m_n)) / (np.sqrt(v_n * ic2) + 1e-8)
                err_th = np.abs(th.cpu().numpy()[b] - th_n)
                assert np.all(err_th <= tol_th), (t, b, float(np.max(err_th - tol_th)))
                r["th_err"] = err_th
            else:
                tt, tg = term_tolerances(out, prec, 1e-4)
                assert _rel_max(ah[b], ah_ref) < 1e-5, (t, b, _rel_max(ah[b], ah_ref))
                want = oracle_terms(out)
                assert np.all(np.abs(got_loss[b, :6] - want) <= tt * np.abs(want) + 1e-7 * abs(want[5]))
                # after the first step m = (1 - b1) dL/dtheta: the weight gradient itself
                md = m.cpu().numpy()[b]
                assert _rel_max(md, m_n) < tg, (b, _rel_max(md, m_n), tg)
                # the first Adam step is lr sign(g) wherever |g| >> eps; weights whose gradient is
                # below the FP32 noise of the largest one may take either sign
                g = m_n / 0.1
                strong = np.abs(g) > 1e-2 * np.max(np.abs(g))
                d = np.abs(th.cpu().numpy()[b] - th_n)
                assert np.max(d[strong]) < 1e-6, np.max(d[strong])
                assert np.max(d) <= 2.0 * 1e-2 * (1 + 1e-6)
            r.update(theta=th_n, m=m_n, v=v_n)
    s.close()


def test_fcnn_step_with_adam_state_fp32():
    """Step 3 of the benchmark shape from the oracle's state after two steps: moments, weights
    and alpha_hat of a step whose v is no longer a copy of g^2."""
    M, K, Ni, Ns, B, H = 64, 15, 32, 32, 1, 128
    print("case fcnn fp32 step 3 from the oracle's state", flush=True)
    case = make_case(M, K, Ni, Ns, seeds=(0,))
    c = case["cases"][0]
    a0, theta = _inputs(case, B, K, H, Ni, seed=7)
    P = ofcnn.n_params(K, H)
    sc = dict(s_in=1.0 / float(np.sqrt(np.mean(np.abs(a0) ** 2))), s_out=1.0 / H)
    th, m, v = theta[0].copy(), np.zeros(P), np.zeros(P)
    for t in (1, 2):
        th, m, v, _, _ = ofcnn.step(th, m, v, t, a0[0], c["prob"], K, H, **sc)
    th3, m3, v3, ah3, out3 = ofcnn.step(th, m, v, 3, a0[0], c["prob"], K, H, **sc)
    s = solver_for(case, "fp32")
    td = torch.tensor(th[None], dtype=torch.float32, device=DEV)
    mdv = torch.tensor(m[None], dtype=torch.float32, device=DEV)
    vdv = torch.tensor(v[None], dtype=torch.float32, device=DEV)
    ah = s.fcnn_step(H, torch.tensor(a0, dtype=s.cdtype, device=DEV), td, mdv, vdv, 3, **sc).cpu().numpy()[0]
    _, tg = term_tolerances(out3, "fp32", 1e-4)
    assert _rel_max(ah, ah3) < 1e-5
    assert _rel_max(mdv.cpu().numpy()[0], m3) < tg
    assert _rel_max(vdv.cpu().numpy()[0], v3) < 2 * tg
    # the update is lr m_hat / (sqrt(v_hat) + eps): its error follows that of m relative to sqrt(v)
    step_ref = th - th3
    step_dev = th - td.cpu().numpy()[0].astype(np.float64)
    big = np.abs(step_ref) > 1e-3 * 1e-2
    assert _rel_max(step_dev[big], step_ref[big]) < 50 * tg
    s.close()


def test_fcnn_forward_zero_output_layer_is_alpha0_and_full_size_forward():
    case = make_case(64, 15, 32, 32, seeds=(0, 1))
    s = solver_for(case, "fp32")
    H = 256
    a0 = np.stack([rand_alpha((32, 15, 15), scale=0.05, seed=70 + b) for b in range(2)])
    a0d = torch.tensor(a0, dtype=s.cdtype, device=DEV)
    th0 = torch.tensor(si.fcnn_theta(3, 2, 15, H, out_scale=0.0), dtype=torch.float32, device=DEV)
    assert torch.equal(s.fcnn_forward(H, a0d, th0), a0d)
    theta = si.fcnn_theta(4, 2, 15, H, out_scale=1.0)
    for s_in, s_out in ((1.0, 1.0), (30.0, 1.0 / H)):
        ah = s.fcnn_forward(H, a0d, torch.tensor(theta, dtype=torch.float32, device=DEV), s_in, s_out).cpu().numpy()
        for b in range(2):
            ref = ofcnn.forward(theta[b], a0[b], 15, H, s_in, s_out)[0]
            assert _rel_max(ah[b] - a0[b], ref - a0[b]) < 1e-5
    s.close()


def test_fcnn_argument_checks():
    case = make_case(16, 5, 6, 8, seeds=(0,))
    s = solver_for(case, "fp32")
    a0 = torch.zeros(s.alpha_shape, dtype=s.cdtype, device=DEV)
    th = torch.zeros((1, s.fcnn_size(8)), dtype=torch.float32, device=DEV)
    with pytest.raises(pdf.PdfError) as e:
        s.fcnn_size(0)
    assert e.value.code == pdf.binding.PDF_EINVAL
    lib = pdf.binding.load()
    p = pdf.binding._ptr
    out = torch.empty_like(a0)
    assert lib.pdf_fcnn_forward(s.h, 8, 1.0, 1.0, p(a0), p(th), p(a0)) == pdf.binding.PDF_EINVAL   # alias
    assert lib.pdf_fcnn_step(s.h, 8, 1.0, 1.0, p(a0), p(th), p(th), p(th), 0, p(out), None) \
        == pdf.binding.PDF_EINVAL                                                                  # t = 0
    assert lib.pdf_fcnn_forward(s.h, 5000, 1.0, 1.0, p(a0), p(th), p(out)) == pdf.binding.PDF_EINVAL
    assert lib.pdf_fcnn_forward(s.h, 8, float("nan"), 1.0, p(a0), p(th), p(out)) == pdf.binding.PDF_EINVAL
    s.close()


def test_fcnn_step_batch_of_256_sampled():
    """The network leg's configuration (cfg2, 256 instances, H = 256, the benchmark's scales): one
    step, alpha_hat, loss terms and weight gradient of sampled instances against the oracle."""
    M, K, Ni, Ns, B, H = 64, 15, 32, 32, 256, 256
    sample = (0, 128, 255)
    print("case fcnn B=256 H=256 sampled", sample, flush=True)
    case = make_case(M, K, Ni, Ns, seeds=(0,))
    rng = np.random.default_rng(77)
    es = 0.1 * (rng.standard_normal((B, Ni, Ns)) + 1j * rng.standard_normal((B, Ni, Ns)))
    a0 = np.stack([rand_alpha((Ni, K, K), scale=0.02, seed=500 + b) for b in range(B)])
    theta = si.fcnn_theta(9, B, K, H, out_scale=0.2)
    s_in, s_out = 1.0 / float(np.sqrt(np.mean(np.abs(a0) ** 2))), 1.0 / H
    s = pdf.Solver(M, case["wl"].side, case["wl"].freq_hz, case["tx"], case["rx"], K, batch=B, device=DEV)
    s.set_data(torch.tensor(es, dtype=s.cdtype, device=DEV))
    th = torch.tensor(theta, dtype=torch.float32, device=DEV)
    m, v = torch.zeros_like(th), torch.zeros_like(th)
    loss = torch.zeros((B, pdf.binding.LOSS_STRIDE), dtype=torch.float64, device=DEV)
    ah = s.fcnn_step(H, torch.tensor(a0, dtype=s.cdtype, device=DEV), th, m, v, 1, loss=loss, s_in=s_in,
                     s_out=s_out).cpu().numpy()
    got_loss, md = loss.cpu().numpy(), m.cpu().numpy()
    for b in sample:
        prob = oloss.build_problem(M, K, case["wl"].side, [case["wl"].freq_hz], case["tx"], case["rx"], es[b])
        _, m_n, _, ah_ref, out = ofcnn.step(theta[b], np.zeros(theta.shape[1]), np.zeros(theta.shape[1]), 1, a0[b],
                                            prob, K, H, s_in=s_in, s_out=s_out)
        tt, tg = term_tolerances(out, "fp32", 1e-4)
        assert _rel_max(ah[b], ah_ref) < 1e-5, b
        want = oracle_terms(out)
        assert np.all(np.abs(got_loss[b, :6] - want) <= tt * np.abs(want) + 1e-7 * abs(want[5])), b
        assert _rel_max(md[b], m_n) < tg, (b, _rel_max(md[b], m_n))
    s.close()
