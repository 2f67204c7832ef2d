"""Adjoint (dot-product) tests of the device's own linear operators, through the C ABI
(pdf_apply): the basis synthesis B (Sec. 2.3, Eq. 9) against the analysis of the adjoint kernel,
the domain operator composed with it, G_D B (Sec. 2.1, Eq. 3), against B^H G_D^H of the adjoint
convolution (conj of the spectrum), G_D from currents against its own symmetry (G_D^T = G_D),
and the receiver GEMM G_S (Sec. 2.1, Eq. 4) against the G_S^H GEMM:
<A x, y> = <x, A^H y> within tol ||A x|| ||y||.  Each forward operator is also compared with the
FP64 oracle's."""
import numpy as np
import pytest
import torch

from oracle import fourier, operators as ops
from tests.common import make_case, rel
from tests.test_gpu_parity import DEV

pytestmark = pytest.mark.gpu

pdf = pytest.importorskip("paper_2602_13805_amd")


def _rand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _dot(a, b):
    return np.vdot(b, a)   # <a, b> = sum a conj(b)


CASES = [  # M, K, Ni, Ns, B, precision
    (16, 7, 6, 8, 2, "fp64"),
    (32, 14, 12, 20, 2, "fp64"),     # corner blocks, ragged receiver tiles
    (64, 15, 4, 8, 1, "fp64"),
    (32, 9, 16, 24, 2, "fp32"),
    (48, 13, 12, 20, 1, "fp32"),
    (64, 15, 32, 32, 2, "fp32"),     # the benchmark's shape
    (96, 21, 8, 16, 1, "fp32"),
]


@pytest.mark.parametrize("M,K,Ni,Ns,B,prec", CASES)
def test_adjoint_dot_products_and_operator_parity(M, K, Ni, Ns, B, prec):
    print(f"case adjoint M={M} K={K} Ni={Ni} Ns={Ns} B={B} {prec}", flush=True)
    case = make_case(M, K, Ni, Ns, seeds=(0,))
    wl = case["wl"]
    s = pdf.Solver(M, wl.side, wl.freq_hz, case["tx"], case["rx"], K, batch=B,
                   params=pdf.default_params(prec), device=DEV)
    tol_dot, tol_op = (1e-13, 1e-12) if prec == "fp64" else (1e-5, 1e-5)
    prob = case["cases"][0]["prob"]
    rng = np.random.default_rng(M * 100 + K)
    dev = lambda a: torch.tensor(a, dtype=s.cdtype, device=DEV)
    host = lambda t: t.cpu().numpy().astype(np.complex128)
    a = _rand(rng, (B, Ni, K, K))
    J = _rand(rng, (B, Ni, M, M))
    y = _rand(rng, (B, Ni, M, M))
    d = _rand(rng, (B, Ni, Ns))
    # what the device computes in FP32 is its input rounded; the oracle takes the same values
    a, J, y, d = (host(dev(v)) for v in (a, J, y, d))

    def check(Ax, x, AHy, yy, name):
        lhs, rhs = _dot(Ax, yy), _dot(x, AHy)
        scale = np.linalg.norm(Ax) * np.linalg.norm(yy)
        print(f"  {name}: |<Ax,y> - <x,A^H y>| / (|Ax||y|) = {abs(lhs - rhs) / scale:.2e}", flush=True)
        assert abs(lhs - rhs) <= tol_dot * scale, name

    Ba = host(s.apply("synth", dev(a)))
    BHy = host(s.apply("synth_adj", dev(y)))
    check(Ba, a, BHy, y, "B")
    assert rel(Ba, fourier.synthesize(a, M)) < tol_op
    assert rel(BHy, fourier.synth_adjoint(y, K)) < tol_op

    GBa = host(s.apply("gd_synth", dev(a)))
    BGHy = host(s.apply("gd_synth_adj", dev(y)))
    check(GBa, a, BGHy, y, "G_D B")
    ghat = prob.ghat[0]
    assert rel(GBa, ops.gd_apply(fourier.synthesize(a, M), ghat)) < tol_op
    assert rel(BGHy, fourier.synth_adjoint(ops.gd_adjoint_apply(y, ghat), K)) < tol_op

    GJ = host(s.apply("gd", dev(J)))
    GHy = np.conj(host(s.apply("gd", dev(np.conj(y)))))
    check(GJ, J, GHy, y, "G_D")
    assert rel(GJ, ops.gd_apply(J, ghat)) < tol_op

    GSJ = host(s.apply("gs", dev(J)))
    GSHd = host(s.apply("gs_adj", dev(d)))
    check(GSJ, J, GSHd, d, "G_S")
    gs = prob.gs[0]
    assert rel(GSJ, J.reshape(B, Ni, M * M) @ gs.T) < tol_op
    assert rel(GSHd, (d @ np.conj(gs)).reshape(B, Ni, M, M)) < tol_op
    with pytest.raises(pdf.PdfError):
        x = dev(J)
        pdf.binding.load()
        s._call(pdf.binding.load().pdf_apply, 9, pdf.binding._ptr(x), pdf.binding._ptr(x))
    s.close()
