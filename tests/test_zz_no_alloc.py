"""The CSI start through the entry point that allocates nothing (its workspace is the
library's static device scratch) against pdf_init_alpha_csi, bit for bit: two calls in a
row on different handles, the second with a smaller input, then a request too large for
the scratch, which is refused before any work."""
import numpy as np
import pytest
import torch

from tests.common import make_case
from tests.test_gpu_parity import solver_for

pytestmark = pytest.mark.gpu

pdf = pytest.importorskip("paper_2602_13805_amd")


def _check_case(M, K, Ni, Ns, B, prec, n_iter):
    print(f"case no-alloc csi M={M} K={K} Ni={Ni} Ns={Ns} B={B} {prec} n_iter={n_iter}", flush=True)
    case = make_case(M, K, Ni, Ns, seeds=tuple(range(B)))
    s = solver_for(case, prec)
    ref = s.init_alpha_csi(n_iter)
    out = torch.full(s.alpha_shape, float("nan"), dtype=s.cdtype, device="cuda:0")
    s.init_alpha_csi_noalloc(n_iter, out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref), float((out - ref).abs().max())
    s.close()
    return ref


def test_no_alloc_csi_equals_the_allocating_entry_point():
    # larger input first, then a smaller one: the second call reuses the scratch the
    # first left behind
    _check_case(32, 9, 16, 24, 3, "fp32", 6)
    _check_case(16, 7, 6, 8, 2, "fp32", 4)
    _check_case(16, 7, 6, 8, 2, "fp64", 3)


def test_no_alloc_csi_refuses_a_workspace_beyond_the_scratch():
    # FP32, B = 17, Ni = 64, K = 63: 17 * 64 * 63^2 * 8 bytes = 34.5 MB > 32 MiB
    M, K, Ni, B = 64, 63, 64, 17
    need = 8 * B * Ni * K * K
    assert need > 32 * 2 ** 20
    tx = np.stack([np.cos(2 * np.pi * np.arange(Ni) / Ni), np.sin(2 * np.pi * np.arange(Ni) / Ni)], 1) * 2.25
    s = pdf.Solver(M, 1.5, 400e6, tx, tx[:16], K, batch=B, device="cuda:0")
    rng = np.random.default_rng(3)
    es = rng.standard_normal((B, Ni, 16)) + 1j * rng.standard_normal((B, Ni, 16))
    s.set_data(torch.tensor(es, dtype=s.cdtype, device="cuda:0"))
    out = torch.zeros(s.alpha_shape, dtype=s.cdtype, device="cuda:0")
    with pytest.raises(pdf.PdfError) as ei:
        s.init_alpha_csi_noalloc(2, out)
    assert ei.value.code == pdf.binding.PDF_EINVAL and "static scratch" in str(ei.value)
    s.close()
