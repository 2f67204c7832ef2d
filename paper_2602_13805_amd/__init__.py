"""MI355X-native hot path of the Physics-Driven Fourier-Spectral (PDF) solver.

The HIP library ``libpdf.so`` (sources in ``csrc/``, C ABI in ``include/pdf.h``)
does all computation; ``binding`` marshals PyTorch device tensors into it.

A ``Solver`` holds one measurement geometry and a batch of data sets:
``set_data`` (measured fields), ``init_alpha`` / ``init_alpha_csi`` (start
values), ``loss_grad`` and ``step`` (one loss + gradient, one Adam step on the
coefficients), ``reconstruct`` (graph-replayed iterations with image-error
tracking), ``image`` (contrast and CCO image), ``fcnn_step`` / ``fcnn_forward``
(the coefficient network: Adam on its weights instead of on the coefficients),
``warm_start`` (a trained ``Mlp``'s start value).  ``reconstruct_multi``
advances solvers of different shapes together; ``synthesize`` and
``synthesize_batch`` compute measured fields by FP64 MoM.
"""
from .binding import (FP32, FP64, LOSS_NAMES, LOSS_STRIDE, Mlp, PdfError, PdfLoss, Solver, default_params,
                      mean_abs2,
                      load, reconstruct_multi, step_multi, synthesize, synthesize_batch, tables_host)

__all__ = ["FP32", "FP64", "LOSS_NAMES", "LOSS_STRIDE", "Mlp", "PdfError", "PdfLoss", "Solver", "default_params",
           "mean_abs2",
           "load", "reconstruct_multi", "step_multi", "synthesize", "synthesize_batch", "tables_host"]
