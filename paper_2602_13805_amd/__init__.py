"""MI355X-native hot path of the Physics-Driven Fourier-Spectral (PDF) solver.

The HIP library ``libpdf.so`` (sources in ``csrc/``, C ABI in ``include/pdf.h``)
does all computation; ``binding`` marshals PyTorch device tensors into it.
"""
from .binding import (FP32, FP64, LOSS_NAMES, LOSS_STRIDE, Mlp, PdfError, PdfLoss, Solver, default_params,
                      load, reconstruct_multi, synthesize, synthesize_batch, tables_host)

__all__ = ["FP32", "FP64", "LOSS_NAMES", "LOSS_STRIDE", "Mlp", "PdfError", "PdfLoss", "Solver", "default_params",
           "load", "reconstruct_multi", "synthesize", "synthesize_batch", "tables_host"]
