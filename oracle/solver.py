"""One PDF reconstruction (Sec. 3, Fig. 3): start value, Adam on the
coefficients with the composite loss, then R -> chi -> CCO.

The paper's network predicts a correction Delta alpha that is added to
alpha_0; with only its output trained this is Adam directly on alpha, which
is what is iterated here.
"""
from __future__ import annotations

import numpy as np

from . import adam, cco, init, loss


def reconstruct(prob: loss.Problem, n_iter: int, alpha_start=None, lr=1e-2,
                eps_true=None, check_every: int = 0):
    if alpha_start is None:
        alpha_start, _ = init.alpha0(prob)
    alpha = np.array(alpha_start, dtype=np.complex128)
    if alpha.ndim == 3:
        alpha = alpha[None]
    m = np.zeros(alpha.shape + (2,))
    v = np.zeros(alpha.shape + (2,))
    hist, errs = [], []
    for t in range(1, n_iter + 1):
        out = loss.evaluate(alpha, prob)
        hist.append(out["L"])
        if eps_true is not None and check_every and (t - 1) % check_every == 0:
            errs.append((t - 1, cco.image_error(cco.cco(out["chi"]), eps_true)))
        alpha, m, v = adam.adam_step(alpha, out["g_alpha"], m, v, t, lr=lr)
    final = loss.evaluate(alpha, prob, grad=False)
    img = cco.cco(final["chi"])
    res = dict(alpha=alpha, m=m, v=v, loss=np.array(hist), chi=final["chi"], chi_cco=img,
               final=final)
    if eps_true is not None:
        res["err"] = cco.image_error(img, eps_true)
        res["err_hist"] = errs
    return res
