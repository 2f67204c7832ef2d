"""Start value of the coefficients (Sec. 3.1, Eq. 12 and the paragraph around it).

1. Back-propagation image: for incidence p, J_p = gamma_p G_S^H e_p with
   e_p the measured field and gamma_p = (v^H e_p)/(v^H v), v = G_S G_S^H e_p,
   the scalar that best fits the data.  The paper cites BP without details;
   this is the textbook form.
2. E_p = E_inc_p + G_D J_p; chi_0 = sum J conj(E) / sum |E|^2 per pixel;
   R_0 = beta chi_0 / (beta chi_0 + 1) (Eq. 7).
3. alpha_0 = one gradient step on L^CSI (Eq. 12, R fixed at R_0) from zero,
   with the exact line-search step of that quadratic (the paper gives no step
   size):  g = grad L^CSI(0),  t* = (||g||^2/2) / (||A_d g||^2/S_d + ||A_s g||^2/S_s),
   alpha_0 = -t* g, where A_d = G_S F_T^* and A_s = [R_0 G_D - beta(I - R_0)] F_T^*.
4. The full CSI start the paper sets aside for its cost: L^CSI is quadratic in
   alpha for fixed R_0, so it is minimised by conjugate gradients (Fletcher-
   Reeves directions, the exact step along each); one CG step is step 3.
"""
from __future__ import annotations

import numpy as np

from . import fourier, operators as ops
from .loss import Problem


def bp_currents(prob: Problem):
    """Back-propagation currents J_p = gamma_p G_S^H e_p, [F, Ni, M, M]."""
    M, F, Ni = prob.M, prob.F, prob.Ni
    Jbp = []
    for f in range(F):
        e = prob.esca[f]                                   # [Ni, Ns]
        u = e @ np.conj(prob.gs[f])                        # u_p = G_S^H e_p  [Ni, N]
        v = u @ prob.gs[f].T                               # v_p = G_S u_p    [Ni, Ns]
        gamma = np.sum(np.conj(v) * e, axis=1) / np.sum(np.abs(v) ** 2, axis=1)
        Jbp.append((gamma[:, None] * u).reshape(Ni, M, M))
    return np.array(Jbp)


def ls_contrast(prob: Problem, J):
    """Contrast of currents J [F, Ni, M, M]: the fields E_p = E_inc_p + G_D J_p of the state
    equation (Eq. 3), the per-pixel least-squares contrast of J_p = chi E_p over all incidences
    (frequencies weighted by 1 / ||E_inc,f||^2), chi_0 = sum J conj(E) / sum |E|^2, and
    R_0 = beta chi_0 / (beta chi_0 + 1) (Eq. 7)."""
    M, F, Ni = prob.M, prob.F, prob.Ni
    beta = prob.params.beta
    w = 1.0 / prob.S_s
    num = np.zeros((M, M), np.complex128)
    den = np.zeros((M, M))
    for f in range(F):
        E = prob.einc[f].reshape(Ni, M, M) + ops.gd_apply(J[f], prob.ghat[f])
        num += w[f] * np.sum(J[f] * np.conj(E), axis=0)
        den += w[f] * np.sum(np.abs(E) ** 2, axis=0)
    chi0 = num / den
    R0 = beta * chi0 / (beta * chi0 + 1.0)
    return chi0, R0


def bp_contrast(prob: Problem):
    """chi_0, R_0 and the currents of the back-propagation start."""
    Jbp = bp_currents(prob)
    chi0, R0 = ls_contrast(prob, Jbp)
    return chi0, R0, Jbp


def csi_gradient_at_zero(prob: Problem, R0):
    """grad L^CSI at alpha = 0 with R fixed at R0, [F, Ni, K, K]."""
    M, F, Ni, K = prob.M, prob.F, prob.Ni, prob.K
    beta = prob.params.beta
    g = []
    for f in range(F):
        Einc = prob.einc[f].reshape(Ni, M, M)
        g_s = 2.0 * (R0[None] * Einc) / prob.S_s[f]          # s = R0 E_inc at J = 0
        g_E = np.conj(R0)[None] * g_s
        d = -prob.esca[f]                                   # G_S J - e at J = 0
        hS = (d @ np.conj(prob.gs[f])).reshape(Ni, M, M)    # G_S^H d
        g_J = -beta * g_s + beta * g_E + ops.gd_adjoint_apply(g_E, prob.ghat[f]) \
            + 2.0 * hS / prob.S_d[f]
        g.append(fourier.synth_adjoint(g_J, K))
    return np.array(g)


def csi_curvature(prob: Problem, R0, g):
    """||A_d g||^2 / S_d + ||A_s g||^2 / S_s summed over frequencies."""
    M, F, Ni = prob.M, prob.F, prob.Ni
    beta = prob.params.beta
    q = 0.0
    for f in range(F):
        Jg = fourier.synthesize(g[f], M)
        Ad = Jg.reshape(Ni, M * M) @ prob.gs[f].T
        As = R0[None] * (ops.gd_apply(Jg, prob.ghat[f]) + beta * Jg) - beta * Jg
        q += np.sum(np.abs(Ad) ** 2) / prob.S_d[f] + np.sum(np.abs(As) ** 2) / prob.S_s[f]
    return float(q)


def csi_loss(prob: Problem, R0, alpha):
    """L^CSI (Eq. 12) at alpha with R fixed at R0."""
    M, F, Ni = prob.M, prob.F, prob.Ni
    beta = prob.params.beta
    tot = 0.0
    for f in range(F):
        J = fourier.synthesize(alpha[f], M)
        D = J.reshape(Ni, M * M) @ prob.gs[f].T
        s = R0[None] * (prob.einc[f].reshape(Ni, M, M) + ops.gd_apply(J, prob.ghat[f]) + beta * J) \
            - beta * J
        tot += np.sum(np.abs(D - prob.esca[f]) ** 2) / prob.S_d[f] \
            + np.sum(np.abs(s) ** 2) / prob.S_s[f]
    return float(tot)


def alpha0(prob: Problem):
    """alpha_0 [F, Ni, K, K] and the diagnostics (chi0, R0, g, t*)."""
    chi0, R0, _ = bp_contrast(prob)
    g = csi_gradient_at_zero(prob, R0)
    t = 0.5 * float(np.sum(np.abs(g) ** 2)) / csi_curvature(prob, R0, g)
    return -t * g, dict(chi0=chi0, R0=R0, g=g, t=t)


def csi_gradient(prob: Problem, R0, alpha):
    """grad L^CSI (dL/dRe + i dL/dIm) at alpha [F, Ni, K, K] with R fixed at R0: 2 A^H (A alpha - b)
    written out through the adjoints of G_S, G_D and the synthesis."""
    M, F, Ni, K = prob.M, prob.F, prob.Ni, prob.K
    beta = prob.params.beta
    g = []
    for f in range(F):
        J = fourier.synthesize(alpha[f], M)
        E = prob.einc[f].reshape(Ni, M, M) + ops.gd_apply(J, prob.ghat[f]) + beta * J
        g_s = 2.0 * (R0[None] * E - beta * J) / prob.S_s[f]
        g_E = np.conj(R0)[None] * g_s
        d = J.reshape(Ni, M * M) @ prob.gs[f].T - prob.esca[f]
        hS = (d @ np.conj(prob.gs[f])).reshape(Ni, M, M)
        g_J = -beta * g_s + beta * g_E + ops.gd_adjoint_apply(g_E, prob.ghat[f]) + 2.0 * hS / prob.S_d[f]
        g.append(fourier.synth_adjoint(g_J, K))
    return np.array(g)


def csi_cg(prob: Problem, n_iter: int):
    """alpha after n_iter conjugate-gradient steps on L^CSI from zero (R fixed at the
    back-propagation R_0): direction p_1 = -g_1, p_k = -g_k + (||g_k||^2 / ||g_{k-1}||^2) p_{k-1},
    step t_k = -Re<g_k, p_k> / (2 (||A_d p_k||^2 / S_d + ||A_s p_k||^2 / S_s)).  n_iter = 1 is
    alpha0().  Returns alpha and the loss after every step."""
    _, R0, _ = bp_contrast(prob)
    alpha = np.zeros((prob.F, prob.Ni, prob.K, prob.K), np.complex128)
    p, gn_old, losses = None, None, []
    for k in range(n_iter):
        g = csi_gradient(prob, R0, alpha)
        gn = float(np.sum(np.abs(g) ** 2))
        p = -g if k == 0 else -g + (gn / gn_old) * p
        gn_old = gn
        q = csi_curvature(prob, R0, p)
        t = -float(np.sum(np.real(np.conj(g) * p))) / (2.0 * q) if q > 0 else 0.0
        alpha = alpha + t * p
        losses.append(csi_loss(prob, R0, alpha))
    return alpha, dict(R0=R0, losses=losses)
