"""Composite PDF loss and its gradient (Sec. 3.2, Eqs. 13-19; Sec. 2.2, Eqs. 6-7).

Given Fourier coefficients alpha[F, N_i, K, K] (F frequencies, N_i incidences):
  J    = F_T^*(alpha)                          induced currents (Eq. 9)
  E    = E_inc + G_D J + beta J                the bracket of the CIE state Eq. 6
  R    = per-pixel least-squares solution of beta J = R E over all incidences
         (and frequencies), R_n = beta sum w J conj(E) / sum w |E|^2, with
         weight w = 1/||E_inc||^2 of the frequency (a reading: the paper only
         says R and chi are "the solutions from CIE"; for one frequency the
         weight cancels)
  chi  = R / (beta (1 - R))                    inverse of Eq. 7
  s    = R E - beta J  = R E_inc + [R G_D - beta (I - R)] J      (Eq. 15)
  L_State  = sum ||s||^2 / ||E_inc||^2         (Eq. 15, summed over frequencies)
  L_Data   = sum ||G_S J - E_sca||^2 / ||E_sca||^2               (Eq. 16)
  L_Bound  = ||ReLU(-Re chi)||^2                                 (Eq. 17)
  L_TV     = sum sqrt(|D_x chi|^2 + |D_y chi|^2 + eps_tv)        (Eq. 18)
  L_Bridge = sum sigma((|chi| - tau_B)/tau_B) exp(-(D_x a)^2 - (D_y a)^2),
             a = sqrt(|chi|^2 + eps_abs)                          (Eq. 19)
  L = L_State + L_Data + lam1 L_Bound + lam2 L_TV + lam3 L_Bridge (Eqs. 13-14)
With cco_in_loss (an option; the paper applies the CCO of Sec. 2.4 to the
final image only) every chi-dependent term sees chi_c = CCO(chi) instead:
the regularisers are evaluated on chi_c and the state residual takes
R_c = beta chi_c / (1 + beta chi_c) (Eq. 7) in place of R, s = R_c E - beta J;
the gradient runs through the CCO as well.
D_x, D_y are forward differences with a zero difference on the last column /
row.  Defaults: beta = 6 (Sec. 4.1), lam = 1e-3, 1e-5, 1e-5 (Sec. 3.2),
tau_B = 0.5 (Sec. 3.2).

Gradient convention (that of PyTorch for a real loss of a complex variable):
g_z = dL/dRe(z) + i dL/dIm(z), so dL = Re(conj(g_z) dz).  The adjoint below is
the chain rule through every step above, including the dependence of R on
(J, E); it is checked by finite differences and by torch autograd.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import cco as occo, fourier, operators as ops


@dataclasses.dataclass
class Params:
    beta: float = 6.0
    lam_bound: float = 1e-3
    lam_tv: float = 1e-5
    lam_bridge: float = 1e-5
    tau_b: float = 0.5
    eps_tv: float = 1e-12
    eps_abs: float = 1e-12
    cco_in_loss: bool = False
    cco_tau: float = 3.0
    cco_eta_max: float = 0.1
    cco_delta: float = 0.5
    gf_radius: int = 1
    gf_eps: float = 1e-2


@dataclasses.dataclass
class Problem:
    """Operator tables of one geometry plus one measured data set.

    ghat [F, 2M, 2M], gs [F, N_s, N], einc [F, N_i, N], esca [F, N_i, N_s].
    """
    M: int
    K: int
    ghat: np.ndarray
    gs: np.ndarray
    einc: np.ndarray
    esca: np.ndarray
    params: Params = dataclasses.field(default_factory=Params)

    @property
    def F(self):
        return self.gs.shape[0]

    @property
    def Ni(self):
        return self.einc.shape[1]

    @property
    def S_s(self):
        return np.sum(np.abs(self.einc) ** 2, axis=(1, 2))

    @property
    def S_d(self):
        return np.sum(np.abs(self.esca) ** 2, axis=(1, 2))


def build_problem(M: int, K: int, side: float, freqs, tx_xy, rx_xy, esca,
                  params: Optional[Params] = None, cx: float = 0.0, cy: float = 0.0) -> Problem:
    h = side / M
    ghat, gs, einc = [], [], []
    for f in np.atleast_1d(freqs):
        k0 = ops.wavenumber(float(f))
        ghat.append(ops.gd_spectrum(M, h, k0))
        gs.append(ops.gs_matrix(rx_xy, M, side, k0, cx, cy))
        einc.append(ops.einc_matrix(tx_xy, M, side, k0, cx, cy))
    esca = np.asarray(esca, dtype=np.complex128)
    if esca.ndim == 2:
        esca = esca[None]
    return Problem(M, K, np.array(ghat), np.array(gs), np.array(einc), esca,
                   params or Params())


# ---------------------------------------------------------------- regularisers

def _dx(z):
    d = np.zeros_like(z)
    d[..., :, :-1] = z[..., :, 1:] - z[..., :, :-1]
    return d


def _dy(z):
    d = np.zeros_like(z)
    d[..., :-1, :] = z[..., 1:, :] - z[..., :-1, :]
    return d


def _dx_adj(g):
    """Adjoint of _dx: out = D_x^T g."""
    out = np.zeros_like(g)
    out[..., :, 1:] += g[..., :, :-1]
    out[..., :, :-1] -= g[..., :, :-1]
    return out


def _dy_adj(g):
    out = np.zeros_like(g)
    out[..., 1:, :] += g[..., :-1, :]
    out[..., :-1, :] -= g[..., :-1, :]
    return out


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def reg_bound(chi):
    """Eq. 17: value and gradient w.r.t. chi."""
    r = np.maximum(-chi.real, 0.0)
    return float(np.sum(r * r)), (-2.0 * r).astype(np.complex128)


def reg_tv(chi, eps_tv):
    """Eq. 18 on a complex image (|.|^2 of complex differences)."""
    dx, dy = _dx(chi), _dy(chi)
    t = np.sqrt(np.abs(dx) ** 2 + np.abs(dy) ** 2 + eps_tv)
    g = _dx_adj(dx / t) + _dy_adj(dy / t)
    return float(np.sum(t)), g


def reg_bridge(chi, tau_b, eps_abs):
    """Eq. 19 with |chi| smoothed to sqrt(|chi|^2 + eps_abs)."""
    a = np.sqrt(np.abs(chi) ** 2 + eps_abs)
    ax, ay = _dx(a), _dy(a)
    sig = _sigmoid((a - tau_b) / tau_b)
    ex = np.exp(-ax * ax - ay * ay)
    val = float(np.sum(sig * ex))
    # dL/da: through the gate sig(a) and through the two differences.
    dsig = sig * (1.0 - sig) / tau_b
    g_a = dsig * ex
    g_ax = -2.0 * ax * sig * ex
    g_ay = -2.0 * ay * sig * ex
    g_a = g_a + _dx_adj(g_ax) + _dy_adj(g_ay)
    return val, g_a * chi / a


# ------------------------------------------------------------------- the loss

def evaluate(alpha: np.ndarray, prob: Problem, grad: bool = True,
             r_stopgrad: bool = False) -> dict:
    """Loss terms (and g_alpha) at alpha[F, N_i, K, K] (a 3-D alpha means F = 1)."""
    p = prob.params
    beta = p.beta
    alpha = np.asarray(alpha, dtype=np.complex128)
    squeeze = alpha.ndim == 3
    if squeeze:
        alpha = alpha[None]
    M = prob.M
    F = prob.F
    w = 1.0 / prob.S_s                                    # [F]
    J = fourier.synthesize(alpha, M)                      # [F, Ni, M, M]
    GJ = np.stack([ops.gd_apply(J[f], prob.ghat[f]) for f in range(F)])
    Einc = prob.einc.reshape(F, prob.Ni, M, M)
    E = Einc + GJ + beta * J
    num = np.einsum("f,fpij->ij", w, J * np.conj(E))
    den = np.einsum("f,fpij->ij", w, np.abs(E) ** 2)
    R = beta * num / den
    chi = R / (beta * (1.0 - R))
    ckw = dict(tau=p.cco_tau, eta_max=p.cco_eta_max, delta=p.cco_delta, r=p.gf_radius, eps_gf=p.gf_eps)
    if p.cco_in_loss:
        chi_c = occo.cco(chi, **ckw)
        R_c = beta * chi_c / (1.0 + beta * chi_c)
    else:
        chi_c, R_c = chi, R
    s = R_c[None, None] * E - beta * J
    L_state = float(np.sum(w * np.sum(np.abs(s) ** 2, axis=(1, 2, 3))))
    Jflat = J.reshape(F, prob.Ni, M * M)
    D = np.einsum("fqn,fpn->fpq", prob.gs, Jflat)          # [F, Ni, Ns]
    d = D - prob.esca
    L_data = float(np.sum(np.sum(np.abs(d) ** 2, axis=(1, 2)) / prob.S_d))
    Lb, gb = reg_bound(chi_c)
    Lt, gt = reg_tv(chi_c, p.eps_tv)
    Lr, gr = reg_bridge(chi_c, p.tau_b, p.eps_abs)
    L = L_state + L_data + p.lam_bound * Lb + p.lam_tv * Lt + p.lam_bridge * Lr
    out = dict(J=J, E=E, num=num, den=den, R=R, chi=chi, chi_c=chi_c, R_c=R_c, s=s, D=D, d=d,
               L_state=L_state, L_data=L_data, L_bound=Lb, L_tv=Lt, L_bridge=Lr, L=L)
    if not grad:
        return out

    # ---- adjoint
    g_chi = p.lam_bound * gb + p.lam_tv * gt + p.lam_bridge * gr
    if r_stopgrad:
        g_R = np.zeros_like(R)
    elif p.cco_in_loss:
        # the state term through its contrast R_c = beta chi_c / (1 + beta chi_c), then back
        # through the CCO to chi and R
        g_chi = g_chi + np.conj(beta / (1.0 + beta * chi_c) ** 2) * 2.0 * (R_c * den - beta * num)
        g_chi = occo.cco_vjp(chi, g_chi, **ckw)
        g_R = np.conj(1.0 / (beta * (1.0 - R) ** 2)) * g_chi
    else:
        g_R = np.conj(1.0 / (beta * (1.0 - R) ** 2)) * g_chi
        # state term through R; zero when R is the exact least-squares optimum
        g_R = g_R + 2.0 * (R * den - beta * num)
    g_s = 2.0 * w[:, None, None, None] * s
    wf = w[:, None, None, None]
    g_E = np.conj(R_c)[None, None] * g_s \
        + wf * (beta * np.conj(g_R)[None, None] * J
                - 2.0 * np.real(np.conj(g_R) * R)[None, None] * E) / den[None, None]
    g_J = -beta * g_s + wf * beta * g_R[None, None] * E / den[None, None]
    g_J = g_J + beta * g_E
    g_J = g_J + np.stack([ops.gd_adjoint_apply(g_E[f], prob.ghat[f]) for f in range(F)])
    hS = np.einsum("fqn,fpq->fpn", np.conj(prob.gs), d)     # G_S^H d
    g_J = g_J + (2.0 / prob.S_d)[:, None, None, None] * hS.reshape(F, prob.Ni, M, M)
    g_alpha = fourier.synth_adjoint(g_J, alpha.shape[-1])
    out.update(g_chi=g_chi, g_R=g_R, g_E=g_E, g_J=g_J,
               g_alpha=g_alpha[0] if squeeze else g_alpha)
    return out


def loss_total(alpha, prob: Problem) -> float:
    return evaluate(alpha, prob, grad=False)["L"]
