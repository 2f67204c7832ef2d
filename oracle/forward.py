"""Forward scattering: method-of-moments synthesis of measured fields.

Solves the Lippmann-Schwinger state equation (Eq. 3) for every incidence,
    (I - G_D X) E_tot = E_inc,      X = diag(chi),  chi = eps_r - 1,
then the data equation (Eq. 4), E_sca = G_S X E_tot.  Only pixels with
chi != 0 couple, so the exact support-restricted system
    (I - G_D[S, S] X_S) E_S = E_inc[S],  E_sca = G_S[:, S] X_S E_S
is what the default path solves (dense LU).  A full-grid dense LU and a
GMRES solve with FFT matvecs are kept for cross-checks.

Also here: the Mie (Bessel-series) field of a homogeneous circular cylinder
under the same line source.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla
from scipy import special

import seeded_inputs as si

from . import operators as ops


def _tables(eps: np.ndarray, side: float, k0: float, tx_xy, rx_xy, cx=0.0, cy=0.0):
    M = eps.shape[0]
    chi = (eps - 1.0).reshape(-1)
    einc = ops.einc_matrix(tx_xy, M, side, k0, cx, cy)
    gs = ops.gs_matrix(rx_xy, M, side, k0, cx, cy)
    return M, chi, einc, gs


def mom_solve(eps: np.ndarray, side: float, k0: float, tx_xy: np.ndarray,
              rx_xy: np.ndarray, method: str = "support", cx: float = 0.0,
              cy: float = 0.0, tol: float = 1e-12):
    """Scattered field [N_i, N_s] and total field [N_i, N] for eps[M, M].

    method: "support" (LU on the chi != 0 pixels), "dense" (LU on the full
    grid) or "gmres" (FFT matvecs, relative residual tol).
    """
    M, chi, einc, gs = _tables(eps, side, k0, tx_xy, rx_xy, cx, cy)
    h = side / M
    N = M * M
    etot = einc.copy()
    if method == "support":
        S = np.nonzero(chi != 0)[0]
        if S.size:
            ker = ops.gd_offset_kernel(M, h, k0)
            ii, jj = S // M, S % M
            gss = ker[ii[:, None] - ii[None, :] + M - 1, jj[:, None] - jj[None, :] + M - 1]
            A = np.eye(S.size) - gss * chi[S][None, :]
            lu = sla.lu_factor(A)
            etot[:, S] = sla.lu_solve(lu, einc[:, S].T).T
    elif method == "dense":
        A = np.eye(N) - ops.gd_dense(M, h, k0) * chi[None, :]
        etot = np.linalg.solve(A, einc.T).T
    elif method == "gmres":
        ghat = ops.gd_spectrum(M, h, k0)

        def mv(v):
            return v - ops.gd_apply((chi * v).reshape(M, M), ghat).reshape(-1)

        A = spla.LinearOperator((N, N), matvec=mv, dtype=np.complex128)
        for p in range(einc.shape[0]):
            x, info = spla.gmres(A, einc[p], rtol=tol, atol=0.0, restart=200, maxiter=50)
            if info != 0:
                raise RuntimeError(f"gmres did not converge (info={info})")
            etot[p] = x
    else:
        raise ValueError(method)
    esca = (gs @ (chi[None, :] * etot).T).T
    return esca, etot


def mie_scattered(eps_r: complex, rho_c: float, centre, tx_xy: np.ndarray,
                  rx_xy: np.ndarray, k0: float, field_centre=(0.0, 0.0),
                  n_extra: int = 20) -> np.ndarray:
    """Exact scattered field [N_i, N_s] of a homogeneous cylinder (radius rho_c).

    Incident field c_p H0(k0 |r - r_p|) expanded by Graf's addition theorem;
    continuity of E_z and dE_z/drho at rho_c gives the coefficients
      a_n = [k1 J_n'(k1 rc) J_n(k0 rc) - k0 J_n(k1 rc) J_n'(k0 rc)]
            / [k0 J_n(k1 rc) H_n'(k0 rc) - k1 J_n'(k1 rc) H_n(k0 rc)],
    E_sca(rho, phi) = c_p sum_n a_n H_n(k0 rho_p) H_n(k0 rho) exp(i n (phi - phi_p)).
    c_p = 1/|H0(k0 |r_p - field_centre|)| matches the MoM incident field.
    """
    k1 = k0 * np.sqrt(complex(eps_r))
    nmax = int(np.ceil(abs(k1) * rho_c + abs(k0) * rho_c)) + n_extra
    n = np.arange(-nmax, nmax + 1)
    x0, x1 = k0 * rho_c, k1 * rho_c
    num = k1 * special.jvp(n, x1) * special.jv(n, x0) - k0 * special.jv(n, x1) * special.jvp(n, x0)
    den = k0 * special.jv(n, x1) * special.h1vp(n, x0) - k1 * special.jvp(n, x1) * special.hankel1(n, x0)
    a = num / den
    tx = tx_xy - np.asarray(centre)[None, :]
    rx = rx_xy - np.asarray(centre)[None, :]
    rt, pt = np.hypot(tx[:, 0], tx[:, 1]), np.arctan2(tx[:, 1], tx[:, 0])
    rr, pr = np.hypot(rx[:, 0], rx[:, 1]), np.arctan2(rx[:, 1], rx[:, 0])
    ct = 1.0 / np.abs(special.hankel1(0, k0 * np.hypot(tx_xy[:, 0] - field_centre[0],
                                                       tx_xy[:, 1] - field_centre[1])))
    Ht = special.hankel1(n[None, :], k0 * rt[:, None])          # [Ni, n]
    Hr = special.hankel1(n[None, :], k0 * rr[:, None])          # [Ns, n]
    phase = np.exp(1j * n[None, None, :] * (pr[None, :, None] - pt[:, None, None]))
    return ct[:, None] * np.sum(a[None, None, :] * Ht[:, None, :] * Hr[None, :, :] * phase, axis=-1)


# Noise is part of the synthetic-data recipe, shared with the GPU side.
add_noise = si.add_noise
