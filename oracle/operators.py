"""Green's operators of the 2-D TM problem (Sec. 2.1, Eqs. 1-4).

Time dependence exp(-i w t): the 2-D scalar Green's function is
g(r, r') = (i/4) H0^(1)(k0 |r - r'|), so a passive medium has Im(chi) >= 0.

The paper names the discretisation only as "the method of moments"; this
oracle uses circular pulse cells of equal area (radius a = h / sqrt(pi)),
for which the cell integrals of k0^2 g have closed forms:
  off-diagonal  (i pi k0 a / 2) J1(k0 a) H0(k0 rho)
  self term     (i pi k0 a / 2) H1(k0 a) - 1
  receiver      (i pi k0 a / 2) J1(k0 a) H0(k0 |r_q - r_n|)
The line-source incident field is c_p H0(k0 |r - r_p|) with
c_p = 1 / |H0(k0 |r_p - centre|)|, unit magnitude at the domain centre.

Grid: row i runs along y, column j along x, pixel n = i * M + j, centres at
centre - side/2 + (index + 1/2) h.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
from scipy import special


def pixel_coords(M: int, side: float, cx: float = 0.0, cy: float = 0.0):
    """Returns (x[j], y[i], h)."""
    h = side / M
    c = -side / 2.0 + (np.arange(M) + 0.5) * h
    return cx + c, cy + c, h


def pixel_positions(M: int, side: float, cx: float = 0.0, cy: float = 0.0) -> np.ndarray:
    """[N, 2] (x, y) of pixel n = i * M + j."""
    x, y, _ = pixel_coords(M, side, cx, cy)
    X, Y = np.meshgrid(x, y)
    return np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)


def cell_factor(k0: float, h: float) -> complex:
    """(i pi k0 a / 2) J1(k0 a): k0^2 times the cell integral of g outside the cell."""
    a = h / np.sqrt(np.pi)
    return 1j * np.pi * k0 * a / 2.0 * special.jv(1, k0 * a)


def self_term(k0: float, h: float) -> complex:
    """k0^2 times the integral of g over its own cell: (i pi k0 a / 2) H1(k0 a) - 1."""
    a = h / np.sqrt(np.pi)
    return 1j * np.pi * k0 * a / 2.0 * special.hankel1(1, k0 * a) - 1.0


def gd_offset_kernel(M: int, h: float, k0: float) -> np.ndarray:
    """G_D as a function of the pixel offset: [2M-1, 2M-1], index (di+M-1, dj+M-1)."""
    d = np.arange(-(M - 1), M)
    DI, DJ = np.meshgrid(d, d, indexing="ij")
    rho = h * np.sqrt(DI.astype(float) ** 2 + DJ.astype(float) ** 2)
    ker = np.empty(rho.shape, dtype=np.complex128)
    nz = rho > 0
    ker[nz] = cell_factor(k0, h) * special.hankel1(0, k0 * rho[nz])
    ker[~nz] = self_term(k0, h)
    return ker


def gd_dense(M: int, h: float, k0: float) -> np.ndarray:
    """Dense N x N domain operator (direct definition; small grids only)."""
    ker = gd_offset_kernel(M, h, k0)
    ii, jj = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    ii = ii.reshape(-1)
    jj = jj.reshape(-1)
    di = ii[:, None] - ii[None, :] + (M - 1)
    dj = jj[:, None] - jj[None, :] + (M - 1)
    return ker[di, dj]


def gd_spectrum(M: int, h: float, k0: float) -> np.ndarray:
    """FFT of the offset kernel embedded in a 2M x 2M circulant.

    Offset (di, dj) goes to index (di mod 2M, dj mod 2M); index M (offset +-M,
    never reached by a linear convolution of support M) is zero.
    """
    P = 2 * M
    ker = gd_offset_kernel(M, h, k0)
    emb = np.zeros((P, P), dtype=np.complex128)
    d = np.arange(-(M - 1), M) % P
    emb[np.ix_(d, d)] = ker
    return sfft.fft2(emb)


def gd_apply(x: np.ndarray, ghat: np.ndarray) -> np.ndarray:
    """G_D x for x[..., M, M]: zero-pad to 2M, multiply spectra, crop."""
    M = x.shape[-1]
    P = ghat.shape[-1]
    pad = np.zeros(x.shape[:-2] + (P, P), dtype=np.complex128)
    pad[..., :M, :M] = x
    y = sfft.ifft2(sfft.fft2(pad) * ghat)
    return y[..., :M, :M]


def gd_adjoint_apply(y: np.ndarray, ghat: np.ndarray) -> np.ndarray:
    """G_D^H y.  The kernel is symmetric in the offset, so the adjoint's
    spectrum is conj(ghat)."""
    return gd_apply(y, np.conj(ghat))


def gs_matrix(rx_xy: np.ndarray, M: int, side: float, k0: float,
              cx: float = 0.0, cy: float = 0.0) -> np.ndarray:
    """Receiver operator G_S [N_s, N] (Eq. 4)."""
    pix = pixel_positions(M, side, cx, cy)
    h = side / M
    dist = np.hypot(rx_xy[:, None, 0] - pix[None, :, 0], rx_xy[:, None, 1] - pix[None, :, 1])
    return cell_factor(k0, h) * special.hankel1(0, k0 * dist)


def einc_matrix(tx_xy: np.ndarray, M: int, side: float, k0: float,
                cx: float = 0.0, cy: float = 0.0) -> np.ndarray:
    """Incident fields [N_i, N] of unit-amplitude-at-centre line sources."""
    pix = pixel_positions(M, side, cx, cy)
    dist = np.hypot(tx_xy[:, None, 0] - pix[None, :, 0], tx_xy[:, None, 1] - pix[None, :, 1])
    rc = np.hypot(tx_xy[:, 0] - cx, tx_xy[:, 1] - cy)
    c = 1.0 / np.abs(special.hankel1(0, k0 * rc))
    return c[:, None] * special.hankel1(0, k0 * dist)


def wavenumber(freq_hz: float) -> float:
    return 2.0 * np.pi * freq_hz / 299_792_458.0
