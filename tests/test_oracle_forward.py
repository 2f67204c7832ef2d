"""Pins of the MoM forward solver (Eqs. 3-5, 8): Mie series, solver
agreement, reciprocity, Born limit, the CIE data equation, noise level."""
import numpy as np
import pytest
from scipy import special

import seeded_inputs as si
from oracle import forward, operators as ops

WL = si.WORKLOADS["cfg1"]
LAM = WL.wavelength
K0 = ops.wavenumber(WL.freq_hz)


def disc(eps, r=0.35, c=(0.1, -0.05)):
    return si.Shape("ellipse", c[0] * LAM, c[1] * LAM, r * LAM, r * LAM, 0.0, complex(eps))


def test_mie_series_converged_and_trivial():
    tx = si.antenna_positions(8, WL.radius)
    rx = si.antenna_positions(12, WL.radius)
    a = forward.mie_scattered(3.0, 0.35 * LAM, (0.0, 0.0), tx, rx, K0)
    b = forward.mie_scattered(3.0, 0.35 * LAM, (0.0, 0.0), tx, rx, K0, n_extra=40)
    assert np.max(np.abs(a - b)) < 1e-14 * np.max(np.abs(a))
    z = forward.mie_scattered(1.0, 0.35 * LAM, (0.0, 0.0), tx, rx, K0)
    assert np.max(np.abs(z)) < 1e-14 * np.max(np.abs(a))


@pytest.mark.slow
def test_mom_converges_to_mie():
    tx = si.antenna_positions(WL.n_tx, WL.radius)
    rx = si.antenna_positions(WL.n_rx, WL.radius)
    for eps_r in (3.0, 2.0 + 0.5j):
        mie = forward.mie_scattered(eps_r, 0.35 * LAM, (0.1 * LAM, -0.05 * LAM), tx, rx, K0)
        errs = []
        for Mf in (32, 64, 128):
            e, _ = forward.mom_solve(si.rasterize([disc(eps_r)], Mf, WL.side), WL.side, K0, tx, rx)
            errs.append(np.linalg.norm(e - mie) / np.linalg.norm(mie))
        # at least first-order convergence under refinement, and a bound at the finest grid
        assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1], errs
        assert errs[2] < 5e-3, errs


def test_solvers_agree():
    tx = si.antenna_positions(4, WL.radius)
    rx = si.antenna_positions(6, WL.radius)
    eps = si.rasterize([disc(2.5, 0.3)], 24, WL.side)
    a, _ = forward.mom_solve(eps, WL.side, K0, tx, rx, "support")
    b, _ = forward.mom_solve(eps, WL.side, K0, tx, rx, "dense")
    c, _ = forward.mom_solve(eps, WL.side, K0, tx, rx, "gmres")
    n = np.linalg.norm(a)
    assert np.linalg.norm(a - b) < 1e-10 * n
    assert np.linalg.norm(a - c) < 1e-10 * n


def test_reciprocity():
    # Tx positions = Rx positions: the scattered-field matrix is symmetric.
    ant = si.antenna_positions(10, WL.radius)
    shapes = si.draw_profile(WL, 3)
    eps = si.rasterize(shapes, 32, WL.side)
    S, _ = forward.mom_solve(eps, WL.side, K0, ant, ant)
    assert np.max(np.abs(S - S.T)) < 1e-12 * np.max(np.abs(S))


def test_born_limit():
    tx = si.antenna_positions(4, WL.radius)
    rx = si.antenna_positions(5, WL.radius)
    M = 16
    base = si.rasterize([disc(2.0, 0.3)], M, WL.side) - 1.0
    gs = ops.gs_matrix(rx, M, WL.side, K0)
    einc = ops.einc_matrix(tx, M, WL.side, K0)
    ratios = []
    for t in (1e-2, 5e-3, 2.5e-3):
        chi = t * base
        e, _ = forward.mom_solve(1.0 + chi, WL.side, K0, tx, rx)
        born = (gs @ (chi.reshape(-1)[None, :] * einc).T).T
        ratios.append(np.linalg.norm(e - born) / t ** 2)
    # the remainder is O(chi^2): its ratio to t^2 is constant as t -> 0
    assert abs(ratios[1] / ratios[0] - 1) < 0.02 and abs(ratios[2] / ratios[1] - 1) < 0.01


@pytest.mark.parametrize("beta", [1.0, 6.0, 2.0 + 1.0j])
def test_cie_data_equation(beta):
    # Eq. 8: E_sca = (1/beta) G_S [I - R (I + G_D/beta)]^-1 R E_inc, R = beta chi/(beta chi + 1)
    M = 12
    tx = si.antenna_positions(3, WL.radius)
    rx = si.antenna_positions(4, WL.radius)
    eps = si.rasterize([disc(3.0, 0.3)], M, WL.side)
    e, _ = forward.mom_solve(eps, WL.side, K0, tx, rx, "dense")
    chi = (eps - 1).reshape(-1)
    R = beta * chi / (beta * chi + 1)
    G = ops.gd_dense(M, WL.side / M, K0)
    gs = ops.gs_matrix(rx, M, WL.side, K0)
    einc = ops.einc_matrix(tx, M, WL.side, K0)
    A = np.eye(M * M) - R[:, None] * (np.eye(M * M) + G / beta)
    cie = (gs @ np.linalg.solve(A, R[:, None] * einc.T) / beta).T
    assert np.linalg.norm(cie - e) < 1e-10 * np.linalg.norm(e)


def test_noise_level_and_reproducibility():
    rng = np.random.default_rng(0)
    e = rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64))
    n1, n2 = si.draw_noise(7, e.shape)
    m1, m2 = si.draw_noise(7, e.shape)
    assert np.array_equal(n1, m1) and np.array_equal(n2, m2)
    for nu in (0.05, 0.1, 10 ** (-10 / 20)):
        noisy = forward.add_noise(e, nu, n1, n2)
        ratio = np.linalg.norm(noisy - e) / np.linalg.norm(e)
        assert abs(ratio / nu - 1) < 0.03


def test_position_errors_change_the_data_linearly_in_sigma():
    """The antenna-position study's premise: displacing every antenna by sigma times a fixed random
    direction changes the scattered field by an amount proportional to sigma (first order), so the
    relative data change at 2 sigma is twice that at sigma."""
    wl = si.WORKLOADS["cfg1"]
    k0 = ops.wavenumber(wl.freq_hz)
    tx = si.antenna_positions(6, wl.radius)
    rx = si.antenna_positions(8, wl.radius)
    eps = si.rasterize(si.draw_profile(wl, 0), 16, wl.side)
    e0, _ = forward.mom_solve(eps, wl.side, k0, tx, rx)
    dt, dr = si.draw_position_errors(3, 6, 8, 1.0)
    ch = []
    for sg in (1e-4, 2e-4):
        e, _ = forward.mom_solve(eps, wl.side, k0, tx + sg * dt, rx + sg * dr)
        ch.append(np.linalg.norm(e - e0) / np.linalg.norm(e0))
    assert abs(ch[1] / ch[0] - 2.0) < 0.01


def _shift_case(M=16):
    """A disc well inside a 16 x 16 grid (the border rows and columns stay background)."""
    eps = si.rasterize([disc(2.5, r=0.3, c=(0.05, -0.1))], M, WL.side)
    assert np.all(eps[0] == 1) and np.all(eps[-1] == 1) and np.all(eps[:, 0] == 1) and np.all(eps[:, -1] == 1)
    return eps, WL.side / M


@pytest.mark.parametrize("axis", [0, 1])
def test_antenna_displacement_equals_object_shift(axis):
    """What the antenna-position study rests on (Sec. 4): the scattered field depends only on where
    the antennas are relative to the object.  Every Tx and Rx moved by one pixel width h along x
    (axis 1: column index) or y (axis 0: row index) sees the same field as the fixed antennas with
    the object moved by -h, which on the pixel grid is the raster shifted by one index.  The MoM
    matrix depends only on pixel offsets, so the two solves agree to rounding once each source's
    amplitude is divided out (a source is normalised to unit field magnitude at the grid centre,
    so moving it changes its amplitude by |H_0(k0 r_c)| / |H_0(k0 r_c')|); swapping x and y in the
    pixel centres, or the sign of a displacement, breaks it."""
    eps, h = _shift_case()
    tx = si.antenna_positions(8, WL.radius)
    rx = si.antenna_positions(12, WL.radius)
    d = np.zeros(2)
    d[1 - axis] = h                     # (x, y) displacement: axis 1 -> x, axis 0 -> y
    amp = lambda t: 1.0 / np.abs(special.hankel1(0, K0 * np.hypot(t[:, 0], t[:, 1])))[:, None]
    moved, _ = forward.mom_solve(eps, WL.side, K0, tx + d, rx + d)
    moved = moved / amp(tx + d)
    shifted = np.roll(eps, -1, axis=axis)   # eps'(r) = eps(r + d)
    fixed, _ = forward.mom_solve(shifted, WL.side, K0, tx, rx)
    fixed = fixed / amp(tx)
    scale = np.max(np.abs(fixed))
    assert np.max(np.abs(moved - fixed)) < 1e-11 * scale
    # and the displacement matters at all: the unshifted object gives another field
    base, _ = forward.mom_solve(eps, WL.side, K0, tx, rx)
    base = base / amp(tx)
    assert np.max(np.abs(moved - base)) > 1e-3 * scale
    # the other axis's shift does not reproduce it
    other, _ = forward.mom_solve(np.roll(eps, -1, axis=1 - axis), WL.side, K0, tx, rx)
    other = other / amp(tx)
    assert np.max(np.abs(moved - other)) > 1e-3 * scale


def test_data_change_is_linear_in_small_position_errors():
    """The field is smooth in the antenna positions, so the relative data change
    ||E(x0 + s u) - E(x0)|| / ||E(x0)|| of one displacement direction u grows linearly in s for
    displacements far below a wavelength (first order of the Taylor expansion; the mm-scale study
    reports it per sigma)."""
    eps, _ = _shift_case()
    tx = si.antenna_positions(8, WL.radius)
    rx = si.antenna_positions(12, WL.radius)
    dt, dr = si.draw_position_errors(7, 8, 12, 1.0)     # direction; unit standard deviation
    e0, _ = forward.mom_solve(eps, WL.side, K0, tx, rx)
    ch = []
    for s in (1e-3, 2e-3, 3e-3):
        e, _ = forward.mom_solve(eps, WL.side, K0, tx + s * dt, rx + s * dr)
        ch.append(np.linalg.norm(e - e0) / np.linalg.norm(e0))
    assert 1e-4 < ch[0] < 1e-1
    assert abs(ch[1] / ch[0] - 2.0) < 0.02 and abs(ch[2] / ch[0] - 3.0) < 0.03
