"""Pins of the oracle's Green's operators (Sec. 2.1) against library routines,
quadrature, brute force and symmetry."""
import json
import os

import mpmath
import numpy as np
import pytest
from scipy import integrate, special

import seeded_inputs as si
from oracle import operators as ops

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_paper_geometry_is_two_wavelengths():
    # 1.5 m at 400 MHz is 2.0 wavelengths (Sec. 4); the workloads use 2 lambda.
    lam = si.C0 / GOLD["freq_hz"]["value"]
    assert abs(GOLD["doi_side_m"]["value"] / lam - 2.0) < 0.002
    assert si.WORKLOADS["paper"].n_tx == GOLD["n_tx"]["value"]
    assert si.WORKLOADS["paper"].radius_wl == GOLD["radius_wl"]["value"]
    assert si.WORKLOADS["paper"].M == GOLD["grid"]["value"]


@pytest.mark.parametrize("x", [0.05, 0.3, 1.7, 9.2, 40.0])
def test_hankel_against_mpmath(x):
    for n in (0, 1):
        ref = complex(mpmath.hankel1(n, x))
        assert abs(special.hankel1(n, x) - ref) <= 1e-14 * max(1.0, abs(ref))


@pytest.mark.parametrize("x", [0.1, 1.0, 3.3, 25.0])
def test_wronskian(x):
    w = special.jv(1, x) * special.yv(0, x) - special.jv(0, x) * special.yv(1, x)
    assert abs(w - 2.0 / (np.pi * x)) < 1e-14


def test_self_term_matches_quadrature():
    # k0^2 * integral over a disc of radius a of (i/4) H0(k0 rho); log singular at 0.
    k0 = 2 * np.pi
    for h in (1 / 32, 1 / 8):
        a = h / np.sqrt(np.pi)
        re = integrate.quad(lambda r: -0.25 * special.yv(0, k0 * r) * 2 * np.pi * r, 0, a,
                            limit=200, epsabs=1e-15)[0]
        im = integrate.quad(lambda r: 0.25 * special.jv(0, k0 * r) * 2 * np.pi * r, 0, a,
                            epsabs=1e-15)[0]
        ref = k0 ** 2 * (re + 1j * im)
        assert abs(ops.self_term(k0, h) - ref) < 1e-10
    # small-cell limit: the self term tends to 0, e.g. about 0.0172 + 0.0096i at h = lambda/32
    v = ops.self_term(2 * np.pi, 1 / 32)
    assert abs(v - (0.0172 + 0.0096j)) < 2e-4


def test_cell_factor_matches_quadrature():
    # Integral over a disc of H0(k0 |r - r'|) seen from outside = (2 pi a / k0) J1(k0 a) H0(k0 rho).
    k0, h, rho = 2 * np.pi, 0.1, 0.37
    a = h / np.sqrt(np.pi)

    def integrand(r, phi, part):
        d = np.sqrt(rho ** 2 + r ** 2 - 2 * rho * r * np.cos(phi))
        v = 0.25j * special.hankel1(0, k0 * d) * r
        return v.real if part == 0 else v.imag

    re = integrate.dblquad(lambda phi, r: integrand(r, phi, 0), 0, a, 0, 2 * np.pi, epsabs=1e-13)[0]
    im = integrate.dblquad(lambda phi, r: integrand(r, phi, 1), 0, a, 0, 2 * np.pi, epsabs=1e-13)[0]
    ref = k0 ** 2 * (re + 1j * im)
    got = ops.cell_factor(k0, h) * special.hankel1(0, k0 * rho)
    assert abs(got - ref) < 1e-10 * abs(ref) + 1e-13


def test_gd_symmetric_not_hermitian():
    G = ops.gd_dense(6, 0.05, 2 * np.pi)
    assert np.allclose(G, G.T, atol=0, rtol=1e-15)
    assert not np.allclose(G, G.conj().T)


@pytest.mark.parametrize("M", [4, 7, 16])
def test_fft_conv_equals_direct_sum(M):
    rng = np.random.default_rng(M)
    h, k0 = 0.9 / M, 2 * np.pi
    x = rng.standard_normal((3, M, M)) + 1j * rng.standard_normal((3, M, M))
    ghat = ops.gd_spectrum(M, h, k0)
    fast = ops.gd_apply(x, ghat)
    G = ops.gd_dense(M, h, k0)
    # brute-force direct sum of the definition, one output pixel at a time
    direct = np.einsum("mn,pn->pm", G, x.reshape(3, -1)).reshape(3, M, M)
    assert np.max(np.abs(fast - direct)) <= 1e-13 * np.max(np.abs(direct))


def test_gd_adjoint_dot_product():
    M = 9
    rng = np.random.default_rng(1)
    ghat = ops.gd_spectrum(M, 0.1, 2 * np.pi)
    x = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    y = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    lhs = np.vdot(y, ops.gd_apply(x, ghat))
    rhs = np.vdot(ops.gd_adjoint_apply(y, ghat), x)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_gs_adjoint_and_geometry():
    M, side, k0 = 8, 1.0, 2 * np.pi
    rx = si.antenna_positions(5, 3.0)
    gs = ops.gs_matrix(rx, M, side, k0)
    # first receiver at angle 0; pixel (i, j) centre at -side/2 + (idx+1/2) h
    pos = ops.pixel_positions(M, side)
    assert np.allclose(pos[0], [-side / 2 + side / 16, -side / 2 + side / 16])
    assert np.allclose(pos[1], [-side / 2 + 3 * side / 16, -side / 2 + side / 16])   # j is x
    assert np.allclose(pos[M], [-side / 2 + side / 16, -side / 2 + 3 * side / 16])   # i is y
    d = np.hypot(rx[0, 0] - pos[5, 0], rx[0, 1] - pos[5, 1])
    assert abs(gs[0, 5] - ops.cell_factor(k0, side / M) * special.hankel1(0, k0 * d)) < 1e-15
    rng = np.random.default_rng(2)
    x = rng.standard_normal(M * M) + 1j * rng.standard_normal(M * M)
    y = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    assert abs(np.vdot(y, gs @ x) - np.vdot(gs.conj().T @ y, x)) < 1e-12 * abs(np.vdot(y, gs @ x))


def test_incident_field_unit_at_centre():
    k0 = 2 * np.pi
    tx = si.antenna_positions(4, 3.0)
    M = 2
    einc = ops.einc_matrix(tx, M, 1e-9, k0)    # all pixels at the centre
    assert np.allclose(np.abs(einc), 1.0, atol=1e-6)
