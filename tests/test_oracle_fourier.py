"""Pins of the truncated Fourier basis (Sec. 2.3): Parseval, round trip,
numpy.fft, adjoint, and the paper's four-corner-block mode set."""
import numpy as np
import pytest

from oracle import fourier


def rand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("M,K", [(16, 7), (32, 9), (64, 15), (16, 6), (12, 12)])
def test_parseval_and_round_trip(M, K):
    rng = np.random.default_rng(M + K)
    a = rand(rng, (3, K, K))
    J = fourier.synthesize(a, M)
    assert abs(np.sum(np.abs(J) ** 2) - M * M * np.sum(np.abs(a) ** 2)) < 1e-10 * np.sum(np.abs(J) ** 2)
    assert np.max(np.abs(fourier.analyze(J, K) - a)) < 1e-12


@pytest.mark.parametrize("M,K", [(16, 7), (32, 9), (16, 8)])
def test_equals_numpy_ifft_of_zero_filled_spectrum(M, K):
    rng = np.random.default_rng(3)
    a = rand(rng, (K, K))
    spec = np.zeros((M, M), complex)
    k = fourier.modes(K) % M
    spec[np.ix_(k, k)] = a
    ref = M * M * np.fft.ifft2(spec)
    assert np.max(np.abs(fourier.synthesize(a, M) - ref)) < 1e-12 * np.max(np.abs(ref))
    J = rand(rng, (M, M))
    ref_a = np.fft.fft2(J)[np.ix_(k, k)] / (M * M)
    assert np.max(np.abs(fourier.analyze(J, K) - ref_a)) < 1e-13


def test_synthesis_adjoint_dot_product():
    rng = np.random.default_rng(4)
    M, K = 20, 9
    x, y = rand(rng, (K, K)), rand(rng, (M, M))
    lhs = np.vdot(y, fourier.synthesize(x, M))
    rhs = np.vdot(fourier.synth_adjoint(y, K), x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_corner_set_is_four_mf_blocks():
    # Sec. 2.3: four M_F x M_F blocks at the corners of the DFT spectrum, M_0 = 4 M_F^2.
    M, MF = 64, 7
    k = fourier.modes(2 * MF) % M
    mask = np.zeros((M, M), bool)
    mask[np.ix_(k, k)] = True
    idx = np.arange(M)
    corner = (idx < MF) | (idx >= M - MF)
    assert np.array_equal(mask, corner[:, None] & corner[None, :])
    assert mask.sum() == 4 * MF * MF


def test_centred_odd_set():
    assert list(fourier.modes(5)) == [-2, -1, 0, 1, 2]
    assert list(fourier.modes(4)) == [-2, -1, 0, 1]
