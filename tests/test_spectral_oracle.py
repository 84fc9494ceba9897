"""Pins of the oracle's wavelength-dependent colour (paper Sec. 3.5): PSF
sampling at any q, the achromatic tilt, and the reduction to the grey
simulator when all channels share one basis and network.
"""
import math

import numpy as np
import pytest

import p2s_synth as S
from oracle import basis as obasis
from oracle import psf, spectral
from oracle.simulate import simulate as osimulate


def test_any_q_sampling_equals_the_padded_fft_for_integer_q():
    """The direct Fourier sum at integer q gives exactly the zero-padded FFT
    PSF (catches a wrong frequency scale or an axis swap)."""
    rng = np.random.default_rng(1)
    Np = 32
    _, _, mask = psf.pupil_grid(Np)
    phase = rng.standard_normal((3, Np, Np)) * 0.7
    for Q, P in ((2, 33), (3, 41)):
        a = psf.psf_from_phase(phase, mask, Q, P)
        b = psf.psf_from_phase_q(phase, mask, float(Q), P)
        assert np.max(np.abs(a - b)) < 1e-14


def test_airy_first_zero_at_1_22_q_pixels():
    """Unaberrated circular pupil: the first dark ring lies at 1.22 lambda/D,
    i.e. 1.22 q pixels, for a non-integer q (choose q so that it falls on the
    third pixel)."""
    Np, P = 96, 15
    _, _, mask = psf.pupil_grid(Np)
    q = 3.0 / 1.2197
    h = psf.psf_from_phase_q(np.zeros((Np, Np)), mask, q, P)
    R = P // 2
    assert h[R, R + 3] / h[R, R] < 3e-3
    assert h[R, R + 1] / h[R, R] > 0.3


def test_tilt_displacement_is_achromatic():
    """A reference-wavelength tilt alpha moves the PSF of every channel by the
    same 2 q_ref alpha / pi pixels (phase scaled by lambda_ref / lambda,
    sampling by lambda / lambda_ref), so one warp serves all channels."""
    a = 0.6
    want = 4.0 * a / math.pi
    R = 24
    xs = np.arange(-R, R + 1)
    for lam in spectral.WAVELENGTHS_NM + (spectral.REFERENCE_NM,):
        q, s = spectral.channel_sampling(lam)
        h = psf.psf_from_zernike(np.array([a, 0.0]), [2, 3], Np=64, Q=q, P=2 * R + 1, phase_scale=s)
        cx = abs(float(np.sum(h.sum(0) * xs)))
        assert cx == pytest.approx(want, rel=0.02), lam


def test_channel_sampling_values():
    q, s = spectral.channel_sampling(450.0)
    assert q == pytest.approx(2.0 * 450.0 / 525.0) and s == pytest.approx(525.0 / 450.0)
    q, s = spectral.channel_sampling(525.0)
    assert q == 2.0 and s == 1.0


def test_shared_channels_reduce_to_the_grey_simulator():
    """With one basis and one network for every channel the colour frame is
    the grey simulator's frame (the same fields, weights, blur and warp)."""
    z = S.standard_normals((256, 33), 3)
    basis, _ = obasis.pca_basis(obasis.dataset(z, np.full(256, 1.5), P=9), 8)
    Ws, bs = S.xavier_mlp((33, 16, 8), 2, bias_scale=0.02)
    img = S.blob_image(20, 23, 3, 1)
    grey = osimulate(img, 2.0, basis, Ws, bs, seed=4)["out"]
    col = spectral.simulate_spectral(img, 2.0, [basis] * 3, [Ws] * 3, [bs] * 3, seed=4)
    assert np.max(np.abs(col - grey)) < 1e-12
    with pytest.raises(ValueError):
        spectral.simulate_spectral(img, 2.0, [basis] * 2, [Ws] * 2, [bs] * 2, seed=4)


def test_spectral_pixels_equal_the_whole_frame():
    """The pixel-sampled colour frame equals the whole colour frame at every
    pixel of a small frame with different bases and networks per channel."""
    z = S.standard_normals((256, 33), 3)
    bases, Ws, bs = [], [], []
    for k, lam in enumerate(spectral.WAVELENGTHS_NM):
        q, s = spectral.channel_sampling(lam)
        bases.append(obasis.pca_basis(obasis.dataset(z, np.full(256, 1.5), P=9, Q=q, phase_scale=s), 8)[0])
        w, b = S.xavier_mlp((33, 16, 8), 10 + k, bias_scale=0.02)
        Ws.append(w)
        bs.append(b)
    img = S.blob_image(12, 15, 3, 2)
    full = spectral.simulate_spectral(img, 2.0, bases, Ws, bs, seed=6)
    pix = [(c, y, x) for c in range(3) for y in range(12) for x in range(15)]
    got = spectral.simulate_spectral_pixels(img, 2.0, bases, Ws, bs, 6, pix)
    assert np.max(np.abs(got - full.ravel())) < 1e-12
