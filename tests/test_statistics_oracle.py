"""Pins of the oracle's validation statistics (paper Sec. 4.1): tilt
variance and covariance against separation, and the exposure MTFs.

Each test checks the oracle against something other than itself: a
literature constant, a second route to the same quantity, brute force on a
small grid, or a closed form that a special case reduces to.
"""
import math

import numpy as np
import pytest

from oracle import anchors, fields, psf, statistics


def test_tilt_variance_is_the_kolmogorov_z_tilt():
    """Single-axis Z-tilt variance of Kolmogorov turbulence: 0.182 (D/r0)^(5/3)
    (lambda/D)^2 (Fried 1965; Tyler 1994, JOSA A 11, 358).  The simulator's
    tilt s alpha_2 with s = 2 q / pi pixels and q pixels per lambda/D must give
    it (catches a wrong displacement scale or a wrong tilt variance)."""
    for q in (2.0, 3.0):
        for d in (0.5, 3.0, 7.0):
            var_lod = statistics.tilt_shift_variance(d, q) / q ** 2
            assert var_lod == pytest.approx(0.182 * d ** (5.0 / 3.0), rel=5e-3)


def test_psf_tilt_moves_by_the_warp_displacement():
    """A tilt alpha_2 = a in the pupil phase moves the pupil-FFT PSF by
    2 Q a / pi pixels, the displacement the warp applies (both conventions
    meet in the exposure statistics)."""
    for a in (0.4, -0.9):
        h = psf.psf_from_zernike(np.array([a, 0.0]), [2, 3], Np=32, Q=2, P=49)
        R = 24
        xs = np.arange(-R, R + 1)
        cx = float(np.sum(h.sum(0) * xs))
        cy = float(np.sum(h.sum(1) * xs))
        assert abs(abs(cx) - 4.0 * abs(a) / math.pi) < 0.02
        assert abs(cy) < 1e-9


def test_fft_model_correlation_matches_the_2d_transform():
    """The 1-D covariance c_x equals row 0 of the 2-D periodic covariance
    IDFT(S) of the full PSD (a separable PSD; catches a wrong normalisation or
    grid), and is 1 at lag 0."""
    N, ell = 100, 6.0
    Nf = fields.grid_size(N, ell)
    c2 = np.real(np.fft.ifft2(fields.psd(Nf, Nf, ell)))
    lags = np.arange(0, 40)
    got = statistics.fft_model_correlation(N, lags, ell)
    assert got[0] == pytest.approx(1.0, abs=1e-12)
    assert np.allclose(got, c2[0, lags], rtol=0.0, atol=1e-12)


def test_anchor_model_covariance_brute_force():
    """Mean covariance at a lag of the interpolated anchor field equals the
    brute-force M R_s M^T, M the interpolation matrix built by interpolating
    unit anchor vectors (catches a wrong corner, weight or axis)."""
    G, H, W, ell = 4, 11, 14, 1.5
    M = np.stack([anchors.interpolate(np.eye(G * G)[:, [k]], G, H, W)[0].ravel() for k in range(G * G)], 1)
    Cpix = M @ anchors.anchor_correlation(G, ell) @ M.T
    idx = np.arange(H * W).reshape(H, W)
    for axis, lags in ((1, range(0, 6)), (0, range(0, 5))):
        got = statistics.anchor_model_covariance(G, H, W, list(lags), axis, ell)
        for k, lag in enumerate(lags):
            if axis == 1:
                a, b = idx[:, :W - lag].ravel(), idx[:, lag:].ravel()
            else:
                a, b = idx[:H - lag, :].ravel(), idx[lag:, :].ravel()
            assert got[k] == pytest.approx(float(np.mean(Cpix[a, b])), rel=1e-12)


U = [0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8]


def test_diffraction_mtf_matches_the_zero_aberration_psf():
    """The MTF of the pupil-FFT PSF with no aberration is the circular-pupil
    MTF (within the pupil's sampling on 32 points)."""
    h = psf.psf_from_zernike(np.zeros((1, 1)), [4], Np=32, Q=2, P=63)[0]
    got = statistics.radial_mtf(np.fft.fft2(h, s=(128, 128)), 2.0, U)
    assert np.max(np.abs(got - statistics.diffraction_mtf(U))) < 0.02


def test_kolmogorov_curves_limits():
    """Both Kolmogorov MTFs are the diffraction MTF at D/r0 = 0 and 1 at u = 0;
    the tilt-removed one lies above the long-exposure one; at the u where
    3.44 (D/r0)^(5/3) u^(5/3) = 1 the long-exposure MTF is T(u)/e."""
    u = np.array(U)
    assert np.allclose(statistics.kolmogorov_long_exposure_mtf(u, 0.0), statistics.diffraction_mtf(u))
    assert np.allclose(statistics.kolmogorov_short_exposure_mtf(u, 0.0), statistics.diffraction_mtf(u))
    assert statistics.kolmogorov_long_exposure_mtf(0.0, 5.0) == pytest.approx(1.0)
    assert np.all(statistics.kolmogorov_short_exposure_mtf(u, 3.0) > statistics.kolmogorov_long_exposure_mtf(u, 3.0))
    d = 3.0
    u1 = (1.0 / (3.44 * d ** (5.0 / 3.0))) ** 0.6
    assert statistics.kolmogorov_long_exposure_mtf(u1, d) == pytest.approx(statistics.diffraction_mtf(u1) / math.e)


def test_exposure_mtfs_tilt_only_closed_form():
    """With tilt alone the PSF is the diffraction PSF shifted by a Gaussian
    displacement of variance s^2 per axis, so the long-exposure MTF is
    T(u) exp(-2 pi^2 s^2 f^2) with f = u / q cycles per pixel, and the mean
    short-exposure MTF is T(u) (catches a wrong average or frequency axis)."""
    d = 2.0
    le, se = statistics.exposure_mtfs(d, 3000, 5, U, n_modes=2)
    s2 = statistics.tilt_shift_variance(d, 2.0)
    f = np.array(U) / 2.0
    want = statistics.diffraction_mtf(U) * np.exp(-2.0 * np.pi ** 2 * s2 * f ** 2)
    assert np.max(np.abs(le - want)) < 0.04
    assert np.max(np.abs(se - statistics.diffraction_mtf(U))) < 0.03


def test_exposure_mtfs_zero_turbulence_and_order():
    """No turbulence: both MTFs are the diffraction MTF; with turbulence the
    mean short-exposure MTF exceeds the long-exposure one."""
    le0, se0 = statistics.exposure_mtfs(0.0, 4, 1, U)
    assert np.max(np.abs(le0 - statistics.diffraction_mtf(U))) < 0.03
    assert np.allclose(le0, se0, atol=1e-12)
    le, se = statistics.exposure_mtfs(3.0, 512, 2, U)
    assert np.all(se[1:] > le[1:])
