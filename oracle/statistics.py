"""The statistics a turbulence simulator is validated against (Sec. 4.1):
tilt correlation against separation (Evaluation 1) and the short- and
long-exposure PSFs (Evaluation 2).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module.

What the simulator should reproduce, per field model:

* tilt -- the Zernike tilt alpha_2 (x) and alpha_3 (y) moves the image by
  s alpha pixels, s = 2 q / pi; its variance per axis is s^2 V_2 (D/r0)^(5/3)
  pixels^2, which in units of (lambda/D)^2 is (4 / pi^2) V_2 (D/r0)^(5/3), the
  single-axis Z-tilt variance of Kolmogorov turbulence.
* tilt covariance against lag -- for the FFT model the periodic covariance
  c = IDFT(S) of the field PSD (separable: c(dy, dx) = c_y(dy) c_x(dx)); for
  the anchor model the covariance of bilinearly interpolated anchor values,
  sum_{i,i'} w_i(p) w_i'(p') R_s[i][i'], averaged over all pixel pairs at the
  lag (the interpolated field is not stationary inside a cell).
* exposure MTFs -- for an ensemble of aberrations alpha ~ N(0, R_Z (D/r0)^(5/3))
  (the simulator's own statistics), the long-exposure MTF |E OTF| and the
  mean short-exposure MTF E |OTF| of the pupil-FFT PSFs (Eq. 2).  For
  reference, Fried's Kolmogorov curves with every mode (the simulator keeps
  Noll modes 2..36): long exposure T(u) exp(-3.44 (D/r0)^(5/3) u^(5/3)), tilt
  removed T(u) exp(-3.44 (D/r0)^(5/3) u^(5/3) (1 - u^(1/3))), with T the
  diffraction MTF of a circular pupil and u the spatial frequency over the
  cut-off D / lambda.

Parity: pinned (Z-tilt variance against the literature value, the FFT-model
covariance against a lag average of an exactly known periodic field, the
anchor covariance against brute force, the diffraction MTF against the MTF of
the zero-aberration PSF, the Kolmogorov curves at their limits).
"""
import math

import numpy as np

from . import anchors, fields, noll, psf


def tilt_shift_variance(d_over_r0: float, q: float = 2.0) -> float:
    """Variance per axis of the tilt displacement, in pixels^2."""
    return (2.0 * q / math.pi) ** 2 * noll.noll_variance(2) * d_over_r0 ** (5.0 / 3.0)


def fft_model_correlation(N: int, lags, corr_len: float = 16.0) -> np.ndarray:
    """Correlation of an FFT-model plane at lags along an axis of length N."""
    Nf = fields.grid_size(N, corr_len)
    f = np.fft.fftfreq(Nf)
    s = np.exp(-2.0 * np.pi ** 2 * corr_len ** 2 * f ** 2)
    c = np.real(np.fft.ifft(s / s.mean()))
    return c[np.asarray(lags) % Nf]


def _interp_weights(N: int, G: int):
    """Anchor index and weight of the two anchors bracketing each coordinate."""
    g = np.arange(N) * ((G - 1) / (N - 1)) if N > 1 else np.zeros(1)
    i0 = np.minimum(np.floor(g).astype(np.int64), G - 2)
    t = g - i0
    return np.stack([i0, i0 + 1], 1), np.stack([1.0 - t, t], 1)


def anchor_model_covariance(G: int, H: int, W: int, lags, axis: int, corr_len: float = 2.0) -> np.ndarray:
    """Mean over pixel pairs (p, p + lag along axis; 0 = rows, 1 = columns) of
    Cov(alpha(p), alpha(p + lag)) / C_jj for any plane j: the covariance of
    the bilinear interpolation of anchors correlated by R_s."""
    R = anchors.anchor_correlation(G, corr_len).reshape(G, G, G, G)
    iy, wy = _interp_weights(H, G)
    ix, wx = _interp_weights(W, G)
    out = []
    for lag in lags:
        if axis == 1:
            y0, x0, y1, x1 = np.arange(H), np.arange(W - lag), np.arange(H), np.arange(lag, W)
        else:
            y0, x0, y1, x1 = np.arange(H - lag), np.arange(W), np.arange(lag, H), np.arange(W)
        tot = 0.0
        for a in range(2):
            for b in range(2):
                for c in range(2):
                    for d in range(2):
                        # sum over rows and columns of w w' R[ay, bx, cy', dx'], separable sums
                        wr = wy[y0, a][:, None] * wy[y1, c][:, None]
                        wc = wx[x0, b][None, :] * wx[x1, d][None, :]
                        Rsub = R[iy[y0, a][:, None], ix[x0, b][None, :], iy[y1, c][:, None], ix[x1, d][None, :]]
                        tot += np.sum(wr * wc * Rsub)
        out.append(tot / (len(y0) * len(x0)))
    return np.array(out)


def diffraction_mtf(u) -> np.ndarray:
    """MTF of a circular pupil, u = frequency / cut-off in [0, 1]."""
    u = np.clip(np.asarray(u, dtype=np.float64), 0.0, 1.0)
    return (2.0 / np.pi) * (np.arccos(u) - u * np.sqrt(1.0 - u * u))


def kolmogorov_long_exposure_mtf(u, d_over_r0: float) -> np.ndarray:
    u = np.asarray(u, dtype=np.float64)
    return diffraction_mtf(u) * np.exp(-3.44 * d_over_r0 ** (5.0 / 3.0) * u ** (5.0 / 3.0))


def kolmogorov_short_exposure_mtf(u, d_over_r0: float) -> np.ndarray:
    u = np.asarray(u, dtype=np.float64)
    return diffraction_mtf(u) * np.exp(-3.44 * d_over_r0 ** (5.0 / 3.0) * u ** (5.0 / 3.0) * (1.0 - u ** (1.0 / 3.0)))


def radial_mtf(otf: np.ndarray, q: float, u_points) -> np.ndarray:
    """Azimuthal mean of |otf| (unshifted FFT grid of side n, DC at [0, 0],
    normalised to 1 at DC) at u = frequency / cut-off, with the cut-off at 1/q
    cycles per pixel; linear interpolation between unit-width radial bins."""
    n = otf.shape[0]
    f = np.fft.fftfreq(n)
    r = np.hypot(f[:, None], f[None, :]) * n           # radius in bins
    a = np.abs(otf) / np.abs(otf[0, 0])
    rb = np.rint(r).astype(np.int64)
    prof = np.bincount(rb.ravel(), a.ravel()) / np.bincount(rb.ravel())
    want = np.asarray(u_points, dtype=np.float64) / q * n   # u -> bins
    return np.interp(want, np.arange(prof.size), prof)


def exposure_mtfs(d_over_r0: float, n_draws: int, seed: int, u_points, n_modes: int = 35, P: int = 49,
                  Np: int = 32, Q: int = 2, pad: int = 128, full_covariance: bool = False):
    """Long-exposure MTF |mean OTF| and mean short-exposure MTF mean |OTF| of
    pupil-FFT PSFs with tilt (Noll modes 2 .. n_modes + 1), alpha drawn from
    the simulator's covariance (independent modes, or Noll's full R_Z)."""
    rng = np.random.default_rng(seed)
    C = anchors.mode_covariance(n_modes) if full_covariance else np.diag(
        [noll.noll_variance(j) for j in range(2, n_modes + 2)])
    L = np.linalg.cholesky(C) * d_over_r0 ** (5.0 / 6.0)
    modes = range(2, n_modes + 2)
    mean_otf = np.zeros((pad, pad), dtype=np.complex128)
    mean_mag = np.zeros((pad, pad))
    for start in range(0, n_draws, 256):
        m = min(256, n_draws - start)
        alpha = rng.standard_normal((m, n_modes)) @ L.T
        h = psf.psf_from_zernike(alpha, modes, Np, Q, P)
        otf = np.fft.fft2(h, s=(pad, pad))
        mean_otf += otf.sum(0)
        mean_mag += (np.abs(otf) / np.abs(otf[:, :1, :1])).sum(0)
    mean_otf /= n_draws
    mean_mag /= n_draws
    return radial_mtf(mean_otf, Q, u_points), radial_mtf(mean_mag, Q, u_points)


def simulator_model_mtfs(d_over_r0: float, n_draws: int, seed: int, u_points, n_modes: int = 35, P: int = 33,
                         window: int = 49, Np: int = 32, Q: int = 2, pad: int = 128, full_covariance: bool = False):
    """The exposure MTFs of the simulator's own model of a point source, with
    the P2S network replaced by the exact PSF: the PSF of Noll modes
    4 .. n_modes + 1 on the basis' P x P support (normalised to unit sum, as
    the basis dataset is), centred in a window x window patch and moved by the
    tilt warp (bilinear, displacement s (alpha_2, alpha_3)).  Returns
    (|mean OTF|, mean |OTF|) at u_points."""
    from . import warp
    rng = np.random.default_rng(seed)
    C = anchors.mode_covariance(n_modes) if full_covariance else np.diag(
        [noll.noll_variance(j) for j in range(2, n_modes + 2)])
    L = np.linalg.cholesky(C) * d_over_r0 ** (5.0 / 6.0)
    off = (window - P) // 2
    mean_otf = np.zeros((pad, pad), dtype=np.complex128)
    mean_mag = np.zeros((pad, pad))
    for start in range(0, n_draws, 256):
        m = min(256, n_draws - start)
        alpha = rng.standard_normal((m, n_modes)) @ L.T
        h = psf.psf_from_zernike(alpha[:, 2:], range(4, n_modes + 2), Np, Q, P)
        patches = np.zeros((m, window, window))
        for i in range(m):
            img = np.zeros((window, window))
            img[off:off + P, off:off + P] = h[i]
            dx = np.full((window, window), warp.displacement(alpha[i, 0], Q))
            dy = np.full((window, window), warp.displacement(alpha[i, 1], Q))
            patches[i] = warp.warp(img, dx, dy)
        otf = np.fft.fft2(patches, s=(pad, pad))
        mean_otf += otf.sum(0)
        mean_mag += (np.abs(otf) / np.abs(otf[:, :1, :1])).sum(0)
    mean_otf /= n_draws
    mean_mag /= n_draws
    return radial_mtf(mean_otf, Q, u_points), radial_mtf(mean_mag, Q, u_points)
