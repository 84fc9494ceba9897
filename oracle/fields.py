"""Spatially correlated per-pixel Zernike fields by FFT filtering of white
noise.

The paper needs alpha(x) for every pixel with the right spatial correlation
and draws it on an anchor grid from a precomputed correlation matrix, then
interpolates (Sec. 3.4).  The hot path here instead colours seeded white noise
with a Gaussian power spectral density, one independent plane per Zernike mode
(the diagonal of R_Z, Sec. 2.2), scaled to the Noll variance times
(D/r0)^(5/3).  Readings recorded with the design notes:

* grid: Nf = smallest 2^a 3^b 5^c >= N + ceil(4 l) per axis (l = correlation
  length in pixels); a field is the top-left H x W crop of a periodic
  Nf_y x Nf_x field, so wrap-around correlation is below exp(-8);
* PSD: S(fy, fx) = exp(-2 pi^2 l^2 (fy^2 + fx^2)) with f = k/Nf wrapped to
  [-1/2, 1/2), normalised to mean(S) = 1, so that the periodic covariance
  IDFT(S) has c[0] = 1 and approximates exp(-|d|^2 / (2 l^2));
* the white noise is drawn in the frequency domain: for plane pair q,
  N_q(k) = complex standard normal per bin (see ``philox``), and
      G_q(x) = (1 / sqrt(Nf_y Nf_x)) sum_k sqrt(S(k)) N_q(k) exp(2 pi i k.x / Nf);
  Re G_q and Im G_q are two independent stationary Gaussian fields, each with
  covariance IDFT(S) (S is even), which become planes 2q and 2q + 1:
      field_p = crop(Re or Im of G_{p div 2}) * sigma_j,  j = p + 2.

Parity: pinned (the transform equals the brute-force sum on a tiny grid;
sample periodogram and lag covariance match S and IDFT(S); real and imaginary
parts and different pairs are uncorrelated).
"""
import math

import numpy as np

from .noll import noll_variance
from .philox import complex_normal_bins


def is_5smooth(n: int) -> bool:
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def grid_size(N: int, corr_len: float = 16.0) -> int:
    n = N + int(math.ceil(4.0 * corr_len))
    while not is_5smooth(n):
        n += 1
    return n


def psd(Nfy: int, Nfx: int, corr_len: float = 16.0) -> np.ndarray:
    fy = np.fft.fftfreq(Nfy)[:, None]
    fx = np.fft.fftfreq(Nfx)[None, :]
    S = np.exp(-2.0 * np.pi ** 2 * corr_len ** 2 * (fy ** 2 + fx ** 2))
    return S / S.mean()


def colour(noise: np.ndarray, S: np.ndarray) -> np.ndarray:
    """G = (1/sqrt(N)) sum_k sqrt(S_k) noise_k exp(+2 pi i k.x / Nf): numpy's
    ifft2 carries 1/N, hence the factor sqrt(N)."""
    n = noise.shape[0] * noise.shape[1]
    return np.fft.ifft2(np.sqrt(S) * noise) * math.sqrt(n)


def make_fields(H: int, W: int, d_over_r0: float, n_zernike: int, seed: int,
                corr_len: float = 16.0) -> np.ndarray:
    """Fields [n_zernike][H][W]: plane p is Noll mode j = p + 2."""
    Nfy, Nfx = grid_size(H, corr_len), grid_size(W, corr_len)
    S = psd(Nfy, Nfx, corr_len)
    out = np.empty((n_zernike, H, W), dtype=np.float64)
    for q in range((n_zernike + 1) // 2):
        G = colour(complex_normal_bins(Nfy, Nfx, q, seed), S)[:H, :W]
        for p, part in ((2 * q, G.real), (2 * q + 1, G.imag)):
            if p < n_zernike:
                out[p] = part * math.sqrt(noll_variance(p + 2) * d_over_r0 ** (5.0 / 3.0))
    return out
