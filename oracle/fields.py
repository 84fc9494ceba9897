"""Spatially correlated per-pixel Zernike fields by FFT filtering of white
noise.

The paper needs alpha(x) for every pixel with the right spatial correlation
and draws it on an anchor grid from a precomputed correlation matrix, then
interpolates (Sec. 3.4).  The hot path here instead colours seeded white noise
with a Gaussian power spectral density, one independent plane per Zernike mode
(the diagonal of R_Z, Sec. 2.2), scaled to the Noll variance times
(D/r0)^(5/3).  Readings recorded with the design notes:

* grid: Nf = smallest 2^a 3^b 5^c >= N + ceil(4 l) per axis (l = correlation
  length in pixels); the field is the top-left H x W crop of the periodic
  Nf_y x Nf_x field, so wrap-around correlation is below exp(-8);
* PSD: S(fy, fx) = exp(-2 pi^2 l^2 (fy^2 + fx^2)) with f = k/Nf wrapped to
  [-1/2, 1/2), normalised to mean(S) = 1, so that the periodic covariance
  IDFT(S) has c[0] = 1 and approximates exp(-|d|^2 / (2 l^2));
* field_p = crop(real(IDFT2(sqrt(S) DFT2(n_p)))) * sigma_j, n_p the Philox
  normals of plane p, plane p carrying Noll mode j = p + 2.

Parity: pinned (FFT filtering equals brute-force circular convolution;
sample periodogram and lag covariance match sigma^2 S and sigma^2 IDFT(S)).
"""
import math

import numpy as np

from .noll import noll_variance
from .philox import normal_grid


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
    """Periodic field real(IDFT2(sqrt(S) * DFT2(noise)))."""
    return np.real(np.fft.ifft2(np.sqrt(S) * np.fft.fft2(noise)))


def make_fields(H: int, W: int, d_over_r0: float, n_zernike: int, seed: int,
                corr_len: float = 16.0) -> np.ndarray:
    """Fields [n_zernike][H][W]: plane p is Noll mode j = p + 2."""
    Nfy, Nfx = grid_size(H, corr_len), grid_size(W, corr_len)
    S = psd(Nfy, Nfx, corr_len)
    out = np.empty((n_zernike, H, W), dtype=np.float64)
    for p in range(n_zernike):
        sigma = math.sqrt(noll_variance(p + 2) * d_over_r0 ** (5.0 / 3.0))
        f = colour(normal_grid(Nfy, Nfx, p, seed), S)
        out[p] = f[:H, :W] * sigma
    return out
