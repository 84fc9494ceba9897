"""Spatially varying blur (Sec. 3.1).

Exact form (Eq. 3): y_n = h_n^T x, the PSF h_n of pixel n applied around it.
Basis form (Eq. 4-5): h_n = sum_m beta_{m,n} phi_m, hence
y_n = sum_m beta_{m,n} (phi_m^T x): M invariant convolutions and a per-pixel
multiply-add.

Readings recorded with the design notes: PSF tap b[i][j] sits at offset
u = (i - R, j - R) from the centre, R = (P-1)/2, and acts as a true
convolution, y(x) = sum_u b(u) I(x - u); the weights of the output pixel are
used (gather form of the rows of H); image borders replicate the edge pixel.

Parity: pinned (one-hot weights equal a brute-force convolution and
scipy.ndimage.convolve; a complete orthonormal basis with projection weights
equals the exact per-pixel blur; constants are preserved by normalised PSFs).
"""
import numpy as np
from numpy.lib.stride_tricks import sliding_window_view


def _windows(image: np.ndarray, P: int) -> np.ndarray:
    """win[y, x, a, b] = I(clamp(y + R - a), clamp(x + R - b)) -- the P x P
    neighbourhood of (y, x) ordered so that a dot product with a PSF b[a][b]
    is the convolution sum_u b(u) I(x - u)."""
    R = (P - 1) // 2
    padded = np.pad(np.asarray(image, dtype=np.float64), R, mode="edge")
    win = sliding_window_view(padded, (P, P))       # padded[y + a', x + b']
    return win[:, :, ::-1, ::-1]                     # a' = P-1-a


def invariant_conv(image: np.ndarray, psf: np.ndarray) -> np.ndarray:
    """phi^T x for every pixel: one spatially invariant convolution."""
    P = psf.shape[-1]
    return np.einsum("yxab,ab->yx", _windows(image, P), psf)


def basis_blur(image: np.ndarray, basis: np.ndarray, w: np.ndarray, rows_per_chunk: int = 64) -> np.ndarray:
    """Eq. 5: sum_k w_k(x) (b_k conv I)(x).  image [H][W], basis [K][P][P],
    w [H][W][K] -> [H][W].  The K convolutions are one matrix product per
    band of output rows."""
    H, W = image.shape
    K, P, _ = basis.shape
    w = np.asarray(w, dtype=np.float64).reshape(H, W, K)
    Bm = np.asarray(basis, dtype=np.float64).reshape(K, P * P).T     # [U][K]
    win = _windows(image, P)
    out = np.empty((H, W), dtype=np.float64)
    for y0 in range(0, H, rows_per_chunk):
        y1 = min(H, y0 + rows_per_chunk)
        patches = win[y0:y1].reshape((y1 - y0) * W, P * P)
        conv = patches @ Bm                                          # [pix][K] = b_k conv I
        out[y0:y1] = np.sum(conv * w[y0:y1].reshape(-1, K), axis=1).reshape(y1 - y0, W)
    return out


def exact_blur(image: np.ndarray, psfs: np.ndarray) -> np.ndarray:
    """Eq. 3 with a PSF per pixel: psfs [H][W][P][P] -> [H][W]."""
    P = psfs.shape[-1]
    return np.einsum("yxab,yxab->yx", _windows(image, P), np.asarray(psfs, dtype=np.float64))


def projection_weights(psfs: np.ndarray, basis: np.ndarray) -> np.ndarray:
    """beta_k(x) = <h_x, phi_k>: psfs [..., P, P], basis [K][P][P] -> [..., K]."""
    K, P, _ = basis.shape
    return np.asarray(psfs, dtype=np.float64).reshape(-1, P * P) @ basis.reshape(K, P * P).T \
        if psfs.ndim == 3 else \
        np.tensordot(np.asarray(psfs, dtype=np.float64), np.asarray(basis, dtype=np.float64), axes=([-2, -1], [1, 2]))
