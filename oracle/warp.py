"""Tilt displacement (Sec. 2.2 and 3.3): the first two Zernike coefficients
shift pixels after the high-order blur.

Readings recorded with the design notes: alpha_2 displaces along x (columns)
and alpha_3 along y (rows); with Nyquist image sampling (Q = 2 pixels per
lambda/D) a Noll-normalised tilt coefficient alpha moves the image by
2 Q alpha / pi pixels; the output pixel (y, x) samples the blurred image at
(y + d_y, x + d_x) by bilinear interpolation, sample positions clamped to the
image (replicate border).

Parity: pinned (zero tilt is the identity; integer shifts are exact shifts
with clamped edges; fractional shifts equal scipy.ndimage.map_coordinates with
order 1 and mode 'nearest').
"""
import numpy as np


def displacement(alpha: np.ndarray, q: float = 2.0) -> np.ndarray:
    return (2.0 * q / np.pi) * np.asarray(alpha, dtype=np.float64)


def warp(image: np.ndarray, dx: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """Bilinear resampling of image [H][W] at (y + dy, x + dx), in pixels."""
    H, W = image.shape
    img = np.asarray(image, dtype=np.float64)
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    sx = np.clip(xx + dx, 0.0, W - 1.0)
    sy = np.clip(yy + dy, 0.0, H - 1.0)
    x0 = np.floor(sx).astype(np.int64)
    y0 = np.floor(sy).astype(np.int64)
    x1 = np.minimum(x0 + 1, W - 1)
    y1 = np.minimum(y0 + 1, H - 1)
    fx = sx - x0
    fy = sy - y0
    top = (1.0 - fx) * img[y0, x0] + fx * img[y0, x1]
    bot = (1.0 - fx) * img[y1, x0] + fx * img[y1, x1]
    return (1.0 - fy) * top + fy * bot


def tilt_warp(image: np.ndarray, alpha2: np.ndarray, alpha3: np.ndarray, q: float = 2.0) -> np.ndarray:
    return warp(image, displacement(alpha2, q), displacement(alpha3, q))
