"""The paper's own field model (Sec. 3.4, "Interpolation across the grid",
with R_Z of Sec. 2.2): Zernike coefficients drawn jointly on a G x G grid of
anchor points from a precomputed correlation matrix, then carried to every
pixel by bilinear interpolation of the coefficients (interpolation in the
phase domain, not of PSFs).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module.

Readings (each recorded with the design notes):

* mode covariance -- Noll's full R_Z, cross terms included (Noll 1976).  Modes
  j, j' of radial orders n, n' and azimuthal frequencies m, m' covary only when
  m = m' and either m = 0 or j, j' have the same parity (both cos or both sin
  terms); then, per (D/r0)^(5/3),

      C_jj' = K (-1)^((n + n' - 2m)/2) sqrt((n+1)(n'+1)) Gamma((n + n' - 5/3)/2)
              / [Gamma((n - n' + 17/3)/2) Gamma((n' - n + 17/3)/2) Gamma((n + n' + 23/3)/2)],

  whose diagonal is the variance of ``noll``; K is the constant of ``noll``.
* spatial correlation between anchors -- the paper takes it from angle-of-
  arrival statistics whose formulas it does not print, so a stand-in is used:
  rho(d) = exp(-(d / l)^(5/3)), d the distance between two anchors in anchor
  spacings, l = corr_len (2 by default), the same for every mode.  It is
  positive definite on the plane (the characteristic function of a symmetric
  5/3-stable law) and follows Kolmogorov's 5/3 structure-function law at
  short range.
* joint law -- Cov(alpha_j(p), alpha_j'(q)) = rho(d_pq) C_jj' (D/r0)^(5/3): the
  Kronecker product of the G^2 x G^2 anchor correlation matrix and R_Z.
* draw -- A = L_s E L_Z^T (D/r0)^(5/6) with L_s, L_Z the lower Cholesky
  factors of the two matrices and E [G^2][n] standard normals, so that
  Cov(vec A) = (L_Z (x) L_s)(L_Z (x) L_s)^T = C_Z (x) R_s.
* normals -- E[p][i] (anchor p = a G + b, plane i = Noll mode i + 2) from
  Philox4x32-10 with key (seed mod 2^32, seed >> 32) and counter
  (p, i >> 1, 0, 1), Box-Muller on outputs o0, o1 as in ``philox``:
  sqrt(-2 ln u_a) cos(2 pi u_b) for even i, the sine for odd i.  The last
  counter word keeps these draws apart from the frequency-domain noise.
* anchors -- anchor (a, b) sits at pixel (a (H-1)/(G-1), b (W-1)/(G-1)): the
  grid spans the image from corner to corner, so every pixel lies inside one
  anchor cell (a single pixel row or column takes anchor row or column 0).
* interpolation -- bilinear over that cell, per plane.

Parity: pinned.  R_Z's radial part against a quadrature of the Bessel-product
integral of Noll's Fourier representation, its signs and selection rules
against a real-space double integral of the 5/3 structure function over the
pupil; the draw against the exact covariance of its linear map; the
interpolation by exactness at the anchors and on planar fields.
"""
import math

import numpy as np

from .noll import KC
from .philox import philox4x32_10
from .zernike import noll_to_nm

THIRDS_5 = 5.0 / 3.0


def mode_covariance(n_planes: int) -> np.ndarray:
    """R_Z of Noll modes 2 .. n_planes + 1 (plane i = mode i + 2), per
    (D/r0)^(5/3): [n_planes][n_planes]."""
    C = np.zeros((n_planes, n_planes))
    for p in range(n_planes):
        j = p + 2
        n, m = noll_to_nm(j)
        for q in range(n_planes):
            jj = q + 2
            nn, mm = noll_to_nm(jj)
            if m != mm or (m != 0 and (j - jj) % 2 != 0):
                continue
            sign = -1.0 if ((n + nn - 2 * m) // 2) % 2 else 1.0
            g = (math.gamma((n + nn - THIRDS_5) / 2.0)
                 / (math.gamma((n - nn + 17.0 / 3.0) / 2.0) * math.gamma((nn - n + 17.0 / 3.0) / 2.0)
                    * math.gamma((n + nn + 23.0 / 3.0) / 2.0)))
            C[p, q] = KC * sign * math.sqrt((n + 1.0) * (nn + 1.0)) * g
    return C


def anchor_correlation(G: int, corr_len: float = 2.0) -> np.ndarray:
    """R_s[p][q] = exp(-(d_pq / corr_len)^(5/3)), anchors p = a G + b."""
    a, b = np.divmod(np.arange(G * G), G)
    d = np.hypot(a[:, None] - a[None, :], b[:, None] - b[None, :])
    return np.exp(-(d / corr_len) ** THIRDS_5)


def anchor_normals(G: int, n_planes: int, seed: int) -> np.ndarray:
    """E [G^2][n_planes] of standard normals (counter (p, i >> 1, 0, 1))."""
    p = np.arange(G * G, dtype=np.uint64)[:, None]
    pair = np.arange((n_planes + 1) // 2, dtype=np.uint64)[None, :]
    o0, o1, _, _ = philox4x32_10(p, pair, np.uint64(0), np.uint64(1), seed & 0xFFFFFFFF,
                                 (seed >> 32) & 0xFFFFFFFF)
    ua = (np.floor(o0.astype(np.float64) / 256.0) + 1.0) * 2.0 ** -24
    ub = np.floor(o1.astype(np.float64) / 256.0) * 2.0 ** -24
    rad = np.sqrt(-2.0 * np.log(ua))
    E = np.empty((G * G, 2 * pair.shape[1]))
    E[:, 0::2] = rad * np.cos(2.0 * np.pi * ub)
    E[:, 1::2] = rad * np.sin(2.0 * np.pi * ub)
    return E[:, :n_planes]


def anchor_coefficients(E: np.ndarray, G: int, d_over_r0: float, corr_len: float = 2.0) -> np.ndarray:
    """A = L_s E L_Z^T (D/r0)^(5/6): coefficients [G^2][n_planes] at the
    anchors for given normals E."""
    Ls = np.linalg.cholesky(anchor_correlation(G, corr_len))
    Lz = np.linalg.cholesky(mode_covariance(E.shape[1]))
    return (Ls @ E @ Lz.T) * d_over_r0 ** (5.0 / 6.0)


def interpolate(A: np.ndarray, G: int, H: int, W: int) -> np.ndarray:
    """Bilinear interpolation of anchor values A [G^2][n] to planes
    [n][H][W]."""
    def axis(N):
        g = np.arange(N) * ((G - 1) / (N - 1)) if N > 1 else np.zeros(1)
        i0 = np.minimum(np.floor(g).astype(np.int64), G - 2)
        return i0, g - i0
    ay, ty = axis(H)
    ax, tx = axis(W)
    V = A.T.reshape(A.shape[1], G, G)
    ty = ty[:, None]
    tx = tx[None, :]
    return ((1.0 - ty) * (1.0 - tx) * V[:, ay[:, None], ax[None, :]]
            + (1.0 - ty) * tx * V[:, ay[:, None], ax[None, :] + 1]
            + ty * (1.0 - tx) * V[:, ay[:, None] + 1, ax[None, :]]
            + ty * tx * V[:, ay[:, None] + 1, ax[None, :] + 1])


def make_fields(H: int, W: int, d_over_r0: float, n_planes: int, seed: int, G: int = 64,
                corr_len: float = 2.0) -> np.ndarray:
    """Fields [n_planes][H][W] of the anchor model: plane i is Noll mode i + 2."""
    if G < 2:
        raise ValueError("the anchor grid needs G >= 2")
    A = anchor_coefficients(anchor_normals(G, n_planes, seed), G, d_over_r0, corr_len)
    return interpolate(A, G, H, W)
