"""Set-up of the anchor-grid field model (paper Sec. 3.4 with the mode
covariance R_Z of Sec. 2.2): the two covariance matrices and their lower
Cholesky factors, computed once on the host and handed to the library
(p2s_anchor_create), which then draws and interpolates the fields of every
frame on the GPU.

* R_Z: Noll's modal covariance of Kolmogorov phase, cross terms included.
  Modes covary only with equal azimuthal frequency m and, for m > 0, equal
  cos/sin parity; the entry is
      K (-1)^((n+n'-2m)/2) sqrt((n+1)(n'+1)) G((n+n'-5/3)/2)
        / [G((n-n'+17/3)/2) G((n'-n+17/3)/2) G((n+n'+23/3)/2)]
  with G the Gamma function.  K comes from the library's Noll variances
  (its diagonal), so the two agree by construction.
* anchor correlation: rho(d) = exp(-(d / corr_len)^(5/3)) with d the distance
  in anchor spacings -- a stand-in for the angle-of-arrival covariance the
  paper takes from the literature without printing it: positive definite in
  the plane and locally of Kolmogorov's 5/3 form.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np

from . import p2s


def _noll_nm(j: int):
    """(n, m) of Noll index j: n the radial order, m >= 0."""
    n = int(math.ceil((math.sqrt(8 * j + 1) - 3) / 2))
    while (n + 1) * (n + 2) // 2 < j:
        n += 1
    while n * (n + 1) // 2 >= j:
        n -= 1
    first = n * (n + 1) // 2 + 1           # first Noll index of order n
    pos = j - first                        # 0 .. n
    m = (n % 2) + 2 * ((pos + (1 - n % 2)) // 2)
    return n, m


def mode_covariance(n_planes: int) -> np.ndarray:
    """R_Z per (D/r0)^(5/3) over planes i = Noll mode i + 2."""
    nm = [_noll_nm(i + 2) for i in range(n_planes)]
    var = np.array([p2s.noll_variance(i + 2) for i in range(n_planes)])

    def shape(n, nn):
        return (math.sqrt((n + 1) * (nn + 1)) * math.gamma((n + nn - 5.0 / 3.0) / 2.0)
                / (math.gamma((n - nn + 17.0 / 3.0) / 2.0) * math.gamma((nn - n + 17.0 / 3.0) / 2.0)
                   * math.gamma((n + nn + 23.0 / 3.0) / 2.0)))

    R = np.zeros((n_planes, n_planes))
    for a in range(n_planes):
        n, m = nm[a]
        for b in range(n_planes):
            nn, mm = nm[b]
            if m != mm or (m > 0 and (a - b) % 2):
                continue
            sign = 1.0 if ((n + nn) // 2 - m) % 2 == 0 else -1.0
            R[a, b] = sign * shape(n, nn) / math.sqrt(shape(n, n) * shape(nn, nn))
    return R * np.sqrt(np.outer(var, var))


def anchor_correlation(G: int, corr_len: float = 2.0) -> np.ndarray:
    """R_s [G^2][G^2] over anchors p = a G + b."""
    idx = np.arange(G * G)
    ya, xa = (idx // G).astype(np.float64), (idx % G).astype(np.float64)
    d2 = (ya[:, None] - ya[None, :]) ** 2 + (xa[:, None] - xa[None, :]) ** 2
    return np.exp(-np.power(np.sqrt(d2) / corr_len, 5.0 / 3.0))


@lru_cache(maxsize=4)
def _factors(G: int, n_planes: int, corr_len: float):
    Ls = np.linalg.cholesky(anchor_correlation(G, corr_len))
    Lz = np.linalg.cholesky(mode_covariance(n_planes))
    return Ls, Lz


def anchor_model(G: int = 64, n_zernike: int = 35, corr_len: float = 2.0) -> "p2s.Anchors":
    """Device handle of the stand-in model on a G x G anchor grid (the
    factorisation of the G^2 x G^2 matrix takes about a second for G = 64
    and is cached per process)."""
    Ls, Lz = _factors(int(G), int(n_zernike), float(corr_len))
    return p2s.Anchors(G, Ls, Lz)
