"""Zernike polynomials in Noll's ordering and normalisation (Sec. 2.2, Eq. 1).

The phase over the aperture is expanded as phi(rho) = sum_j alpha_j Z_j(rho).
Noll ordering: j -> (n, m), with even j carrying cos(m theta) and odd j
sin(m theta) for m > 0; normalisation (1/pi) int_disk Z_j^2 = 1.

Parity: pinned (orthonormality by exact quadrature, explicit low-order forms).
"""
from math import factorial

import numpy as np


def noll_to_nm(j: int):
    """Radial order n and azimuthal frequency m (>= 0) of Noll index j >= 1."""
    if j < 1:
        raise ValueError("Noll index starts at 1")
    n = 0
    while (n + 1) * (n + 2) // 2 < j:
        n += 1
    k = j - n * (n + 1) // 2 - 1          # position inside radial order n
    if n % 2 == 0:
        m = 2 * ((k + 1) // 2)
    else:
        m = 2 * (k // 2) + 1
    return n, m


def radial(n: int, m: int, rho: np.ndarray) -> np.ndarray:
    """R_n^m(rho) by its finite factorial sum."""
    out = np.zeros_like(rho, dtype=np.float64)
    for s in range((n - m) // 2 + 1):
        c = ((-1) ** s * factorial(n - s)
             / (factorial(s) * factorial((n + m) // 2 - s) * factorial((n - m) // 2 - s)))
        out += c * rho ** (n - 2 * s)
    return out


def zernike(j: int, rho: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """Noll-normalised Z_j on polar coordinates (not masked to the disk)."""
    n, m = noll_to_nm(j)
    r = radial(n, m, np.asarray(rho, dtype=np.float64))
    if m == 0:
        return np.sqrt(n + 1.0) * r
    if j % 2 == 0:
        return np.sqrt(2.0 * (n + 1)) * r * np.cos(m * theta)
    return np.sqrt(2.0 * (n + 1)) * r * np.sin(m * theta)
