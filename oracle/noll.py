"""Diagonal of Noll's Zernike covariance R_Z (Sec. 2.2: alpha ~ N(0, R_Z),
with R_Z from Noll 1976).

Variance of a mode of radial order n >= 1, in units of (D/r0)^(5/3):

    V_n = K (n+1) Gamma(n - 5/6) / (Gamma(17/6)^2 Gamma(n + 23/6)).

Reading recorded with the design notes: the often-quoted constant
K = Gamma(14/3) [(24/5) Gamma(6/5)]^(5/6) Gamma(11/6)^2 / (2 pi^2) = 2.2698
makes the modal variances sum to 1.0433 over j >= 2, 1.29 % more than the
piston-removed phase variance 1.0299 of Noll's Table IV, and exceeds every
radial order of that table by the same factor.  K is therefore fixed so that
sum_{j>=2} V_j = 1.0299, which reproduces the table at every order within its
rounding.  Only the diagonal is used (modes drawn independently); the cross
terms of R_Z are dropped.

Parity: pinned against Noll's tabulated residual differences for every radial
order and against his asymptotic residual law.
"""
from math import exp, lgamma, gamma, pi

from .zernike import noll_to_nm

K_QUOTED = gamma(14.0 / 3.0) * ((24.0 / 5.0) * gamma(6.0 / 5.0)) ** (5.0 / 6.0) * gamma(11.0 / 6.0) ** 2 / (2.0 * pi ** 2)
PISTON_REMOVED_VARIANCE = 1.0299


def _shape(n: int) -> float:
    """(n+1) Gamma(n-5/6) / (Gamma(17/6)^2 Gamma(n+23/6))."""
    return (n + 1) * exp(lgamma(n - 5.0 / 6.0) - 2.0 * lgamma(17.0 / 6.0) - lgamma(n + 23.0 / 6.0))


def _mode_sum(n_max: int = 200000) -> float:
    """sum over j >= 2 of the shape: radial order n holds n+1 modes."""
    return sum((n + 1) * _shape(n) for n in range(1, n_max))


KC = PISTON_REMOVED_VARIANCE / _mode_sum()


def noll_variance_n(n: int) -> float:
    """Variance of one Zernike mode of radial order n >= 1, per (D/r0)^(5/3)."""
    if n < 1:
        raise ValueError("piston (n=0) has no finite variance")
    return KC * _shape(n)


def noll_variance(j: int) -> float:
    """Variance of Noll mode j >= 2, per (D/r0)^(5/3)."""
    n, _ = noll_to_nm(j)
    return noll_variance_n(n)


def mode_sigma(j: int, d_over_r0: float) -> float:
    """Standard deviation of alpha_j at turbulence strength D/r0."""
    return (noll_variance(j) * d_over_r0 ** (5.0 / 3.0)) ** 0.5
