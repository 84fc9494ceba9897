"""PSF dataset and PCA basis (Sec. 3.2).

The paper draws Zernike vectors with covariance R_Z over weak to strong
turbulence, forms the tilt-free PSFs with Eq. 2 and keeps the top M principal
components as the basis phi_m of Eq. 4.

Readings recorded with the design notes: the PCA is uncentred (the
eigenvectors of the second-moment matrix (1/N) sum h h^T), because a mean term
would add a constant PSF outside the pure form of Eq. 5; each basis vector's
sign is fixed so that its taps sum to a non-negative value (if the sum is
zero to round-off, the largest-magnitude tap is made positive).  The standard
normals behind the draws are inputs, scaled here by the Noll standard
deviations.

Parity: pinned through the blur pins (completeness with K = U and
orthonormality); the dataset itself is Eq. 2, pinned in ``psf``.
"""
import numpy as np

from .noll import noll_variance
from .psf import psf_from_zernike


def dataset(normals: np.ndarray, d_over_r0: np.ndarray, modes=range(4, 37),
            Np: int = 32, Q: float = 2, P: int = 33, chunk: int = 1024, phase_scale: float = 1.0) -> np.ndarray:
    """PSFs [n][P][P] for alpha_j = normals[:, i] * sqrt(V_j (D/r0)^(5/3)),
    sampled at Q pixels per lambda/D, phase scaled by phase_scale."""
    modes = list(modes)
    var = np.array([noll_variance(j) for j in modes])
    sig = np.sqrt(var[None, :] * np.asarray(d_over_r0, dtype=np.float64)[:, None] ** (5.0 / 3.0))
    alpha = np.asarray(normals, dtype=np.float64) * sig
    out = []
    for s in range(0, alpha.shape[0], chunk):
        out.append(psf_from_zernike(alpha[s:s + chunk], modes, Np, Q, P, phase_scale))
    return np.concatenate(out, axis=0)


def fix_sign(v: np.ndarray) -> np.ndarray:
    s = v.sum()
    if abs(s) > 1e-12 * np.abs(v).max():
        return v if s > 0 else -v
    return v if v[np.argmax(np.abs(v))] > 0 else -v


def pca_basis(psfs: np.ndarray, K: int):
    """Top-K eigenvectors of the uncentred second-moment matrix.
    Returns (basis [K][P][P], eigenvalues [K])."""
    n, P, _ = psfs.shape
    X = psfs.reshape(n, P * P)
    S = X.T @ X / n
    evals, evecs = np.linalg.eigh(S)
    order = np.argsort(evals)[::-1][:K]
    B = np.stack([fix_sign(evecs[:, i]) for i in order])
    return B.reshape(K, P, P), evals[order]
