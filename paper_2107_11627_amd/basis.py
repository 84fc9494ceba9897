"""One-time basis learning on the host (Sec. 3.2), FP64.

Draw tilt-free Zernike vectors alpha_4.. with the Noll variances (scaled by
(D/r0)^(5/3)) from the library, form each PSF with Eq. 2 on a sampled pupil,
and keep the top K right singular vectors of the PSF data matrix (the
uncentred principal components).  This runs once per configuration, before
any frame, and its result is uploaded with p2s_basis_create; it is not part
of the per-frame path.

Sampling: the pupil of diameter D is Np x Np cell-centred samples, zero-padded
to Q*Np (Q = 2: Nyquist), power spectrum centred and cropped to P x P around
DC, normalised to unit sum.  Sign of each component: taps sum >= 0 (else the
largest-magnitude tap positive).
"""
from __future__ import annotations

import numpy as np
from scipy.special import eval_jacobi

from . import p2s


def noll_nm(j: int):
    n = int(np.ceil((-3.0 + np.sqrt(9.0 + 8.0 * (j - 1))) / 2.0))
    first = n * (n + 1) // 2 + 1                # first Noll index of order n
    k = j - first
    m = (n % 2) + 2 * ((k + (1 - n % 2)) // 2)
    return n, m


def zernike_on_pupil(j: int, Np: int) -> np.ndarray:
    """Noll-normalised Z_j on the cell-centred Np x Np pupil samples.
    Radial part via the Jacobi form R_n^m(r) = (-1)^s r^m P_s^(m,0)(1 - 2 r^2),
    s = (n - m)/2."""
    n, m = noll_nm(j)
    c = (np.arange(Np) + 0.5) * (2.0 / Np) - 1.0
    X, Y = np.meshgrid(c, c)                    # X along columns, Y along rows
    r = np.sqrt(X * X + Y * Y)
    th = np.arctan2(Y, X)
    s = (n - m) // 2
    rad = (-1.0) ** s * r ** m * eval_jacobi(s, m, 0, 1.0 - 2.0 * r * r)
    if m == 0:
        return np.sqrt(n + 1.0) * rad
    ang = np.cos(m * th) if j % 2 == 0 else np.sin(m * th)
    return np.sqrt(2.0 * (n + 1.0)) * rad * ang


def psf_dataset(normals: np.ndarray, d_over_r0: np.ndarray, P: int, n_zernike: int = 35,
                Np: int = 32, Q: float = 2, chunk: int = 512, phase_scale: float = 1.0) -> np.ndarray:
    """PSFs [n][P][P] of alpha_4.. = normals * sqrt(V_j (D/r0)^(5/3)), the phase
    multiplied by phase_scale (lambda_ref / lambda for another wavelength),
    sampled at Q pixels per lambda/D: by a zero-padded FFT for integer Q,
    else by the Fourier sum at the P x P output offsets directly."""
    modes = np.arange(4, n_zernike + 2)
    sig = np.sqrt(np.array([p2s.noll_variance(int(j)) for j in modes]))
    Zs = np.stack([zernike_on_pupil(int(j), Np) for j in modes]).reshape(len(modes), -1)
    c = (np.arange(Np) + 0.5) * (2.0 / Np) - 1.0
    pupil = (c[None, :] ** 2 + c[:, None] ** 2 <= 1.0).astype(np.float64)
    R = (P - 1) // 2
    integer_q = float(Q) == int(Q)
    if integer_q:
        nf = int(Q) * Np
    else:
        # F[u][x] = exp(-2 pi i u x / (Q Np)), u = -R..R output offsets
        F = np.exp(-2j * np.pi * np.outer(np.arange(-R, R + 1), np.arange(Np)) / (float(Q) * Np))
    out = np.empty((normals.shape[0], P, P))
    d53 = np.asarray(d_over_r0, dtype=np.float64) ** (5.0 / 6.0)   # sqrt of (D/r0)^(5/3)
    for s0 in range(0, normals.shape[0], chunk):
        a = normals[s0:s0 + chunk] * sig[None, :] * d53[s0:s0 + chunk, None]
        phase = phase_scale * (a @ Zs).reshape(-1, Np, Np)
        if integer_q:
            field = np.zeros((phase.shape[0], nf, nf), dtype=np.complex128)
            field[:, :Np, :Np] = pupil * np.exp(-1j * phase)
            spec = np.fft.fft2(field)
            h = np.roll(np.abs(spec) ** 2, (nf // 2, nf // 2), axis=(1, 2))[:, nf // 2 - R:nf // 2 + R + 1,
                                                                             nf // 2 - R:nf // 2 + R + 1]
        else:
            h = np.abs(F @ (pupil * np.exp(-1j * phase)) @ F.T) ** 2
        out[s0:s0 + chunk] = h / h.sum(axis=(1, 2), keepdims=True)
    return out


def pca(psfs: np.ndarray, K: int):
    """Top-K uncentred principal components (right singular vectors of the
    data matrix / sqrt(N)).  Returns (basis [K][P][P], eigenvalues [K])."""
    n, P, _ = psfs.shape
    X = psfs.reshape(n, P * P) / np.sqrt(n)
    _, sv, Vt = np.linalg.svd(X, full_matrices=False)
    B = Vt[:K].copy()
    for k in range(K):
        s = B[k].sum()
        if abs(s) > 1e-12 * np.abs(B[k]).max():
            if s < 0:
                B[k] = -B[k]
        elif B[k][np.argmax(np.abs(B[k]))] < 0:
            B[k] = -B[k]
    return B.reshape(K, P, P), sv[:K] ** 2


def learn_basis(normals: np.ndarray, d_over_r0: np.ndarray, K: int, P: int, n_zernike: int = 35,
                Q: float = 2, phase_scale: float = 1.0):
    return pca(psf_dataset(normals, d_over_r0, P, n_zernike, Q=Q, phase_scale=phase_scale), K)
