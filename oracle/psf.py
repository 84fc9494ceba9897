"""PSF formation from the pupil phase (Sec. 2.2, Eq. 2):

    h = | F{ W(rho) exp(-j phi(rho)) } |^2,   phi = sum_j alpha_j Z_j.

Sampling reading (the paper leaves it to its supplement): the pupil of
diameter D is sampled on Np x Np cell-centred points, zero-padded to
Nfft = Q*Np (Q = 2 is Nyquist sampling of the diffraction-limited PSF), the
power spectrum is centred with fftshift, cropped to P x P around DC and
normalised to unit sum.  Tilts (Noll 2, 3) are left out, which centres the
PSF (Sec. 3.2).

Parity: pinned (Parseval and the zero-phase peak exactly; zero phase against
the Airy pattern with the error shrinking as Np grows).
"""
import numpy as np

from .zernike import zernike


def pupil_grid(Np: int):
    """(rho, theta, mask) on Np x Np cell-centred samples of the unit disk;
    rows are y, columns are x."""
    c = (2.0 * np.arange(Np) + 1.0 - Np) / Np
    y, x = np.meshgrid(c, c, indexing="ij")
    rho = np.hypot(x, y)
    theta = np.arctan2(y, x)
    return rho, theta, (rho <= 1.0).astype(np.float64)


def zernike_stack(modes, Np: int) -> np.ndarray:
    """Z_j sampled on the pupil grid for each Noll index in ``modes``."""
    rho, theta, _ = pupil_grid(Np)
    return np.stack([zernike(j, rho, theta) for j in modes])


def psf_from_phase(phase: np.ndarray, mask: np.ndarray, Q: int, P: int, normalise: bool = True) -> np.ndarray:
    """Eq. 2 for one or more pupil phases [..., Np, Np] -> PSFs [..., P, P]."""
    Np = mask.shape[-1]
    nfft = Q * Np
    field = mask * np.exp(-1j * phase)
    pad = np.zeros(phase.shape[:-2] + (nfft, nfft), dtype=np.complex128)
    pad[..., :Np, :Np] = field
    h = np.abs(np.fft.fft2(pad)) ** 2
    h = np.fft.fftshift(h, axes=(-2, -1))
    R = (P - 1) // 2
    c = nfft // 2
    h = h[..., c - R:c + R + 1, c - R:c + R + 1]
    if normalise:
        h = h / h.sum(axis=(-2, -1), keepdims=True)
    return h


def psf_from_phase_q(phase: np.ndarray, mask: np.ndarray, q: float, P: int, normalise: bool = True) -> np.ndarray:
    """Eq. 2 sampled at q pixels per lambda/D for any real q > 0: the field
    at pixel offset (v, u), |u|, |v| <= R, is the discrete Fourier sum
    sum_{y,x} W e^{-j phi} exp(-2 pi i (u x + v y) / (q Np)) over the pupil
    samples (for integer q these are the bins of the zero-padded FFT)."""
    Np = mask.shape[-1]
    R = (P - 1) // 2
    u = np.arange(-R, R + 1, dtype=np.float64)
    x = np.arange(Np, dtype=np.float64)
    A = np.exp(-2j * np.pi * np.outer(u, x) / (q * Np))          # [P][Np]
    field = mask * np.exp(-1j * phase)
    E = A @ field @ A.T                                           # rows v, columns u
    h = np.abs(E) ** 2
    if normalise:
        h = h / h.sum(axis=(-2, -1), keepdims=True)
    return h


def psf_from_zernike(alpha: np.ndarray, modes, Np: int = 32, Q: float = 2, P: int = 33,
                     phase_scale: float = 1.0) -> np.ndarray:
    """PSFs for Zernike coefficient vectors alpha [..., len(modes)]; the phase
    is phase_scale * sum alpha_j Z_j (a wavelength other than the one alpha
    is given at: phase_scale = lambda_ref / lambda); non-integer sampling Q
    goes through psf_from_phase_q."""
    Z = zernike_stack(modes, Np)
    _, _, mask = pupil_grid(Np)
    phase = phase_scale * np.tensordot(np.asarray(alpha, dtype=np.float64), Z, axes=([-1], [0]))
    if float(Q) == int(Q):
        return psf_from_phase(phase, mask, int(Q), P)
    return psf_from_phase_q(phase, mask, float(Q), P)
