"""Wavelength-dependent colour (paper Sec. 3.5): every colour channel is
blurred with the PSFs of its own wavelength, through its own PCA basis and
P2S network, instead of one PSF for all channels (about three times the
network and blur work of a grey frame).

The fields stay those of one reference wavelength (525 nm, D/r0 given there):
the optical path difference is the same at every wavelength, so at lambda the
phase is (525 / lambda) times the reference phase, and with a fixed pixel
pitch the sampling grows as q = 2 lambda / 525 pixels per lambda/D.  The tilt
displacement 2 q alpha / pi pixels is therefore the same for every channel
and one warp by the reference tilt serves all of them.  Channel c's basis is
learned (once, on the host) from PSFs formed that way, and its network maps
the reference alpha_4.. to that basis' coefficients; both are ordinary
handles, and p2s_simulate_spectral runs the frame.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from . import basis as pbasis
from . import p2s

REFERENCE_NM = 525.0
WAVELENGTHS_NM = (450.0, 540.0, 570.0)


def channel_sampling(wavelength_nm: float, q_ref: float = 2.0):
    """(q, phase_scale) of a wavelength: pixels per lambda/D, and the factor
    on the reference-wavelength phase."""
    return q_ref * wavelength_nm / REFERENCE_NM, REFERENCE_NM / wavelength_nm


def channel_basis(normals: np.ndarray, d_over_r0: np.ndarray, K: int, P: int, wavelength_nm: float,
                  n_zernike: int = 35):
    """PCA basis of the PSFs of one wavelength (Sec. 3.2 at that wavelength)."""
    q, s = channel_sampling(wavelength_nm)
    return pbasis.learn_basis(normals, d_over_r0, K, P, n_zernike, Q=q, phase_scale=s)


class SpectralSimulator:
    """Resident per-channel bases and networks + workspace for frames of one
    size (p2s_simulate_spectral)."""

    def __init__(self, bases: Sequence[np.ndarray], weights, biases, n_zernike: int = 35, corr_len_px: float = 16.0,
                 q_sampling: float = 2.0):
        if not (len(bases) == len(weights) == len(biases)):
            raise ValueError("one basis and one network per channel")
        self.bases = [p2s.Basis(b) for b in bases]
        self.nets = [p2s.Mlp(w, b) for w, b in zip(weights, biases)]
        self.n_zernike = n_zernike
        self.corr_len_px = corr_len_px
        self.q_sampling = q_sampling
        self._ws = None

    def workspace(self, C, H, W):
        import torch
        K = max(b.K for b in self.bases[:C])
        n = p2s.workspace_bytes(C, H, W, self.n_zernike, K, self.corr_len_px)
        if n == 0:
            raise p2s.P2SError(p2s.P2S_EINVAL, "invalid frame size")
        if self._ws is None or self._ws.numel() < n:
            self._ws = torch.empty(n, dtype=torch.uint8, device="cuda")
        return self._ws

    def __call__(self, image, d_over_r0, seed, precision="bf16", out=None, stream=None):
        import torch
        C, H, W = image.shape
        if out is None:
            out = torch.empty_like(image)
        p2s.simulate_spectral(image, d_over_r0, self.bases[:C], self.nets[:C], seed, precision, out,
                              self.workspace(C, H, W), self.n_zernike, self.corr_len_px, self.q_sampling, stream)
        return out
