"""Wavelength-dependent colour (Sec. 3.5): each colour channel blurred with
the PSFs of its own wavelength (the paper's three: 450, 540 and 570 nm),
through its own basis and network, instead of one PSF for all channels.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module.

Readings (each recorded with the design notes):

* the fields alpha are given in radians of phase at a reference wavelength,
  525 nm (the paper's single-PSF colour image uses 525 nm), with D/r0 at that
  wavelength; the optical path difference is achromatic, so at wavelength
  lambda the phase is (lambda_ref / lambda) sum alpha_j Z_j;
* the pixel pitch is fixed, so the sampling q, pixels per lambda/D, grows
  with lambda: q_c = q_ref lambda_c / lambda_ref (q_ref = 2);
* the tilt displacement s alpha, s = 2 q / pi pixels per radian, is then the
  same at every wavelength (q_c alpha_c = q_ref alpha_ref): one warp by the
  reference tilt serves all channels;
* channel c's basis is the PCA basis of PSFs formed that way, and its network
  maps the reference alpha_4.. to that basis' coefficients.

Parity: pinned (achromatic tilt displacement for every channel; with one
basis and network for all channels the frame equals the grey simulator's).
"""
import numpy as np

from . import blur, fields, mlp, warp

REFERENCE_NM = 525.0
WAVELENGTHS_NM = (450.0, 540.0, 570.0)


def channel_sampling(wavelength_nm: float, q_ref: float = 2.0):
    """(q, phase_scale) of a channel: pixels per lambda/D and the factor on
    the reference-wavelength phase."""
    return q_ref * wavelength_nm / REFERENCE_NM, REFERENCE_NM / wavelength_nm


def simulate_spectral(image: np.ndarray, d_over_r0: float, bases, Ws, bs, seed: int = 0, n_zernike: int = 35,
                      corr_len: float = 16.0, q: float = 2.0) -> np.ndarray:
    """One frame: shared fields (reference wavelength), channel c blurred by
    the basis bases[c] with the weights of network (Ws[c], bs[c]) at every
    pixel, every channel warped by the reference tilt.  Returns [C][H][W]."""
    img = np.asarray(image, dtype=np.float64)
    C, H, W = img.shape
    if not (len(bases) == len(Ws) == len(bs) == C):
        raise ValueError("one basis and one network per channel")
    F = fields.make_fields(H, W, d_over_r0, n_zernike, seed, corr_len)
    alpha_hi = np.moveaxis(F[2:], 0, -1).reshape(H * W, n_zernike - 2)
    out = np.empty_like(img)
    for c in range(C):
        K = bases[c].shape[0]
        w = mlp.forward(Ws[c], bs[c], alpha_hi).reshape(H, W, K)
        bl = blur.basis_blur(img[c], bases[c], w)
        out[c] = warp.tilt_warp(bl, F[0], F[1], q)
    return out


def simulate_spectral_pixels(image: np.ndarray, d_over_r0: float, bases, Ws, bs, seed: int, pixels,
                             n_zernike: int = 35, corr_len: float = 16.0, q: float = 2.0) -> np.ndarray:
    """simulate_spectral()[c, y, x] at chosen pixels only: channels are
    independent given the shared fields, so each pixel is the grey
    simulator's pixel of its channel plane with that channel's basis and
    network.  pixels: sequence of (c, y, x); returns float64 [len(pixels)]."""
    from .simulate import simulate_pixels
    img = np.asarray(image, dtype=np.float64)
    out = np.empty(len(pixels))
    for c in range(img.shape[0]):
        sel = [k for k, p in enumerate(pixels) if p[0] == c]
        if sel:
            out[sel] = simulate_pixels(img[c:c + 1], d_over_r0, bases[c], Ws[c], bs[c], seed,
                                       [(0, pixels[k][1], pixels[k][2]) for k in sel], n_zernike, corr_len, q)
    return out
