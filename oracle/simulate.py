"""One frame of the P2S simulator end to end (Fig. 3; Sec. 2.2, 3.1, 3.3,
3.5): correlated Zernike fields -> P2S network on alpha_4.. at every pixel ->
basis blur of every colour channel with the same weights -> tilt warp of
every channel with alpha_2, alpha_3.

``weights="projection"`` replaces the network by the projection of each
pixel's exact PSF onto the basis (used to measure truncation error),
``exact_blur`` adds the per-pixel pupil-FFT blur of Eq. 3 (tiny frames only),
and ``blur_operands="fp8"`` feeds the basis blur E4M3-rounded image and basis
values (the FP8 precision variant; everything else unchanged).
"""
import numpy as np

from . import blur, fields, fp8, mlp, psf, warp


def simulate(image: np.ndarray, d_over_r0: float, basis: np.ndarray, Ws=None, bs=None, seed: int = 0,
             n_zernike: int = 35, corr_len: float = 16.0, q: float = 2.0,
             weights: str = "mlp", exact: bool = False, Np: int = 32, blur_operands: str = "exact"):
    img = np.asarray(image, dtype=np.float64)
    if img.ndim == 2:
        img = img[None]
    C, H, W = img.shape
    K, P, _ = basis.shape
    F = fields.make_fields(H, W, d_over_r0, n_zernike, seed, corr_len)
    alpha_hi = np.moveaxis(F[2:], 0, -1).reshape(H * W, n_zernike - 2)      # [pix][j=4..]
    res = {"fields": F}
    psfs = None
    if weights == "projection" or exact:
        psfs = psf.psf_from_zernike(alpha_hi, range(4, n_zernike + 2), Np, int(q), P).reshape(H, W, P, P)
    if weights == "mlp":
        w = mlp.forward(Ws, bs, alpha_hi)
    elif weights == "projection":
        w = blur.projection_weights(psfs, basis).reshape(H * W, K)
    else:
        raise ValueError(weights)
    res["w"] = w
    if blur_operands == "exact":
        bl = np.stack([blur.basis_blur(img[c], basis, w.reshape(H, W, K)) for c in range(C)])
    elif blur_operands == "fp8":
        bl = np.stack([fp8.fp8_blur(img[c], basis, w.reshape(H, W, K)) for c in range(C)])
    else:
        raise ValueError(blur_operands)
    res["blurred"] = bl
    res["out"] = np.stack([warp.tilt_warp(bl[c], F[0], F[1], q) for c in range(C)])
    if exact:
        ex = np.stack([blur.exact_blur(img[c], psfs) for c in range(C)])
        res["exact_blurred"] = ex
        res["exact_out"] = np.stack([warp.tilt_warp(ex[c], F[0], F[1], q) for c in range(C)])
    return res
