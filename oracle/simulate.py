"""One frame of the P2S simulator end to end (Fig. 3; Sec. 2.2, 3.1, 3.3,
3.5): correlated Zernike fields -> P2S network on alpha_4.. at every pixel ->
basis blur of every colour channel with the same weights -> tilt warp of
every channel with alpha_2, alpha_3.

``weights="projection"`` replaces the network by the projection of each
pixel's exact PSF onto the basis (used to measure truncation error),
``exact_blur`` adds the per-pixel pupil-FFT blur of Eq. 3 (tiny frames only),
``blur_operands="fp8"`` feeds the basis blur E4M3-rounded image and basis
values (the FP8 precision variant; everything else unchanged), and
``field_model="anchor"`` draws the fields on a G x G anchor grid and
interpolates them (Sec. 3.4, ``anchors``) instead of FFT filtering.
"""
import numpy as np

from . import anchors, blur, fields, fp8, mlp, psf, warp


def _fields(H, W, d_over_r0, n_zernike, seed, corr_len, field_model, G, anchor_corr):
    if field_model == "fft":
        return fields.make_fields(H, W, d_over_r0, n_zernike, seed, corr_len)
    if field_model == "anchor":
        return anchors.make_fields(H, W, d_over_r0, n_zernike, seed, G, anchor_corr)
    raise ValueError(field_model)


def simulate(image: np.ndarray, d_over_r0: float, basis: np.ndarray, Ws=None, bs=None, seed: int = 0,
             n_zernike: int = 35, corr_len: float = 16.0, q: float = 2.0,
             weights: str = "mlp", exact: bool = False, Np: int = 32, blur_operands: str = "exact",
             field_model: str = "fft", G: int = 64, anchor_corr: float = 2.0):
    img = np.asarray(image, dtype=np.float64)
    if img.ndim == 2:
        img = img[None]
    C, H, W = img.shape
    K, P, _ = basis.shape
    F = _fields(H, W, d_over_r0, n_zernike, seed, corr_len, field_model, G, anchor_corr)
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


def simulate_pixels(image: np.ndarray, d_over_r0: float, basis: np.ndarray, Ws, bs, seed: int, pixels,
                    n_zernike: int = 35, corr_len: float = 16.0, q: float = 2.0, field_model: str = "fft",
                    G: int = 64, anchor_corr: float = 2.0) -> np.ndarray:
    """simulate()["out"] at chosen output pixels only, for frames too large
    to blur whole on the host.  The same steps, evaluated where they are
    needed: the fields in full; then for each output pixel (c, y, x) its tilt
    sample position (Sec. 2.2; clamped, bilinear as in ``warp``) and, at each
    of the four blurred pixels that sample reads, the network on that pixel's
    alpha_4.. (Sec. 3.3) dotted with the K convolutions there (Eq. 5: taps
    b_k[i][j] at offset (i - R, j - R), replicate border).  pixels: sequence
    of (c, y, x); returns float64 [len(pixels)].

    Parity: pinned against simulate() at every pixel of small frames."""
    img = np.asarray(image, dtype=np.float64)
    if img.ndim == 2:
        img = img[None]
    C, H, W = img.shape
    K, P, _ = basis.shape
    R = (P - 1) // 2
    B = np.asarray(basis, dtype=np.float64)
    F = _fields(H, W, d_over_r0, n_zernike, seed, corr_len, field_model, G, anchor_corr)
    dx = warp.displacement(F[0], q)
    dy = warp.displacement(F[1], q)
    offs = np.arange(P) - R
    blurred = {}

    def blurred_at(c, y, x):
        if (c, y, x) not in blurred:
            w = mlp.forward(Ws, bs, F[2:, y, x][None, :])[0]                   # [K]
            ys = np.clip(y - offs, 0, H - 1)                                   # I(y - (i - R))
            xs = np.clip(x - offs, 0, W - 1)
            patch = img[c][np.ix_(ys, xs)]                                     # patch[i][j]
            conv = np.tensordot(B, patch, axes=([1, 2], [0, 1]))               # b_k conv I at (y, x)
            blurred[(c, y, x)] = float(np.dot(w, conv))
        return blurred[(c, y, x)]

    out = np.empty(len(pixels), dtype=np.float64)
    for n, (c, y, x) in enumerate(pixels):
        sx = min(max(x + dx[y, x], 0.0), W - 1.0)
        sy = min(max(y + dy[y, x], 0.0), H - 1.0)
        x0, y0 = int(np.floor(sx)), int(np.floor(sy))
        x1, y1 = min(x0 + 1, W - 1), min(y0 + 1, H - 1)
        fx, fy = sx - x0, sy - y0
        top = (1.0 - fx) * blurred_at(c, y0, x0) + fx * blurred_at(c, y0, x1)
        bot = (1.0 - fx) * blurred_at(c, y1, x0) + fx * blurred_at(c, y1, x1)
        out[n] = (1.0 - fy) * top + fy * bot
    return out
