"""Statistical validation of the simulator (paper Sec. 4.1), measured on
what the GPU path produces.

* Tilt statistics (Evaluation 1): many frames of fields from the field
  generator (FFT filtering, or the anchor grid); the mean products
  alpha(p) alpha(p + lag) of both tilt planes along rows and along columns,
  in units of the tilt variance V_2 (D/r0)^(5/3), and the variance of the
  tilt displacement in pixels^2.  Differential tilt D(lag) = 2 (c(0) - c(lag))
  follows from them.
* Exposure statistics (Evaluation 2): frames of a grid of point sources
  through the whole simulator; around every source a window of the output is
  one realisation of the spatially varying PSF with its tilt.  Long exposure:
  the MTF of the mean window, |mean OTF|; short exposure: the mean of the
  windows' own MTFs, mean |OTF| / |OTF(0)| (independent of where each
  realisation sits, so no re-centring is needed).

The frames run through the library's kernels; the statistics are reductions
of their outputs (PyTorch on the device for the lag products, NumPy for the
MTFs).  Run as a script on a GPU to print both as JSON.
"""
from __future__ import annotations

import json
import math
import sys

import numpy as np

from . import p2s


def tilt_statistics(H: int, W: int, d_over_r0: float, frames: int, lags, seed0: int = 100, anchors=None,
                    n_zernike: int = 35, q: float = 2.0, corr_len_px: float = 16.0):
    """Mean lag products of the two tilt planes over `frames` frames."""
    import torch
    lags = [int(l) for l in lags]
    F = torch.empty((n_zernike, H, W), dtype=torch.float32, device="cuda")
    if anchors is None:
        ws = torch.empty(p2s.fields_workspace_bytes(H, W, n_zernike, corr_len_px), dtype=torch.uint8, device="cuda")
    else:
        ws = torch.empty(anchors.fields_workspace_bytes(), dtype=torch.uint8, device="cuda")
    along_x = torch.zeros(len(lags), dtype=torch.float64, device="cuda")
    along_y = torch.zeros(len(lags), dtype=torch.float64, device="cuda")
    for f in range(frames):
        if anchors is None:
            p2s.make_fields(H, W, d_over_r0, n_zernike, seed0 + f, F, ws, corr_len_px)
        else:
            p2s.make_fields_anchor(anchors, H, W, d_over_r0, seed0 + f, F, ws)
        t = F[:2].double()
        for k, l in enumerate(lags):
            along_x[k] += (t[:, :, :W - l] * t[:, :, l:]).mean()
            along_y[k] += (t[:, :H - l, :] * t[:, l:, :]).mean()
    var = p2s.noll_variance(2) * d_over_r0 ** (5.0 / 3.0)
    ax = (along_x / frames / var).cpu().numpy()
    ay = (along_y / frames / var).cpu().numpy()
    shift = (2.0 * q / math.pi) ** 2 * var * float(0.5 * (ax[0] + ay[0]))
    return {"lags": lags, "cov_along_x": ax.tolist(), "cov_along_y": ay.tolist(),
            "shift_variance_px2": shift, "frames": frames, "H": H, "W": W}


def _radial(a: np.ndarray, q: float, u_points) -> np.ndarray:
    n = a.shape[0]
    k = np.fft.fftfreq(n) * n
    rad = np.rint(np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)).astype(np.int64)
    prof = np.bincount(rad.ravel(), weights=a.ravel()) / np.bincount(rad.ravel())
    return np.interp(np.asarray(u_points, dtype=np.float64) * n / q, np.arange(prof.size), prof)


def exposure_statistics(sim: "p2s.Simulator", d_over_r0: float, frames: int, u_points, precision: str = "bf16",
                        H: int = 512, W: int = 512, spacing: int = 64, window: int = 49, pad: int = 128,
                        seed0: int = 500, anchors=None, q: float = 2.0):
    """Long- and short-exposure MTFs of point sources through the simulator."""
    import torch
    R = window // 2
    ys = np.arange(spacing // 2, H - R, spacing)
    xs = np.arange(spacing // 2, W - R, spacing)
    img = torch.zeros((1, H, W), dtype=torch.float32, device="cuda")
    for y in ys:
        img[0, int(y), torch.from_numpy(xs).cuda()] = 1.0
    out = torch.empty_like(img)
    if anchors is not None:
        ws = torch.empty(anchors.workspace_bytes(1, H, W, sim.basis.K), dtype=torch.uint8, device="cuda")
    sum_patch = torch.zeros((window, window), dtype=torch.float64, device="cuda")
    sum_mag = torch.zeros((pad, pad), dtype=torch.float64, device="cuda")
    n = 0
    for f in range(frames):
        if anchors is None:
            sim(img, d_over_r0, seed0 + f, precision, out=out)
        else:
            p2s.simulate_anchor(img, d_over_r0, anchors, sim.basis, sim.net, seed0 + f, precision, out, ws,
                                sim.q_sampling)
        o = out[0].double()
        patches = torch.stack([o[int(y) - R:int(y) + R + 1, int(x) - R:int(x) + R + 1] for y in ys for x in xs])
        sum_patch += patches.sum(0)
        otf = torch.fft.fft2(patches, s=(pad, pad))
        sum_mag += (otf.abs() / otf[:, :1, :1].abs()).sum(0)
        n += patches.shape[0]
    mean_patch = (sum_patch / n).cpu().numpy()
    le_otf = np.abs(np.fft.fft2(mean_patch, s=(pad, pad)))
    le = _radial(le_otf / le_otf[0, 0], q, u_points)
    se = _radial((sum_mag / n).cpu().numpy(), q, u_points)
    return {"u": list(u_points), "long_exposure_mtf": le.tolist(), "short_exposure_mtf": se.tolist(),
            "realisations": n, "precision": precision}


def main():
    import torch
    import p2s_synth as S
    from . import anchors as panch
    from . import basis as pbasis
    from . import train as ptrain
    torch.cuda.set_device(0)
    wl = S.workload("single512")
    z, d = wl.basis_draws()
    basis, _ = pbasis.learn_basis(z, d, wl.K, wl.P, wl.n_zernike)
    Ws, bs, _ = ptrain.load("p2s_single512", basis)
    sim = p2s.Simulator(basis, Ws, bs, n_zernike=wl.n_zernike)
    model = panch.anchor_model(64, wl.n_zernike, 2.0)
    u = [0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8]
    lags = list(range(0, 65, 4))
    rep = {"d_over_r0": 3.0,
           "tilt_fft": tilt_statistics(512, 512, 3.0, 64, lags),
           "tilt_anchor": tilt_statistics(512, 512, 3.0, 64, lags, anchors=model),
           "exposure_fft": exposure_statistics(sim, 3.0, 128, u),
           "exposure_anchor": exposure_statistics(sim, 3.0, 128, u, anchors=model)}
    json.dump(rep, sys.stdout)
    print()


if __name__ == "__main__":
    main()
