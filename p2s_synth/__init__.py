"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module holds no arithmetic of the simulation method itself: it only draws
random inputs (images, network weights, the standard normals behind the PSF
dataset, per-frame D/r0 and sizes) from NumPy's PCG64 generator and describes
the six workloads by their sizes and seeds.  Both sides receive exactly the
same arrays from here; neither side's arithmetic lives here.

Workloads (sizes follow the paper's 256x256 timing frame and its M=100 basis,
Table 2 and Sec. 3.2; the remaining sizes are the synthetic stand-ins described
in the design notes):

* ``single128``  128x128 C=1, D/r0=1.5, K=16 basis of 17x17, MLP 33-64-64-16.
* ``single512``  512x512 C=1, D/r0=3, K=100 basis of 33x33, MLP 33-100-100-100.
* ``batch256``   64 frames 256x256 RGB, D/r0 ~ U[1,4].
* ``ragged``     200 frames, sizes from a fixed set, C in {1,3}, D/r0 ~ U[0.5,5].
* ``serving``    1000 requests, sizes 128..2048 (multiples of 64), RGB,
                 admission budget 32 GiB; Poisson arrivals at 70 % of the
                 saturated request rate measured in the same run.
* ``spectral512`` 512x512 RGB, D/r0=3, one K=100 basis of 33x33 and one
                 MLP 33-100-100-100 per channel, channels at 450, 540 and
                 570 nm (reference wavelength 525 nm).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

__all__ = [
    "bf16_representable",
    "blob_params",
    "blob_image",
    "blob_image_device",
    "xavier_mlp",
    "standard_normals",
    "FrameSpec",
    "Workload",
    "workload",
    "WORKLOADS",
]


def bf16_representable(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 value (ties to even) and
    return them as float32.  Used so that one set of network weights is exact
    in FP64, FP32 and BF16 alike."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).reshape(a.shape)


def blob_params(H: int, W: int, C: int, seed: int, n_blobs: int = 20,
                sigma_range: Tuple[float, float] = (3.0, 12.0),
                amp_range: Tuple[float, float] = (0.2, 1.0)):
    """The random draws behind ``blob_image``: per channel the blob centres
    (cy, cx), widths and amplitudes, then the generator positioned for the
    optional noise."""
    rng = np.random.default_rng(seed)
    per_channel = []
    for _ in range(C):
        cy = rng.uniform(0.0, H, n_blobs)
        cx = rng.uniform(0.0, W, n_blobs)
        sg = rng.uniform(sigma_range[0], sigma_range[1], n_blobs)
        am = rng.uniform(amp_range[0], amp_range[1], n_blobs)
        per_channel.append((cy, cx, sg, am))
    return per_channel, rng


def blob_image(H: int, W: int, C: int, seed: int, n_blobs: int = 20,
               sigma_range: Tuple[float, float] = (3.0, 12.0),
               amp_range: Tuple[float, float] = (0.2, 1.0),
               noise_std: float = 0.0) -> np.ndarray:
    """Sum of ``n_blobs`` isotropic Gaussian blobs per channel, min-max
    normalised to [0, 1] per channel, plus optional zero-mean uniform noise of
    standard deviation ``noise_std`` (not clipped).  Returns float32 [C][H][W]."""
    chans, rng = blob_params(H, W, C, seed, n_blobs, sigma_range, amp_range)
    yy = np.arange(H, dtype=np.float64)[:, None]
    xx = np.arange(W, dtype=np.float64)[None, :]
    out = np.empty((C, H, W), dtype=np.float64)
    for c, (cy, cx, sg, am) in enumerate(chans):
        img = np.zeros((H, W), dtype=np.float64)
        for b in range(len(cy)):   # separable: exp(-(dy^2 + dx^2)/2s^2) = g(dy) g(dx)
            s2 = 2.0 * sg[b] ** 2
            img += (am[b] * np.exp(-(yy - cy[b]) ** 2 / s2)) * np.exp(-(xx - cx[b]) ** 2 / s2)
        lo, hi = img.min(), img.max()
        out[c] = (img - lo) / (hi - lo) if hi > lo else np.zeros_like(img)
    if noise_std > 0.0:
        a = noise_std * np.sqrt(3.0)
        out += rng.uniform(-a, a, size=out.shape)
    return out.astype(np.float32)


def blob_image_device(H: int, W: int, C: int, seed: int, noise_std: float = 0.0, device="cuda",
                      device_noise: bool = False):
    """The same image as ``blob_image`` (same draws; the sums evaluated in
    float64 by torch on ``device``, so equal up to rounding), for workloads too
    large to build on the host.  The noise is drawn on the host as in
    ``blob_image``, or with ``device_noise`` from torch's generator on the
    device seeded with ``seed`` (a different but equally distributed draw)."""
    import torch
    chans, rng = blob_params(H, W, C, seed)
    yy = torch.arange(H, dtype=torch.float64, device=device)[:, None]
    xx = torch.arange(W, dtype=torch.float64, device=device)[None, :]
    out = torch.empty((C, H, W), dtype=torch.float64, device=device)
    for c, (cy, cx, sg, am) in enumerate(chans):
        s2 = torch.from_numpy(2.0 * sg ** 2).to(device)
        gy = torch.from_numpy(am).to(device)[:, None] * torch.exp(
            -(yy.T - torch.from_numpy(cy).to(device)[:, None]) ** 2 / s2[:, None])          # [n][H]
        gx = torch.exp(-(xx - torch.from_numpy(cx).to(device)[:, None]) ** 2 / s2[:, None])  # [n][W]
        img = gy.T @ gx
        lo, hi = img.min(), img.max()
        out[c] = (img - lo) / (hi - lo) if bool(hi > lo) else torch.zeros_like(img)
    if noise_std > 0.0:
        a = noise_std * np.sqrt(3.0)
        if device_noise:
            g = torch.Generator(device=device)
            g.manual_seed(int(seed))
            out += (torch.rand((C, H, W), generator=g, dtype=torch.float64, device=device) * 2.0 - 1.0) * a
        else:
            out += torch.from_numpy(rng.uniform(-a, a, size=(C, H, W))).to(device)
    return out.to(torch.float32)


def xavier_mlp(dims: Sequence[int], seed: int, bias_scale: float = 0.0):
    """Glorot/Xavier-uniform weights W_l [dims[l+1]][dims[l]], drawn from
    U(-a, a) with a = sqrt(6/(fan_in+fan_out)), rounded once to
    bfloat16-representable values.  Biases are zero unless ``bias_scale`` > 0,
    in which case they are U(-bias_scale, bias_scale), also bf16-representable.
    Returns (weights, biases) as lists of float32 arrays."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for l in range(len(dims) - 1):
        fi, fo = int(dims[l]), int(dims[l + 1])
        a = np.sqrt(6.0 / (fi + fo))
        Ws.append(bf16_representable(rng.uniform(-a, a, size=(fo, fi)).astype(np.float32)))
        if bias_scale > 0.0:
            bs.append(bf16_representable(rng.uniform(-bias_scale, bias_scale, size=fo).astype(np.float32)))
        else:
            bs.append(np.zeros(fo, dtype=np.float32))
    return Ws, bs


def standard_normals(shape, seed: int) -> np.ndarray:
    """i.i.d. N(0,1) float64 draws, e.g. the Zernike draws behind a PSF dataset."""
    return np.random.default_rng(seed).standard_normal(shape)


@dataclass
class FrameSpec:
    H: int
    W: int
    C: int
    d_over_r0: float
    image_seed: int
    field_seed: int
    noise_std: float = 0.0

    def image(self) -> np.ndarray:
        return blob_image(self.H, self.W, self.C, self.image_seed, noise_std=self.noise_std)


@dataclass
class Workload:
    name: str
    frames: List[FrameSpec]
    K: int
    P: int
    n_psf: int
    basis_seed: int
    basis_d_over_r0: Tuple[float, float]   # (lo, hi); lo == hi means one value
    mlp_dims: Tuple[int, ...]
    model_seed: int
    n_zernike: int = 35
    corr_len_px: float = 16.0
    q_sampling: float = 2.0
    extra: dict = field(default_factory=dict)

    def mlp(self, bias_scale: float = 0.0):
        return xavier_mlp(self.mlp_dims, self.model_seed, bias_scale)

    def basis_draws(self):
        """(normals [n_psf][n_zernike-2], d_over_r0 [n_psf]) for the PSF dataset."""
        z = standard_normals((self.n_psf, self.n_zernike - 2), self.basis_seed)
        lo, hi = self.basis_d_over_r0
        if lo == hi:
            d = np.full(self.n_psf, lo)
        else:
            d = np.random.default_rng(self.basis_seed + 1).uniform(lo, hi, self.n_psf)
        return z, d


_RAGGED_SIZES = [(128, 128), (256, 192), (384, 384), (512, 320), (768, 768)]


def workload(name: str) -> Workload:
    if name == "single128":
        return Workload(name, [FrameSpec(128, 128, 1, 1.5, 0, 1)], K=16, P=17, n_psf=2048,
                        basis_seed=3, basis_d_over_r0=(1.5, 1.5), mlp_dims=(33, 64, 64, 16),
                        model_seed=2)
    if name == "single512":
        return Workload(name, [FrameSpec(512, 512, 1, 3.0, 10, 11)], K=100, P=33, n_psf=8192,
                        basis_seed=13, basis_d_over_r0=(3.0, 3.0), mlp_dims=(33, 100, 100, 100),
                        model_seed=12, extra={"latency_field_seeds": list(range(100, 300))})
    if name == "spectral512":
        # RGB frame with one PSF wavelength per channel (blue, green, red)
        return Workload(name, [FrameSpec(512, 512, 3, 3.0, 16, 17)], K=100, P=33, n_psf=8192,
                        basis_seed=15, basis_d_over_r0=(3.0, 3.0), mlp_dims=(33, 100, 100, 100),
                        model_seed=12, extra={"wavelengths_nm": (450.0, 540.0, 570.0), "reference_nm": 525.0})
    shared = dict(K=100, P=33, n_psf=8192, basis_seed=14, basis_d_over_r0=(0.5, 6.0),
                  mlp_dims=(33, 100, 100, 100), model_seed=12)
    if name == "batch256":
        d = np.random.default_rng(20).uniform(1.0, 4.0, 64)
        fr = [FrameSpec(256, 256, 3, float(d[i]), 5000 + i, 1000 + i, 0.02) for i in range(64)]
        return Workload(name, fr, **shared)
    if name == "ragged":
        rng = np.random.default_rng(30)
        si = rng.integers(0, len(_RAGGED_SIZES), 200)
        ch = rng.choice([1, 3], 200)
        d = rng.uniform(0.5, 5.0, 200)
        fr = [FrameSpec(_RAGGED_SIZES[si[i]][0], _RAGGED_SIZES[si[i]][1], int(ch[i]), float(d[i]),
                        6000 + i, 2000 + i, 0.02 if ch[i] == 3 else 0.0) for i in range(200)]
        return Workload(name, fr, **shared)
    if name == "serving":
        rng = np.random.default_rng(40)
        n = 1000
        sizes = np.arange(128, 2049, 64)
        hs = rng.choice(sizes, n)
        ws = rng.choice(sizes, n)
        d = rng.uniform(0.5, 6.0, n)
        fr = [FrameSpec(int(hs[i]), int(ws[i]), 3, float(d[i]), 7000 + i, 3000 + i, 0.02)
              for i in range(n)]
        return Workload(name, fr, extra={"arrival_seed": 41, "load_fraction": 0.7,
                                         "hbm_budget_bytes": 32 << 30}, **shared)
    raise KeyError(name)


WORKLOADS = ("single128", "single512", "batch256", "ragged", "serving", "spectral512")
