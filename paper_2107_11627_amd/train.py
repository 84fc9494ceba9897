"""One-time training of the P2S network (Sec. 3.3) on the host.

The network maps the tilt-free Zernike coefficients alpha_4.. of a PSF to the
coefficients beta of that PSF in the PCA basis (Sec. 3.2).  Training pairs
come from the same construction as the basis: alpha drawn with the Noll
variances scaled by (D/r0)^(5/3) over the basis' range of D/r0, the PSF
formed with Eq. 2, and its target beta = <PSF, phi_m>, the projection onto the
orthonormal basis; the loss is the squared l2 distance between the network
output and beta, averaged over the batch (Adam).

The architecture is the one the kernels run: y = W x + b per layer, ReLU
after the hidden layers, linear output, raw alpha in radians at the input.
For conditioning the training works on standardised inputs and targets; the
scales are folded into the first and last layers afterwards (an exact
rewrite), and the weights and biases are then rounded once to
bfloat16-representable values, so that one model is exact in FP64, FP32 and
BF16 alike.  Like the basis, this runs once per configuration, before any
frame; it is not part of the per-frame path.

Trained models are stored under ``weights/`` as .npz files named by the
SHA-256 of their contents, with a JSON manifest giving the recipe and the
digest of the basis they belong to.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import List, Sequence, Tuple

import numpy as np

from . import basis as pbasis
from . import p2s

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights")


def zernike_sigmas(n_zernike: int = 35) -> np.ndarray:
    return np.sqrt(np.array([p2s.noll_variance(int(j)) for j in range(4, n_zernike + 2)]))


def training_pairs(normals: np.ndarray, d_over_r0: np.ndarray, basis: np.ndarray, n_zernike: int = 35,
                   Q: float = 2, phase_scale: float = 1.0):
    """(alpha [n][n_zernike-2], beta [n][K]) for standard normals and D/r0
    draws: alpha_j = normal * sqrt(V_j (D/r0)^(5/3)); beta = projection of
    the Eq. 2 PSF of alpha onto the basis (for another wavelength: the PSF of
    phase_scale alpha sampled at Q pixels per lambda/D, while the network's
    input stays the reference alpha)."""
    K, P, _ = basis.shape
    alpha = normals * zernike_sigmas(n_zernike)[None, :] * (np.asarray(d_over_r0) ** (5.0 / 6.0))[:, None]
    psfs = pbasis.psf_dataset(normals, d_over_r0, P, n_zernike, Q=Q, phase_scale=phase_scale)
    beta = psfs.reshape(len(psfs), P * P) @ basis.reshape(K, P * P).T
    return alpha, beta


def basis_fingerprint(basis: np.ndarray) -> List[float]:
    """K numbers that identify a basis up to round-off: each basis function
    dotted with one fixed pseudo-random vector of taps.  A model is tied to
    its basis by these (a sign flip or a rotation within a near-degenerate
    pair of components changes them; the last bits of the SVD do not)."""
    K = basis.shape[0]
    r = np.random.default_rng(0).standard_normal(basis[0].size)
    return [float(v) for v in np.asarray(basis, dtype=np.float64).reshape(K, -1) @ r]


def same_basis(fp_a: Sequence[float], fp_b: Sequence[float], tol: float = 1e-7) -> bool:
    return len(fp_a) == len(fp_b) and float(np.max(np.abs(np.subtract(fp_a, fp_b)))) <= tol


def _bf16(x: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).reshape(a.shape)


def train(alpha: np.ndarray, beta: np.ndarray, dims: Sequence[int], seed: int, steps: int = 20000,
          batch: int = 1024, lr: float = 2e-3, log=None) -> Tuple[List[np.ndarray], List[np.ndarray]]:
    """Adam on the mean squared l2 error; returns (weights [out][in],
    biases) as float32, scales folded in, bf16-representable."""
    import torch
    g = torch.Generator().manual_seed(seed)
    torch.manual_seed(seed)
    xm, xs = alpha.mean(0), alpha.std(0) + 1e-12
    ym, ys = beta.mean(0), beta.std(0).mean() + 1e-12     # one output scale: keeps the l2 loss's weighting
    X = torch.from_numpy((alpha - xm) / xs).float()
    Y = torch.from_numpy((beta - ym) / ys).float()
    layers = []
    for l in range(len(dims) - 1):
        lin = torch.nn.Linear(dims[l], dims[l + 1])
        torch.nn.init.xavier_uniform_(lin.weight, generator=g)
        torch.nn.init.zeros_(lin.bias)
        layers.append(lin)
    params = [p for lin in layers for p in lin.parameters()]
    opt = torch.optim.Adam(params, lr=lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, steps)

    def fwd(x):
        for l, lin in enumerate(layers):
            x = lin(x)
            if l + 1 < len(layers):
                x = torch.relu(x)
        return x

    n = X.shape[0]
    for it in range(steps):
        idx = torch.randint(0, n, (batch,), generator=g)
        loss = ((fwd(X[idx]) - Y[idx]) ** 2).sum(1).mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
        sched.step()
        if log and (it % 1000 == 0 or it + 1 == steps):
            log(f"step {it}: loss {loss.item():.4e}")
    Ws = [lin.weight.detach().double().numpy() for lin in layers]
    bs = [lin.bias.detach().double().numpy() for lin in layers]
    # fold the standardisation: x_std = (alpha - xm) / xs, y = ys y_std + ym
    b0 = bs[0] - Ws[0] @ (xm / xs)
    Ws[0] = Ws[0] / xs[None, :]
    bs[0] = b0
    Ws[-1] = Ws[-1] * ys
    bs[-1] = bs[-1] * ys + ym
    return [_bf16(w) for w in Ws], [_bf16(b) for b in bs]


def forward(Ws, bs, x: np.ndarray) -> np.ndarray:
    h = np.asarray(x, dtype=np.float64)
    for l in range(len(Ws)):
        h = h @ np.asarray(Ws[l], dtype=np.float64).T + np.asarray(bs[l], dtype=np.float64)
        if l + 1 < len(Ws):
            h = np.maximum(h, 0.0)
    return h


def save(name: str, Ws, bs, meta: dict) -> str:
    """Write weights/<name>_<sha12>.npz and its manifest; returns the path."""
    os.makedirs(WEIGHTS, exist_ok=True)
    arrays = {}
    for l, (w, b) in enumerate(zip(Ws, bs)):
        arrays[f"W{l}"] = np.ascontiguousarray(w, dtype=np.float32)
        arrays[f"b{l}"] = np.ascontiguousarray(b, dtype=np.float32)
    h = hashlib.sha256()
    for k in sorted(arrays):
        h.update(k.encode())
        h.update(arrays[k].tobytes())
    digest = h.hexdigest()[:12]
    path = os.path.join(WEIGHTS, f"{name}_{digest}.npz")
    np.savez(path, **arrays)
    with open(os.path.join(WEIGHTS, f"{name}.json"), "w") as f:
        json.dump(dict(meta, file=os.path.basename(path), sha256_12=digest), f, indent=1, sort_keys=True)
    return path


def load(name: str, basis: np.ndarray = None):
    """(weights, biases, manifest) of a stored model; checks the content hash
    and, when a basis is given, that the model was trained for it."""
    with open(os.path.join(WEIGHTS, f"{name}.json")) as f:
        meta = json.load(f)
    z = np.load(os.path.join(WEIGHTS, meta["file"]), allow_pickle=False)
    n = len([k for k in z.files if k.startswith("W")])
    Ws = [z[f"W{l}"] for l in range(n)]
    bs = [z[f"b{l}"] for l in range(n)]
    h = hashlib.sha256()
    for k in sorted(z.files):
        h.update(k.encode())
        h.update(z[k].tobytes())
    if h.hexdigest()[:12] != meta["sha256_12"]:
        raise ValueError(f"{meta['file']}: content does not match its hash")
    if basis is not None and not same_basis(basis_fingerprint(basis), meta["basis_fingerprint"]):
        raise ValueError(f"{name}: trained for another basis than the one given")
    return Ws, bs, meta


# Models of the synthetic workloads: (workload whose basis it serves,
# training D/r0 range, training seed, PSF wavelength in nm or None for the
# reference wavelength).  The single-frame workload's basis is learned at
# D/r0 = 3, the shared one over [0.5, 6]; the spectral workload has one basis
# and one network per channel wavelength.
MODELS = {
    "p2s_single512": ("single512", (2.0, 4.0), 201, None),
    "p2s_shared": ("batch256", (0.5, 6.0), 202, None),
    "p2s_rgb450": ("spectral512", (2.0, 4.0), 211, 450.0),
    "p2s_rgb540": ("spectral512", (2.0, 4.0), 212, 540.0),
    "p2s_rgb570": ("spectral512", (2.0, 4.0), 213, 570.0),
}


def workload_basis(wl, wavelength_nm=None):
    """The PCA basis a model of workload wl serves (at a channel wavelength
    for the spectral workload)."""
    z, d = wl.basis_draws()
    if wavelength_nm is None:
        return pbasis.learn_basis(z, d, wl.K, wl.P, wl.n_zernike)[0]
    from . import spectral
    return spectral.channel_basis(z, d, wl.K, wl.P, wavelength_nm, wl.n_zernike)[0]


def build_model(name: str, n_train: int = 65536, n_test: int = 4096, steps: int = 20000, log=print):
    """Train and store the named model; returns (path, held-out relative
    l2 error of beta)."""
    import p2s_synth as S
    wl_name, (dlo, dhi), seed, lam = MODELS[name]
    wl = S.workload(wl_name)
    B = workload_basis(wl, lam)
    rng = np.random.default_rng(seed)
    nz = rng.standard_normal((n_train + n_test, wl.n_zernike - 2))
    dd = rng.uniform(dlo, dhi, n_train + n_test)
    if lam is None:
        alpha, beta = training_pairs(nz, dd, B, wl.n_zernike)
    else:
        from . import spectral
        q, s = spectral.channel_sampling(lam)
        alpha, beta = training_pairs(nz, dd, B, wl.n_zernike, Q=q, phase_scale=s)
    Ws, bs = train(alpha[:n_train], beta[:n_train], wl.mlp_dims, seed, steps=steps, log=log)
    pred = forward(Ws, bs, alpha[n_train:])
    err = float(np.linalg.norm(pred - beta[n_train:]) / np.linalg.norm(beta[n_train:]))
    meta = {"workload_basis": wl_name, "basis_fingerprint": basis_fingerprint(B), "dims": list(wl.mlp_dims),
            "wavelength_nm": lam,
            "train": {"n": n_train, "seed": seed, "d_over_r0": [dlo, dhi], "steps": steps, "batch": 1024,
                      "lr": 2e-3, "schedule": "cosine", "optimizer": "Adam", "loss": "mean squared l2 of beta"},
            "held_out": {"n": n_test, "rel_l2_beta": err}}
    path = save(name, Ws, bs, meta)
    log(f"{name}: held-out relative l2 error of beta {err:.4f} -> {path}")
    return path, err


if __name__ == "__main__":
    import sys
    for nm in (sys.argv[1:] or list(MODELS)):
        build_model(nm)
