"""The trained P2S networks (Sec. 3.3) against the oracle's physics.

The models under paper_2107_11627_amd/weights were trained by the package's
host trainer on PSFs it formed itself; here the oracle forms independent
held-out PSFs with its own Eq. 2 (at the model's wavelength for the per-channel
colour models) and PCA-free projection, and checks:
  * the network's basis coefficients on held-out Zernike draws against the
    projections of the oracle's PSFs (relative l2 of beta);
  * zero turbulence: the network at alpha = 0 against the projection of the
    diffraction-limited (Airy) PSF;
  * a constant image stays close to constant through the whole oracle frame
    with the trained weights (the blur is approximately normalised).
The bounds sit above the measured values (printed) by a margin; they pin the
trained model, not the method, which has no exact value to compare with."""
import numpy as np
import pytest

import p2s_synth as S
from oracle import basis as obasis
from oracle import mlp as omlp
from oracle import psf as opsf
from oracle import spectral
from oracle.simulate import simulate


@pytest.fixture(scope="module")
def models():
    from paper_2107_11627_amd import train
    out = {}
    for name, (wl_name, drange, _, lam) in train.MODELS.items():
        wl = S.workload(wl_name)
        B = train.workload_basis(wl, lam)
        Ws, bs, meta = train.load(name, B)           # checks the content hash and the basis
        q, s = spectral.channel_sampling(lam) if lam else (2.0, 1.0)
        out[name] = (B, Ws, bs, meta, drange, wl, q, s)
    return out


@pytest.mark.parametrize("name,bound", [("p2s_single512", 0.12), ("p2s_shared", 0.15), ("p2s_rgb450", 0.15),
                                        ("p2s_rgb540", 0.12), ("p2s_rgb570", 0.12)])
def test_held_out_coefficients(models, name, bound):
    B, Ws, bs, meta, (dlo, dhi), wl, q, s = models[name]
    rng = np.random.default_rng(987)
    n = 1024
    z = rng.standard_normal((n, wl.n_zernike - 2))
    d = rng.uniform(dlo, dhi, n)
    psfs = obasis.dataset(z, d, P=wl.P, Q=q, phase_scale=s)        # oracle Eq. 2 at the model's wavelength
    beta = psfs.reshape(n, -1) @ B.reshape(wl.K, -1).T              # projection on the basis
    from oracle.noll import noll_variance
    sig = np.sqrt(np.array([noll_variance(j) for j in range(4, wl.n_zernike + 2)]))
    alpha = z * sig[None, :] * (d ** (5.0 / 6.0))[:, None]
    pred = omlp.forward(Ws, bs, alpha)
    err = float(np.linalg.norm(pred - beta) / np.linalg.norm(beta))
    print(f"{name}: held-out relative l2 of beta {err:.4f} (trainer's own held-out {meta['held_out']['rel_l2_beta']:.4f})")
    assert err < bound


@pytest.mark.parametrize("name,bound", [("p2s_single512", 0.06), ("p2s_shared", 0.04), ("p2s_rgb450", 0.10),
                                        ("p2s_rgb540", 0.06), ("p2s_rgb570", 0.06)])
def test_zero_turbulence_gives_airy_projection(models, name, bound):
    B, Ws, bs, meta, _, wl, q, s = models[name]
    airy = opsf.psf_from_zernike(np.zeros((1, wl.n_zernike - 2)), range(4, wl.n_zernike + 2), 32, q, wl.P)[0]
    beta0 = B.reshape(wl.K, -1) @ airy.reshape(-1)
    pred = omlp.forward(Ws, bs, np.zeros((1, wl.n_zernike - 2)))[0]
    err = float(np.linalg.norm(pred - beta0) / np.linalg.norm(beta0))
    print(f"{name}: network at alpha = 0 vs Airy projection {err:.4f}")
    assert err < bound


def test_constant_image_nearly_preserved(models):
    B, Ws, bs, meta, _, wl, _, _ = models["p2s_single512"]
    img = np.full((1, 48, 56), 0.6)
    out = simulate(img, 3.0, B, Ws, bs, seed=5)["out"][0] / 0.6
    dev = np.abs(out - 1.0)
    print(f"constant image: mean |out/c - 1| {dev.mean():.4f}, max {dev.max():.4f}")
    assert dev.mean() < 0.01 and dev.max() < 0.03
