"""GPU parity of wavelength-dependent colour (paper Sec. 3.5) against the FP64
oracle, through the C ABI (p2s_simulate_spectral).

Each channel has its own basis (learned from PSFs of its wavelength: phase
scaled by 525/lambda, sampling 2 lambda/525 pixels per lambda/D) and its own
network; the fields and the tilt are shared.  Tolerances as for the grey
frame: FP32 1e-5, BF16 3e-3 (relative L2).
"""
import numpy as np
import pytest

import p2s_synth as S
from oracle import basis as obasis
from oracle import spectral as ospec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def p2s():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2107_11627_amd import p2s as mod
    mod.lib()
    return mod


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def _channel_models(P=17, K=16, dims=(33, 16, 16, 16)):
    z = S.standard_normals((512, 33), 3)
    bases, Ws, bs = [], [], []
    for k, lam in enumerate(ospec.WAVELENGTHS_NM):
        q, s = ospec.channel_sampling(lam)
        bases.append(obasis.pca_basis(obasis.dataset(z, np.full(512, 1.5), P=P, Q=q, phase_scale=s), K)[0])
        w, b = S.xavier_mlp(dims, 20 + k, bias_scale=0.02)
        Ws.append(w)
        bs.append(b)
    return bases, Ws, bs


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 3e-3)])
def test_spectral_matches_oracle(p2s, prec, tol):
    from paper_2107_11627_amd import spectral
    bases, Ws, bs = _channel_models()
    img = S.blob_image(72, 90, 3, 4)
    sim = spectral.SpectralSimulator(bases, Ws, bs)
    out = sim(torch.from_numpy(img).cuda(), 2.0, 9, prec)
    torch.cuda.synchronize()
    ref = ospec.simulate_spectral(img, 2.0, bases, Ws, bs, seed=9)
    err = rel_l2(out.cpu().numpy(), ref)
    print(f"spectral {prec}: rel-L2 {err:.2e}")
    assert err < tol


def test_spectral_two_stage_network_matches_oracle(p2s):
    """A network wider than the fused kernel holds (64 > one block of 16 for
    K = 16): every channel runs the network and the blur as two kernels."""
    from paper_2107_11627_amd import spectral
    bases, Ws, bs = _channel_models(dims=(33, 64, 16))
    img = S.blob_image(40, 52, 3, 5)
    sim = spectral.SpectralSimulator(bases, Ws, bs)
    out = sim(torch.from_numpy(img).cuda(), 1.5, 3, "bf16")
    torch.cuda.synchronize()
    ref = ospec.simulate_spectral(img, 1.5, bases, Ws, bs, seed=3)
    err = rel_l2(out.cpu().numpy(), ref)
    print(f"spectral two-stage bf16: rel-L2 {err:.2e}")
    assert err < 3e-3


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_shared_channels_equal_the_grey_frame(p2s, prec):
    """With the same basis and network handles for every channel the colour
    frame is bit for bit the grey frame of p2s_simulate (the same kernels)."""
    bases, Ws, bs = _channel_models()
    B, N = p2s.Basis(bases[1]), p2s.Mlp(Ws[1], bs[1])
    img = torch.from_numpy(S.blob_image(64, 80, 3, 6)).cuda()
    ws = torch.empty(p2s.workspace_bytes(3, 64, 80, 35, B.K), dtype=torch.uint8, device="cuda")
    a = torch.empty_like(img)
    b = torch.empty_like(img)
    p2s.simulate(img, 2.5, B, N, 7, prec, a, ws)
    p2s.simulate_spectral(img, 2.5, [B] * 3, [N] * 3, 7, prec, b, ws)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_spectral_argument_errors(p2s):
    bases, Ws, bs = _channel_models()
    B, N = p2s.Basis(bases[0]), p2s.Mlp(Ws[0], bs[0])
    img = torch.zeros((3, 16, 16), device="cuda")
    out = torch.empty_like(img)
    ws = torch.empty(p2s.workspace_bytes(3, 16, 16, 35, B.K), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        p2s.simulate_spectral(img, 1.0, [B] * 2, [N] * 2, 0, "bf16", out, ws)
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(p2s.P2SError):
        p2s.simulate_spectral(img, 1.0, [B] * 3, [N] * 3, 0, "bf16", out, small)


def test_spectral_full_size_trained(p2s):
    """spectral512: 512 x 512 RGB, the three trained channel networks and
    their wavelength bases, BF16 (fused kernel per channel), against the
    oracle at sampled pixels of every channel."""
    from paper_2107_11627_amd import spectral
    from paper_2107_11627_amd import train as ptrain
    wl = S.workload("spectral512")
    fr = wl.frames[0]
    z, d = wl.basis_draws()
    bases, Ws, bs = [], [], []
    for lam, name in zip(ospec.WAVELENGTHS_NM, ("p2s_rgb450", "p2s_rgb540", "p2s_rgb570")):
        q, s = ospec.channel_sampling(lam)
        B = obasis.pca_basis(obasis.dataset(z, d, P=wl.P, Q=q, phase_scale=s), wl.K)[0]
        w, b, _ = ptrain.load(name, B)
        bases.append(B)
        Ws.append(w)
        bs.append(b)
    img = fr.image()
    sim = spectral.SpectralSimulator(bases, Ws, bs)
    out = sim(torch.from_numpy(img).cuda(), fr.d_over_r0, fr.field_seed, "bf16")
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    rng = np.random.default_rng(1)
    pix = [(c, y, x) for c in range(3) for y in (0, 255, 511) for x in (0, 256, 511)]
    pix += [(int(c), int(y), int(x)) for c, y, x in zip(rng.integers(0, 3, 60), rng.integers(0, 512, 60),
                                                         rng.integers(0, 512, 60))]
    ref = ospec.simulate_spectral_pixels(img, fr.d_over_r0, bases, Ws, bs, fr.field_seed, pix)
    g = np.array([got[c, y, x] for c, y, x in pix])
    err = rel_l2(g, ref)
    print(f"spectral512 trained bf16: rel-L2 at {len(pix)} pixels {err:.2e}")
    assert err < 3e-3
