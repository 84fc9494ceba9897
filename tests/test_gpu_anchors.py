"""GPU parity of the anchor-grid field model (paper Sec. 3.4 with Noll's R_Z)
against the FP64 oracle, through the C ABI.

The device path draws the anchor normals with its own Philox, forms
L_s (E L_Z^T) with FP32 MFMA and interpolates in FP32; the oracle does the
same in FP64 from its own matrices.  Tolerance: relative L2 per plane 1e-5
(an FP32 dot product of up to G^2 = 4096 terms of either sign carries a
relative error of a few 1e-7 rms; the bilinear step adds one rounding per
term).  End to end: FP32 1e-5, BF16 3e-3, as for the FFT fields.
"""
import numpy as np
import pytest

import p2s_synth as S
from oracle import anchors as oanch
from oracle import basis as obasis
from oracle.simulate import simulate as osimulate
from oracle.simulate import simulate_pixels as osimulate_pixels

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def p2s():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2107_11627_amd import p2s as mod
    mod.lib()
    return mod


@pytest.fixture(scope="module")
def panch(p2s):
    from paper_2107_11627_amd import anchors as mod
    return mod


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def device_fields(p2s, model, H, W, d, seed):
    ws = torch.empty(model.fields_workspace_bytes(), dtype=torch.uint8, device="cuda")
    F = torch.full((model.n_zernike, H, W), float("nan"), dtype=torch.float32, device="cuda")
    p2s.make_fields_anchor(model, H, W, d, seed, F, ws)
    torch.cuda.synchronize()
    return F.cpu().numpy()


@pytest.mark.parametrize("G,H,W,n,corr", [
    (2, 1, 1, 3, 2.0),        # one pixel, one cell
    (5, 9, 13, 12, 2.0),      # anchors on pixels
    (8, 33, 47, 35, 2.0),     # ragged, one column tile of the product
    (16, 128, 96, 35, 3.0),   # several segments
    (40, 20, 30, 17, 1.5),    # more anchors than pixels: cells with no pixel row
    (12, 1, 200, 64, 2.0),    # a single row, four column tiles
    (12, 150, 1, 1, 2.0),     # a single column, one plane
    (33, 65, 700, 20, 2.5),   # G^2 = 1089: padded to 1120 (odd number of 16-row tiles before padding)
])
def test_anchor_fields_match_oracle(p2s, panch, G, H, W, n, corr):
    model = panch.anchor_model(G, n, corr)
    got = device_fields(p2s, model, H, W, 1.7, 11)
    ref = oanch.make_fields(H, W, 1.7, n, 11, G=G, corr_len=corr)
    assert np.all(np.isfinite(got))
    errs = [rel_l2(got[i], ref[i]) for i in range(n)]
    print(f"anchor fields G={G} {H}x{W} n={n}: max per-plane rel-L2 {max(errs):.2e}")
    assert max(errs) < 1e-5


def test_anchor_fields_full_size(p2s, panch):
    """The 512 x 512 frame on the paper's 64 x 64 anchor grid (the 4096 x 4096
    correlation matrix), every plane of every pixel."""
    model = panch.anchor_model(64, 35, 2.0)
    got = device_fields(p2s, model, 512, 512, 2.0, 5)
    ref = oanch.make_fields(512, 512, 2.0, 35, 5, G=64, corr_len=2.0)
    errs = [rel_l2(got[i], ref[i]) for i in range(35)]
    print(f"anchor fields 64x64 grid, 512x512: max per-plane rel-L2 {max(errs):.2e}")
    assert max(errs) < 1e-5


def test_anchor_fields_deterministic_and_seeded(p2s, panch):
    """Same seed: bit-identical planes; another seed: other planes; zero
    turbulence: zero planes."""
    model = panch.anchor_model(16, 35, 2.0)
    a = device_fields(p2s, model, 64, 80, 1.0, 3)
    b = device_fields(p2s, model, 64, 80, 1.0, 3)
    c = device_fields(p2s, model, 64, 80, 1.0, 4)
    z = device_fields(p2s, model, 64, 80, 0.0, 3)
    assert np.array_equal(a, b)
    assert not np.allclose(a, c)
    assert np.all(z == 0.0)


def test_anchor_workspace_checked(p2s, panch):
    model = panch.anchor_model(8, 35, 2.0)
    ws = torch.empty(model.fields_workspace_bytes() - 256, dtype=torch.uint8, device="cuda")
    F = torch.empty((35, 16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(p2s.P2SError):
        p2s.make_fields_anchor(model, 16, 16, 1.0, 0, F, ws)


def _small_model():
    z = S.standard_normals((512, 33), 3)
    basis, _ = obasis.pca_basis(obasis.dataset(z, np.full(512, 1.5), P=17), 16)
    Ws, bs = S.xavier_mlp((33, 16, 16, 16), 2, bias_scale=0.02)
    return basis, Ws, bs


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 3e-3)])
def test_simulate_anchor_matches_oracle(p2s, panch, prec, tol):
    """A frame end to end with the anchor model as stage 1 (RGB, ragged)."""
    basis, Ws, bs = _small_model()
    img = S.blob_image(72, 90, 3, 4)
    model = panch.anchor_model(16, 35, 2.0)
    B, N = p2s.Basis(basis), p2s.Mlp(Ws, bs)
    x = torch.from_numpy(img).cuda()
    out = torch.empty_like(x)
    ws = torch.empty(model.workspace_bytes(3, 72, 90, 16), dtype=torch.uint8, device="cuda")
    p2s.simulate_anchor(x, 2.0, model, B, N, 9, prec, out, ws)
    torch.cuda.synchronize()
    ref = osimulate(img, 2.0, basis, Ws, bs, seed=9, field_model="anchor", G=16, anchor_corr=2.0)["out"]
    err = rel_l2(out.cpu().numpy(), ref)
    print(f"simulate_anchor {prec}: rel-L2 {err:.2e}")
    assert err < tol


def test_simulate_anchor_full_size_trained(p2s, panch):
    """single512 with the trained network and the 64 x 64 anchor grid, BF16
    (the fused network-and-blur kernel), at sampled output pixels."""
    from paper_2107_11627_amd import train as ptrain
    wl = S.workload("single512")
    z, d = wl.basis_draws()
    basis, _ = obasis.pca_basis(obasis.dataset(z, d, P=wl.P), wl.K)
    Ws, bs, _ = ptrain.load("p2s_single512", basis)
    img = S.blob_image(512, 512, 1, 2)
    model = panch.anchor_model(64, 35, 2.0)
    B, N = p2s.Basis(basis), p2s.Mlp(Ws, bs)
    x = torch.from_numpy(img).cuda()
    out = torch.empty_like(x)
    ws = torch.empty(model.workspace_bytes(1, 512, 512, basis.shape[0]), dtype=torch.uint8, device="cuda")
    p2s.simulate_anchor(x, 3.0, model, B, N, 21, "bf16", out, ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    rng = np.random.default_rng(0)
    pix = [(0, int(y), int(x_)) for y, x_ in zip(rng.integers(0, 512, 48), rng.integers(0, 512, 48))]
    pix += [(0, 0, 0), (0, 511, 511), (0, 0, 511), (0, 255, 256)]
    ref = osimulate_pixels(img, 3.0, basis, Ws, bs, 21, pix, field_model="anchor", G=64, anchor_corr=2.0)
    g = np.array([got[c, y, x_] for c, y, x_ in pix], dtype=np.float64)
    err = rel_l2(g, ref)
    print(f"simulate_anchor single512 bf16 trained: rel-L2 at {len(pix)} pixels {err:.2e}")
    assert err < 3e-3
