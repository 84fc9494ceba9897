"""GPU parity: every C-ABI call against the FP64 oracle on the same seeded
inputs.

Tolerances (relative L2 over the whole output unless stated):
  FP32: 1e-6 per stage, 1e-5 end to end.
  BF16: 3e-3 end to end and for the blur (bf16 image and basis, FP32
        accumulation and weights); 1e-4 for the network (bf16 weights that are
        bf16-representable, activations split as bf16 hi + lo).
  Philox outputs: bit-exact.
Inputs come from p2s_synth or from seeded NumPy draws; the oracle never sees a
value produced by the GPU.
"""
import numpy as np
import pytest

import p2s_synth as S
from oracle import basis as obasis
from oracle import blur as oblur
from oracle import fields as ofields
from oracle import fp8 as ofp8
from oracle import mlp as omlp
from oracle import philox as ophilox
from oracle import warp as owarp
from oracle.simulate import simulate as osimulate

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


@pytest.fixture(scope="module")
def p2s():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2107_11627_amd import p2s as mod
    mod.lib()
    return mod


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


_BASES = {}


def oracle_basis(name):
    """Basis of a workload, learned by the oracle (cached per session)."""
    if name not in _BASES:
        wl = S.workload(name)
        z, d = wl.basis_draws()
        B, _ = obasis.pca_basis(obasis.dataset(z, d, P=wl.P), wl.K)
        _BASES[name] = B
    return _BASES[name]


# ------------------------------------------------------------------ noise
@pytest.mark.parametrize("Nfy,Nfx,pair,seed", [(37, 45, 3, (1 << 40) + 7), (8, 4, 0, 0), (576, 576, 17, 11)])
def test_philox_bitwise_and_normals(p2s, Nfy, Nfx, pair, seed):
    raw = torch.zeros((Nfy, Nfx, 4), dtype=torch.int32, device="cuda")
    nrm = torch.zeros((Nfy, Nfx, 2), dtype=torch.float32, device="cuda")
    p2s.debug_noise(Nfy, Nfx, pair, seed, raw, nrm)
    got = host(raw).view(np.uint32)
    ref = ophilox.raw_bins(Nfy, Nfx, pair, seed)
    assert np.array_equal(got, ref)
    zr = ophilox.complex_normal_bins(Nfy, Nfx, pair, seed)
    zg = host(nrm)
    zg = zg[..., 0] + 1j * zg[..., 1]
    assert np.linalg.norm(zg - zr) / np.linalg.norm(zr) < 1e-6
    assert np.max(np.abs(zg - zr)) < 2e-5


# ----------------------------------------------------------------- fields
@pytest.mark.parametrize("H,W,nz,d,seed,ell", [
    (1, 1, 3, 1.0, 5, 16.0), (5, 7, 4, 2.0, 9, 1.5), (37, 45, 35, 3.0, 123, 16.0),
    (128, 128, 35, 1.5, 1, 16.0), (100, 150, 35, 4.0, 3000, 4.0),
    # 512-pixel sides: the fixed 576-point plan along x (ragged last row item),
    # along y (odd plane count), and a band too wide for it (runtime passes)
    (37, 512, 35, 2.0, 77, 16.0), (512, 45, 5, 1.0, 8, 16.0), (64, 512, 6, 2.0, 5, 8.0),
    # sides below 512 on the same 576-point grid: the last pass's guards on x < W and y < H
    (100, 480, 7, 1.5, 21, 16.0), (480, 64, 4, 2.5, 22, 16.0)])
def test_make_fields(p2s, H, W, nz, d, seed, ell):
    ws = torch.empty(p2s.fields_workspace_bytes(H, W, nz, ell), dtype=torch.uint8, device="cuda")
    F = torch.full((nz, H, W), float("nan"), dtype=torch.float32, device="cuda")
    p2s.make_fields(H, W, d, nz, seed, F, ws, corr_len_px=ell)
    ref = ofields.make_fields(H, W, d, nz, seed, corr_len=ell)
    got = host(F)
    assert np.all(np.isfinite(got))
    assert rel_l2(got, ref) < 1e-6
    for p in range(nz):
        assert rel_l2(got[p], ref[p]) < 2e-6, p


def test_make_fields_zero_turbulence(p2s):
    ws = torch.empty(p2s.fields_workspace_bytes(20, 30, 35), dtype=torch.uint8, device="cuda")
    F = torch.full((35, 20, 30), 7.0, dtype=torch.float32, device="cuda")
    p2s.make_fields(20, 30, 0.0, 35, 4, F, ws)
    assert np.all(host(F) == 0.0)


def test_make_fields_full_size_single512(p2s):
    wl = S.workload("single512")
    f = wl.frames[0]
    ws = torch.empty(p2s.fields_workspace_bytes(f.H, f.W, 35), dtype=torch.uint8, device="cuda")
    F = torch.empty((35, f.H, f.W), dtype=torch.float32, device="cuda")
    p2s.make_fields(f.H, f.W, f.d_over_r0, 35, f.field_seed, F, ws)
    ref = ofields.make_fields(f.H, f.W, f.d_over_r0, 35, f.field_seed)
    assert rel_l2(host(F), ref) < 1e-6


# -------------------------------------------------------------------- mlp
def synthetic_fields(nz, H, W, seed, scale=0.3):
    return (np.random.default_rng(seed).standard_normal((nz, H, W)) * scale).astype(np.float32)


@pytest.mark.parametrize("dims,HW,bias", [((33, 64, 64, 16), (37, 29), 0.1), ((33, 100, 100, 100), (64, 64), 0.05),
                                          ((33, 100, 100, 100), (3, 5), 0.0), ((5, 20, 7), (17, 9), 0.2),
                                          ((62, 128, 128, 128, 128), (16, 33), 0.1), ((10, 10), (8, 8), 0.3)])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mlp(p2s, dims, HW, bias, prec):
    H, W = HW
    nz = dims[0] + 2
    Ws, bs = S.xavier_mlp(dims, seed=sum(dims), bias_scale=bias)
    net = p2s.Mlp(Ws, bs)
    Fh = synthetic_fields(nz, H, W, seed=H * W)
    w = torch.full((H * W, dims[-1]), float("nan"), dtype=torch.float32, device="cuda")
    if prec == "fp32" and len(dims) == 5:
        # 3 x 128x128 FP32 layers do not fit the 160 KiB LDS of one workgroup
        with pytest.raises(p2s.P2SError) as e:
            p2s.mlp(net, dev(Fh), nz, H, W, prec, w)
        assert e.value.code == p2s.P2S_EUNSUPPORTED
        return
    p2s.mlp(net, dev(Fh), nz, H, W, prec, w)
    ref = omlp.forward(Ws, bs, np.moveaxis(Fh[2:], 0, -1).reshape(H * W, nz - 2))
    tol = 1e-6 if prec == "fp32" else 1e-4
    assert rel_l2(host(w), ref) < tol


# ------------------------------------------------------------------- blur
def blur_case(p2s, H, W, C, basis, prec, seed, wscale=1.0):
    K = basis.shape[0]
    img = S.blob_image(H, W, C, seed, noise_std=0.02 if C == 3 else 0.0)
    wh = (np.random.default_rng(seed + 1).standard_normal((H * W, K)) * wscale).astype(np.float32)
    b = p2s.Basis(basis)
    out = torch.full((C, H, W), float("nan"), dtype=torch.float32, device="cuda")
    p2s.blur(dev(img), b, dev(wh), prec, out)
    ref = np.stack([oblur.basis_blur(img[c], basis, wh.reshape(H, W, K)) for c in range(C)])
    return host(out), ref


@pytest.mark.parametrize("H,W,C,K,P", [(37, 45, 2, 20, 5), (16, 32, 1, 16, 17), (1, 1, 1, 3, 3), (50, 70, 3, 10, 9),
                                       (33, 65, 1, 128, 7), (20, 24, 1, 1, 1)])
def test_blur_fp32_random_basis(p2s, H, W, C, K, P):
    basis = np.random.default_rng(K * P).standard_normal((K, P, P)) / P
    got, ref = blur_case(p2s, H, W, C, basis, "fp32", seed=H + W)
    assert rel_l2(got, ref) < 1e-6


@pytest.mark.parametrize("H,W,C,K,P", [(37, 45, 2, 20, 17), (50, 70, 3, 10, 9), (33, 65, 1, 128, 33),
                                       (48, 64, 1, 100, 33), (19, 23, 1, 16, 25)])
def test_blur_bf16_random_basis(p2s, H, W, C, K, P):
    basis = np.random.default_rng(K * P).standard_normal((K, P, P)) / P
    got, ref = blur_case(p2s, H, W, C, basis, "bf16", seed=H + W)
    assert rel_l2(got, ref) < 3e-3


# FP8 E4M3: the GPU and the oracle round the same float32 image and basis
# values to E4M3 (ties to even) with the same per-basis power-of-two scales,
# so the two differ only by the MFMA's FP32 accumulation: 1e-4 rel-L2.  The
# error of the FP8 variant itself (against unrounded operands) is reported and
# bounded at 5e-2 (3 mantissa bits: 2^-4 relative per operand).
@pytest.mark.parametrize("H,W,C,K,P,src", [(37, 45, 2, 20, 17, "random"), (50, 70, 3, 10, 9, "random"),
                                           (33, 65, 1, 128, 33, "random"), (40, 41, 1, 7, 25, "random"),
                                           (128, 128, 1, 16, 17, "single128"), (96, 80, 2, 100, 33, "single512")])
def test_blur_fp8(p2s, H, W, C, K, P, src):
    if src == "random":
        basis = np.random.default_rng(K + P).normal(size=(K, P, P)) / P
        basis *= np.ldexp(1.0, np.random.default_rng(K).integers(-20, 5, K))[:, None, None]   # wide scale range
    else:
        basis = oracle_basis(src)
    rng = np.random.default_rng(H * W)
    img = rng.random((C, H, W)).astype(np.float32)
    img[:, :3, :3] = 0.0                                   # zeros and subnormal-range values
    img[:, 3, :5] = np.float32(1e-3)
    w = rng.normal(size=(H * W, K)).astype(np.float32)
    out = torch.empty((C, H, W), dtype=torch.float32, device="cuda")
    p2s.blur(dev(img), p2s.Basis(basis), dev(w), "fp8", out)
    got = host(out)
    ref_q = np.stack([ofp8.fp8_blur(img[c], basis, w.reshape(H, W, K)) for c in range(C)])
    ref = np.stack([oblur.basis_blur(img[c], basis, w.reshape(H, W, K)) for c in range(C)])
    eq, ee = rel_l2(got, ref_q), rel_l2(got, ref)
    print(f"\nfp8 blur {H}x{W}x{C} K={K} P={P} {src}: vs E4M3-operand oracle {eq:.2e}, vs exact operands {ee:.2e}")
    assert eq < 1e-4
    assert ee < 5e-2


@pytest.mark.parametrize("name", ["single128", "single512"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_blur_learned_basis(p2s, name, prec):
    wl = S.workload(name)
    basis = oracle_basis(name)
    got, ref = blur_case(p2s, 96, 80, 1, basis, prec, seed=3, wscale=0.2)
    assert rel_l2(got, ref) < (1e-6 if prec == "fp32" else 3e-3)


def test_blur_one_hot_is_convolution(p2s):
    """One-hot weights: the fused blur reduces to one invariant convolution."""
    from scipy import ndimage
    basis = np.random.default_rng(0).standard_normal((5, 17, 17))
    H, W = 40, 52
    img = S.blob_image(H, W, 1, 8)
    for k0 in (0, 4):
        wh = np.zeros((H * W, 5), np.float32)
        wh[:, k0] = 1.0
        b = p2s.Basis(basis)
        out = torch.empty((1, H, W), dtype=torch.float32, device="cuda")
        p2s.blur(dev(img), b, dev(wh), "fp32", out)
        ref = ndimage.convolve(img[0].astype(np.float64), basis[k0], mode="nearest")
        assert rel_l2(host(out)[0], ref) < 1e-6


# ------------------------------------------------------------------- warp
@pytest.mark.parametrize("H,W,C,sigma", [(37, 45, 1, 3.0), (64, 64, 3, 0.7), (1, 9, 1, 2.0), (128, 96, 2, 12.0)])
def test_warp(p2s, H, W, C, sigma):
    rng = np.random.default_rng(H * W + C)
    img = rng.uniform(size=(C, H, W)).astype(np.float32)
    tilt = (rng.standard_normal((2, H, W)) * sigma).astype(np.float32)
    out = torch.full((C, H, W), float("nan"), dtype=torch.float32, device="cuda")
    p2s.warp(dev(img), dev(tilt), out)
    ref = np.stack([owarp.tilt_warp(img[c], tilt[0], tilt[1]) for c in range(C)])
    assert rel_l2(host(out), ref) < 1e-6


def test_warp_zero_tilt_is_identity(p2s):
    img = np.random.default_rng(1).uniform(size=(2, 30, 41)).astype(np.float32)
    out = torch.empty((2, 30, 41), dtype=torch.float32, device="cuda")
    p2s.warp(dev(img), torch.zeros((2, 30, 41), device="cuda"), out)
    assert np.array_equal(host(out), img)


# ------------------------------------------------------- fused network+blur
@pytest.mark.parametrize("dims,K,P,C,H,W,prec", [
    ((33, 100, 100, 100), 100, 33, 1, 96, 80, "bf16"),
    ((33, 100, 100, 100), 100, 33, 3, 37, 45, "bf16"),
    ((33, 48, 48, 40), 40, 17, 2, 50, 70, "bf16"),
    ((33, 48, 48, 40), 40, 17, 2, 50, 70, "fp8"),
    ((33, 16, 16), 16, 9, 1, 33, 65, "fp8"),
    # FP8 at the headline shape with three channels (the second tile instance), and P = 25
    ((33, 100, 100, 100), 100, 33, 3, 37, 45, "fp8"),
    ((33, 48, 48, 40), 40, 25, 1, 41, 50, "fp8"),
])
def test_mlp_blur_fused_equals_staged(p2s, dims, K, P, C, H, W, prec):
    """The network evaluated inside the blur epilogue gives bit for bit what
    p2s_mlp followed by p2s_blur gives (same MFMA arithmetic per pixel)."""
    Ws, bs = S.xavier_mlp(dims, 31, bias_scale=0.05)
    net = p2s.Mlp(Ws, bs)
    basis = p2s.Basis(np.random.default_rng(K + P).normal(size=(K, P, P)) / P)
    nz = dims[0] + 2
    F = dev(synthetic_fields(nz, H, W, 5))
    img = dev(np.random.default_rng(6).random((C, H, W)))
    w = torch.empty((H * W, K), dtype=torch.float32, device="cuda")
    staged = torch.empty((C, H, W), dtype=torch.float32, device="cuda")
    fused = torch.full((C, H, W), -1.0, dtype=torch.float32, device="cuda")
    p2s.mlp(net, F, nz, H, W, prec, w)
    p2s.blur(img, basis, w, prec, staged)
    p2s.mlp_blur(net, F, nz, img, basis, prec, fused)
    assert np.array_equal(host(fused), host(staged))


def test_mlp_blur_unsupported(p2s):
    wl = S.workload("single128")
    Ws, bs = wl.mlp()                        # 33-64-64-16: hidden layers wider than the K = 16 basis
    net = p2s.Mlp(Ws, bs)
    basis = p2s.Basis(np.random.default_rng(1).normal(size=(16, 17, 17)))
    F = torch.zeros((35, 8, 8), device="cuda")
    img = torch.zeros((1, 8, 8), device="cuda")
    out = torch.empty_like(img)
    for prec in ("bf16", "fp32"):
        with pytest.raises(p2s.P2SError) as e:
            p2s.mlp_blur(net, F, 35, img, basis, prec, out)
        assert e.value.code == p2s.P2S_EUNSUPPORTED


def test_simulate_fused_equals_staged(p2s):
    """p2s_simulate (network fused into the blur for this workload) against
    the four stage calls made one by one."""
    wl = S.workload("single512")
    f = wl.frames[0]
    basis = oracle_basis("single512")
    Ws, bs = wl.mlp()
    sim = p2s.Simulator(basis, Ws, bs, n_zernike=35)
    img = dev(f.image())
    for prec in ("bf16", "fp8"):
        got = host(sim(img, f.d_over_r0, f.field_seed, prec))
        H, W = f.H, f.W
        F = torch.empty((35, H, W), dtype=torch.float32, device="cuda")
        fws = torch.empty(p2s.fields_workspace_bytes(H, W, 35), dtype=torch.uint8, device="cuda")
        w = torch.empty((H * W, 100), dtype=torch.float32, device="cuda")
        bl = torch.empty_like(img)
        out = torch.empty_like(img)
        p2s.make_fields(H, W, f.d_over_r0, 35, f.field_seed, F, fws)
        p2s.mlp(sim.net, F, 35, H, W, prec, w)
        p2s.blur(img, sim.basis, w, prec, bl)
        p2s.warp(bl, F, out)
        assert np.array_equal(got, host(out)), prec


# --------------------------------------------------------------- simulate
def run_sim(p2s, img, d, basis, Ws, bs, seed, prec, nz=35):
    C, H, W = img.shape
    sim = p2s.Simulator(basis, Ws, bs, n_zernike=nz)
    out = sim(dev(img), d, seed, prec)
    return host(out)


@pytest.mark.parametrize("name", ["single128", "single512"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_simulate_workload(p2s, name, prec):
    wl = S.workload(name)
    f = wl.frames[0]
    basis = oracle_basis(name)
    Ws, bs = wl.mlp()
    img = f.image()
    got = run_sim(p2s, img, f.d_over_r0, basis, Ws, bs, f.field_seed, prec)
    ref = osimulate(img, f.d_over_r0, basis, Ws, bs, seed=f.field_seed)["out"]
    err = rel_l2(got, ref)
    print(f"\n{name} {prec} end-to-end rel-L2 vs FP64 oracle: {err:.3e}")
    assert err < (1e-5 if prec == "fp32" else 3e-3)


@pytest.mark.parametrize("name", ["single128", "single512"])
def test_simulate_fp8(p2s, name):
    """FP8 blur (network on BF16 MFMA with bf16 activations) end to end:
    against the oracle with E4M3 blur operands, 5e-3 (what remains is the
    network's activation rounding: unit roundoff 2^-9 at each of 3 layers,
    about 2e-3 on w for a random network), and the FP8 variant's own error
    against the exact oracle reported."""
    wl = S.workload(name)
    f = wl.frames[0]
    basis = oracle_basis(name)
    Ws, bs = wl.mlp()
    img = f.image()
    got = run_sim(p2s, img, f.d_over_r0, basis, Ws, bs, f.field_seed, "fp8")
    ref_q = osimulate(img, f.d_over_r0, basis, Ws, bs, seed=f.field_seed, blur_operands="fp8")["out"]
    ref = osimulate(img, f.d_over_r0, basis, Ws, bs, seed=f.field_seed)["out"]
    eq, ee = rel_l2(got, ref_q), rel_l2(got, ref)
    print(f"\n{name} fp8 end-to-end rel-L2: vs E4M3-operand oracle {eq:.3e}, vs FP64 oracle {ee:.3e}")
    assert eq < 5e-3
    assert ee < 5e-2


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_simulate_rgb_ragged_with_bias(p2s, prec):
    wl = S.workload("single128")
    basis = oracle_basis("single128")
    Ws, bs = wl.mlp(bias_scale=0.05)
    img = S.blob_image(70, 113, 3, 77, noise_std=0.02)
    got = run_sim(p2s, img, 2.5, basis, Ws, bs, 4242, prec)
    ref = osimulate(img, 2.5, basis, Ws, bs, seed=4242)["out"]
    assert rel_l2(got, ref) < (1e-5 if prec == "fp32" else 3e-3)
    # Sec. 3.5: every channel sees the same distortion
    one = run_sim(p2s, img[1:2].copy(), 2.5, basis, Ws, bs, 4242, prec)
    assert np.array_equal(one[0], got[1])


def test_simulate_deterministic(p2s):
    wl = S.workload("single128")
    basis = oracle_basis("single128")
    Ws, bs = wl.mlp()
    img = wl.frames[0].image()
    a = run_sim(p2s, img, 1.5, basis, Ws, bs, 1, "bf16")
    b = run_sim(p2s, img, 1.5, basis, Ws, bs, 1, "bf16")
    assert np.array_equal(a, b)


def test_errors_through_binding(p2s):
    wl = S.workload("single128")
    Ws, bs = wl.mlp()
    basis = oracle_basis("single128")
    sim = p2s.Simulator(basis, Ws, bs, n_zernike=35)
    img = dev(wl.frames[0].image())
    with pytest.raises(p2s.P2SError) as e:
        p2s.simulate(img, 1.5, sim.basis, sim.net, 1, 7, torch.empty_like(img), sim.workspace(1, 128, 128))
    assert e.value.code == p2s.P2S_EINVAL
    with pytest.raises(p2s.P2SError) as e:
        p2s.simulate(img, 1.5, sim.basis, sim.net, 1, "fp32", torch.empty_like(img), sim.workspace(1, 128, 128),
                     n_zernike=20)
    assert e.value.code == p2s.P2S_EINVAL
    small_ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(p2s.P2SError):
        p2s.simulate(img, 1.5, sim.basis, sim.net, 1, "fp32", torch.empty_like(img), small_ws)
    b5 = p2s.Basis(np.ones((16, 5, 5)) / 25)
    for prec in ("bf16", "fp8"):
        with pytest.raises(p2s.P2SError) as e:
            p2s.blur(img, b5, torch.zeros((128 * 128, 16), device="cuda"), prec, torch.empty_like(img))
        assert e.value.code == p2s.P2S_EUNSUPPORTED


def generic_xavier(dims, seed, bias_scale):
    """Xavier-uniform weights and uniform biases as plain float32 draws (not
    rounded to bfloat16-representable values), as a trained network would
    have them."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for l in range(len(dims) - 1):
        a = np.sqrt(6.0 / (dims[l] + dims[l + 1]))
        Ws.append(rng.uniform(-a, a, size=(dims[l + 1], dims[l])).astype(np.float32))
        bs.append(rng.uniform(-bias_scale, bias_scale, size=dims[l + 1]).astype(np.float32))
    return Ws, bs


def test_bf16_with_generic_fp32_weights(p2s):
    """BF16 network and frame with weights that are not bf16-representable
    (the BF16 path rounds them to bfloat16 once, at p2s_mlp_create), against
    the oracle run with the original float32 weights.  Tolerances: network
    output 5e-3 (weights rounded with unit roundoff 2^-9 = 2e-3 each; the
    errors of a layer's 100 products average out to about 2^-9/sqrt(3) of the
    output, and three layers add in quadrature: ~2e-3); end to end 1e-2 (the
    weight error of w times the blur's median cancellation factor of ~7,
    partly averaged over the frame)."""
    wl = S.workload("single512")
    fr = wl.frames[0]
    Ws, bs = generic_xavier(wl.mlp_dims, 91, 0.05)
    net = p2s.Mlp(Ws, bs)
    H, W, nz = 128, 160, wl.n_zernike
    Fh = synthetic_fields(nz, H, W, seed=5, scale=0.15)
    w = torch.empty((H * W, wl.K), dtype=torch.float32, device="cuda")
    p2s.mlp(net, dev(Fh), nz, H, W, "bf16", w)
    ref = omlp.forward(Ws, bs, np.moveaxis(Fh[2:], 0, -1).reshape(H * W, nz - 2))
    e_net = rel_l2(host(w), ref)
    basis = oracle_basis("single512")
    sim = p2s.Simulator(basis, Ws, bs, n_zernike=nz)
    img = fr.image()
    out = sim(dev(img), fr.d_over_r0, fr.field_seed, "bf16")
    refo = osimulate(img, fr.d_over_r0, basis, Ws, bs, seed=fr.field_seed)["out"]
    e_sim = rel_l2(host(out), refo)
    print(f"generic float32 weights, BF16 path: network {e_net:.2e}, frame {e_sim:.2e}", flush=True)
    assert e_net < 5e-3 and e_sim < 1e-2, (e_net, e_sim)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 3e-3), ("fp8", 5e-3)])
def test_simulate_trained_network(p2s, prec, tol):
    """A whole 512x512 frame with the trained P2S network of that workload's
    basis (weights are data: the kernels are the same) against the oracle;
    FP8 against the oracle fed the same E4M3-rounded blur operands."""
    from paper_2107_11627_amd import train
    wl = S.workload("single512")
    fr = wl.frames[0]
    basis = oracle_basis("single512")
    Ws, bs, _ = train.load("p2s_single512", basis)
    sim = p2s.Simulator(basis, Ws, bs, n_zernike=wl.n_zernike)
    img = fr.image()
    out = sim(dev(img), fr.d_over_r0, fr.field_seed, prec)
    ref = osimulate(img, fr.d_over_r0, basis, Ws, bs, seed=fr.field_seed,
                    blur_operands="fp8" if prec == "fp8" else "exact")["out"]
    err = rel_l2(host(out), ref)
    print(f"trained network, {prec}: rel-L2 vs oracle {err:.2e}", flush=True)
    assert err < tol
