"""GPU tests of the serving loop: requests of mixed sizes arrive while other
batches are on the device; every result equals the same request run alone
through p2s_simulate, bit for bit (the batched kernels do the same arithmetic
per frame); served requests of the serving workload's kind (K = 100 basis of
33x33, network 33-100-100-100, RGB and single-channel, ragged sizes, one of
1024 x 1088) match the FP64 oracle (FP32 1e-5, BF16 3e-3 relative L2; the
large one on sampled pixels); and the device memory the loop allocates stays
within its HBM budget."""
import numpy as np
import pytest

import p2s_synth as S
from oracle import basis as obasis
from oracle.simulate import simulate as osimulate
from oracle.simulate import simulate_pixels as osimulate_pixels

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sim():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2107_11627_amd import p2s
    wl = S.workload("single128")
    z, d = wl.basis_draws()
    B, _ = obasis.pca_basis(obasis.dataset(z, d, P=wl.P), wl.K)
    Ws, bs = wl.mlp(bias_scale=0.05)
    return p2s.Simulator(B, Ws, bs, n_zernike=35)


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_serving_mix_equals_alone(sim, prec):
    from paper_2107_11627_amd import serving as sv
    rng = np.random.default_rng(77)
    n = 40
    sizes = [64, 96, 128, 160, 256]
    reqs = []
    arr = sv.poisson_arrivals(n, 4000.0, 78)
    for i in range(n):
        C = int(rng.choice([1, 3]))
        H, W = int(rng.choice(sizes)), int(rng.choice(sizes))
        img = S.blob_image_device(H, W, C, 500 + i, noise_std=0.02)
        r = sv.Request(i, img, float(rng.uniform(0.5, 6.0)), 9000 + i, float(arr[i]))
        r.out = torch.full_like(img, float("nan"))
        reqs.append(r)
    torch.cuda.synchronize()
    budget = 512 << 20
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    ex = sv.GpuExecutor(sim, prec, budget, n_slots=2)
    eng = sv.Engine(ex, budget, n_slots=2, max_batch_frames=6)
    st = sv.run(eng, reqs)
    torch.cuda.synchronize()
    print(f"\n{prec}: {st}")
    assert st["completed"] == n and st["peak_hbm_bytes"] <= budget
    # what the loop allocated on the device (the arena) is within the budget
    assert torch.cuda.max_memory_allocated() - base <= budget
    assert st["batches"] >= 2
    for r in reqs:
        alone = sim(r.image, r.d_over_r0, r.seed, prec)
        torch.cuda.synchronize()
        assert torch.equal(r.out, alone), r.rid


@pytest.fixture(scope="module")
def serving_sim():
    from paper_2107_11627_amd import p2s
    wl = S.workload("serving")
    z, d = wl.basis_draws()
    B, _ = obasis.pca_basis(obasis.dataset(z, d, P=wl.P), wl.K)
    Ws, bs = wl.mlp()
    return p2s.Simulator(B, Ws, bs, n_zernike=wl.n_zernike), B, Ws, bs


def sample_pixels(C, H, W, n, seed):
    """n output pixels of a C x H x W frame: the four corners and edge
    midpoints of every channel, the rest uniform."""
    rng = np.random.default_rng(seed)
    pix = [(c, y, x) for c in range(C) for y in (0, H // 2, H - 1) for x in (0, W // 2, W - 1)]
    while len(pix) < n:
        pix.append((int(rng.integers(C)), int(rng.integers(H)), int(rng.integers(W))))
    return pix


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 3e-3)])
def test_served_requests_match_oracle(serving_sim, prec, tol):
    """Requests of the serving workload's kind, served while others run,
    against the FP64 oracle on the same seeded inputs."""
    from paper_2107_11627_amd import serving as sv
    sim, B, Ws, bs = serving_sim
    shapes = [(3, 128, 192), (1, 97, 131), (3, 256, 320), (3, 1024, 1088), (3, 192, 128)]
    ds = [0.5, 2.7, 6.0, 3.3, 4.1]
    arr = [0.0, 0.0002, 0.0004, 0.0006, 0.0008]
    reqs = []
    for i, (C, H, W) in enumerate(shapes):
        img = S.blob_image(H, W, C, 7100 + i, noise_std=0.02)
        r = sv.Request(i, torch.from_numpy(img).cuda(), ds[i], 3100 + i, arr[i])
        r.out = torch.full_like(r.image, float("nan"))
        r.host_image = img
        reqs.append(r)
    budget = 4 << 30
    ex = sv.GpuExecutor(sim, prec, budget, n_slots=2)
    eng = sv.Engine(ex, budget, n_slots=2, max_batch_frames=2)
    st = sv.run(eng, reqs)
    torch.cuda.synchronize()
    assert st["completed"] == len(reqs) and st["batches"] >= 2
    for r in reqs:
        C, H, W = r.shape
        got = r.out.cpu().numpy().astype(np.float64)
        if H * W <= 256 * 320:
            ref = osimulate(r.host_image, r.d_over_r0, B, Ws, bs, seed=r.seed)["out"]
            err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        else:
            pix = sample_pixels(C, H, W, 1500, r.rid)
            ref = osimulate_pixels(r.host_image, r.d_over_r0, B, Ws, bs, r.seed, pix)
            g = np.array([got[c, y, x] for c, y, x in pix])
            err = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
        print(f"{prec} request {r.rid} {r.shape} D/r0 {r.d_over_r0}: rel-L2 vs oracle {err:.2e}", flush=True)
        assert err < tol, (prec, r.rid, err)
