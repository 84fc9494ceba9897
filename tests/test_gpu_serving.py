"""GPU test of the serving loop: requests of mixed sizes arrive while other
batches are on the device; every result equals the same request run alone
through p2s_simulate, bit for bit (the batched kernels do the same arithmetic
per frame), and the HBM budget holds."""
import numpy as np
import pytest

import p2s_synth as S
from oracle import basis as obasis

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
        reqs.append(sv.Request(i, img, float(rng.uniform(0.5, 6.0)), 9000 + i, float(arr[i])))
    torch.cuda.synchronize()
    budget = 512 << 20
    ex = sv.GpuExecutor(sim, prec, budget, n_slots=2)
    eng = sv.Engine(ex, budget, n_slots=2, max_batch_frames=6)
    st = sv.run(eng, reqs)
    torch.cuda.synchronize()
    print(f"\n{prec}: {st}")
    assert st["completed"] == n and st["peak_hbm_bytes"] <= budget
    assert st["batches"] >= 2
    for r in reqs:
        alone = sim(r.image, r.d_over_r0, r.seed, prec)
        torch.cuda.synchronize()
        assert torch.equal(r.out, alone), r.rid
