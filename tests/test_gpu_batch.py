"""GPU tests of the batched path (p2s_batch_* / p2s_simulate_batch).

A frame run inside a batch does the same arithmetic as the same frame run
alone through p2s_simulate (only the schedule differs), so the batch output is
compared with the solo output bit for bit; the solo path is itself checked
against the FP64 oracle in test_gpu_parity.py, and one batch frame is also
checked against the oracle directly here.  Full-size batches (64 RGB 256x256
frames; 200 ragged frames up to 768x768) are checked on sampled frames.
"""
import numpy as np
import pytest

import p2s_synth as S
from oracle import basis as obasis
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def small_sim(p2s):
    """K = 16, P = 17 basis learned by the oracle; 33-64-64-16 network with bias."""
    wl = S.workload("single128")
    z, d = wl.basis_draws()
    B, _ = obasis.pca_basis(obasis.dataset(z, d, P=wl.P), wl.K)
    Ws, bs = wl.mlp(bias_scale=0.05)
    return p2s.Simulator(B, Ws, bs, n_zernike=35), B, Ws, bs


@pytest.fixture(scope="module")
def big_sim(p2s):
    """The K = 100, P = 33 basis shared by the batch workloads (package learner)."""
    from paper_2107_11627_amd import basis as pb
    wl = S.workload("batch256")
    z, d = wl.basis_draws()
    B, _ = pb.learn_basis(z, d, wl.K, wl.P)
    Ws, bs = wl.mlp()
    return p2s.Simulator(B, Ws, bs, n_zernike=wl.n_zernike)


SMALL_FRAMES = [(1, 64, 80), (3, 100, 37), (1, 128, 128), (2, 33, 200), (1, 7, 5), (1, 1, 1), (3, 48, 48)]


def small_batch():
    rng = np.random.default_rng(123)
    imgs = [S.blob_image(H, W, C, 900 + i, noise_std=0.01) for i, (C, H, W) in enumerate(SMALL_FRAMES)]
    d = [float(x) for x in rng.uniform(0.5, 5.0, len(imgs))]
    seeds = [int(x) for x in rng.integers(0, 2 ** 63, len(imgs))]
    return imgs, d, seeds


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_batch_equals_solo(p2s, small_sim, prec):
    sim = small_sim[0]
    imgs, d, seeds = small_batch()
    dimgs = [dev(im) for im in imgs]
    outs = sim.batch(dimgs, d, seeds, prec)
    for k, im in enumerate(dimgs):
        solo = host(sim(im, d[k], seeds[k], prec))
        got = host(outs[k])
        assert np.array_equal(got, solo), (k, SMALL_FRAMES[k], np.abs(got - solo).max())


def test_batch_512_sides_equal_solo(p2s, small_sim):
    """A frame with a 512-pixel side runs its field transforms on the fixed
    576-point plan when alone and on the runtime-sized passes inside a batch;
    both do the same arithmetic, so the frames agree bit for bit."""
    sim = small_sim[0]
    shapes = [(1, 512, 512), (3, 512, 72), (1, 40, 512)]
    imgs = [S.blob_image(H, W, C, 950 + i, noise_std=0.01) for i, (C, H, W) in enumerate(shapes)]
    d, seeds = [2.0, 1.0, 3.5], [31, 32, 33]
    dimgs = [dev(im) for im in imgs]
    for prec in ("fp32", "bf16"):
        outs = sim.batch(dimgs, d, seeds, prec)
        for k, im in enumerate(dimgs):
            solo = host(sim(im, d[k], seeds[k], prec))
            got = host(outs[k])
            assert np.array_equal(got, solo), (shapes[k], prec, np.abs(got - solo).max())


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_frame_vs_oracle(p2s, small_sim, prec):
    sim, B, Ws, bs = small_sim
    imgs, d, seeds = small_batch()
    outs = sim.batch([dev(im) for im in imgs], d, seeds, prec)
    k = 1                                           # 3 x 100 x 37, RGB and ragged
    ref = osimulate(imgs[k], d[k], B, Ws, bs, seed=seeds[k])["out"]
    assert rel_l2(host(outs[k]), ref) < (1e-5 if prec == "fp32" else 3e-3)


def test_batch_schedule_options(p2s, small_sim):
    """Persistent or one-workgroup-per-item, 16- or 8-row blur items: the same
    per-pixel arithmetic, so the same output."""
    sim = small_sim[0]
    imgs, d, seeds = small_batch()
    dimgs = [dev(im) for im in imgs]
    ref = [host(o) for o in sim.batch(dimgs, d, seeds, "bf16")]
    for rows, persistent in ((16, False), (8, True), (8, False)):
        b, outs = sim.plan(dimgs, d, seeds, "bf16", blur_tile_rows=rows, persistent=persistent)
        b.upload()
        b.launch()
        items, grid = b.info()
        assert all(g <= i for g, i in zip(grid, items))
        if not persistent:
            assert grid == items
        for k in range(len(imgs)):
            got = host(outs[k])
            if rows == 16:
                assert np.array_equal(got, ref[k])
            else:
                assert rel_l2(got, ref[k]) < 1e-6
        torch.cuda.synchronize()
        b.close()


def test_batch_graph_replay(p2s, small_sim):
    """p2s_batch_launch captured once into a HIP graph and replayed; eager work
    and synchronisation between replays; every replay equals the eager run."""
    sim = small_sim[0]
    imgs, d, seeds = small_batch()
    dimgs = [dev(im) for im in imgs]
    b, outs = sim.plan(dimgs, d, seeds, "bf16")
    b.upload()
    b.launch()
    ref = [host(o) for o in outs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            with pytest.raises(p2s.P2SError) as e:
                b.upload(stream=s)                  # copies are refused under capture
            assert e.value.code == p2s.P2S_EUNSUPPORTED
            b.launch(stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        for o in outs:
            o.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in range(len(outs)):
            assert np.array_equal(host(outs[k]), ref[k]), (rep, k)
    del g
    b.close()


def test_batch_empty_and_errors(p2s, small_sim):
    sim = small_sim[0]
    p2s.simulate_batch([], [], [], sim.basis, sim.net, "bf16", [], None)
    b = p2s.Batch([], [], [], [], sim.basis, sim.net, "fp32", None)
    b.upload()
    b.launch()
    assert b.info() == ([0] * 5, [0] * 5)
    b.close()
    imgs, d, seeds = small_batch()
    dimgs = [dev(im) for im in imgs[:3]]
    ws = sim.batch_workspace([tuple(t.shape) for t in dimgs])
    shared = torch.empty(4 * 128 * 128, device="cuda")
    outs = [shared[: t.numel()].view(t.shape) for t in dimgs]
    with pytest.raises(p2s.P2SError) as e:
        p2s.simulate_batch(dimgs, d[:3], seeds[:3], sim.basis, sim.net, "bf16", outs, ws)
    assert e.value.code == p2s.P2S_EINVAL and "overlap" in str(e.value)
    outs = [torch.empty_like(t) for t in dimgs]
    with pytest.raises(p2s.P2SError) as e:
        p2s.simulate_batch(dimgs, d[:3], seeds[:3], sim.basis, sim.net, "bf16", outs, ws[:4096])
    assert e.value.code == p2s.P2S_EINVAL and "workspace" in str(e.value)
    with pytest.raises(p2s.P2SError) as e:
        p2s.simulate_batch(dimgs, d[:3], seeds[:3], sim.basis, sim.net, 7, outs, ws)
    assert e.value.code == p2s.P2S_EINVAL
    with pytest.raises(p2s.P2SError) as e:
        p2s.Batch(dimgs, outs, d[:3], seeds[:3], sim.basis, sim.net, "bf16", ws, blur_tile_rows=12)
    assert e.value.code == p2s.P2S_EINVAL


def run_workload_sampled(p2s, sim, name, prec, sample):
    wl = S.workload(name)
    imgs = [dev(f.image()) for f in wl.frames]
    d = [f.d_over_r0 for f in wl.frames]
    seeds = [f.field_seed for f in wl.frames]
    b, outs = sim.plan(imgs, d, seeds, prec)
    b.upload()
    b.launch()
    torch.cuda.synchronize()
    for k in sample:
        solo = host(sim(imgs[k], d[k], seeds[k], prec))
        assert np.array_equal(host(outs[k]), solo), (name, k)
    for o in outs:
        assert bool(torch.isfinite(o).all())
    b.close()


def test_batch256_full_size_sampled(p2s, big_sim):
    run_workload_sampled(p2s, big_sim, "batch256", "bf16", [0, 17, 63])


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_ragged_full_size_sampled(p2s, big_sim, prec):
    wl = S.workload("ragged")
    big = max(range(len(wl.frames)), key=lambda i: wl.frames[i].H * wl.frames[i].W * wl.frames[i].C)
    run_workload_sampled(p2s, big_sim, "ragged", prec, [0, 1, 199, big])


def test_batch256_full_size_sampled_fp32(p2s, big_sim):
    """The FP32 batched kernels at the full 64-frame RGB 256x256 size."""
    run_workload_sampled(p2s, big_sim, "batch256", "fp32", [0, 31, 63])
