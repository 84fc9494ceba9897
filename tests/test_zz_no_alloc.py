"""The allocation-free entry point p2s_simulate_noalloc against p2s_simulate.

Both run the same kernels on the same inputs, so the frames must agree bit
for bit; two calls in a row (the second on a smaller frame, so that the
device scratch still holds the larger frame's intermediates) and every
precision.  The reference workspace is filled with NaN first, so neither side
can lean on zeroed memory.  A frame too large for the scratch is refused on
the host before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest

import p2s_synth as S
from oracle import basis as obasis

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def p2s():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2107_11627_amd import p2s as mod
    mod.lib()
    return mod


@pytest.fixture(scope="module")
def sim(p2s):
    wl = S.workload("single512")
    z, d = wl.basis_draws()
    basis, _ = obasis.pca_basis(obasis.dataset(z[:2048], d[:2048], P=wl.P), wl.K)
    Ws, bs = wl.mlp()
    return p2s.Simulator(basis, Ws, bs, n_zernike=wl.n_zernike)


def solo(p2s, sim, img, d, seed, prec):
    C_, H, W = img.shape
    ws = torch.full((p2s.workspace_bytes(C_, H, W, sim.n_zernike, sim.basis.K) // 4,), float("nan"),
                    dtype=torch.float32, device="cuda")
    out = torch.full_like(img, float("nan"))
    p2s.simulate(img, d, sim.basis, sim.net, seed, prec, out, ws, sim.n_zernike)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("prec", ["bf16", "fp32", "fp8"])
def test_noalloc_equals_simulate_two_calls(p2s, sim, prec):
    big = torch.from_numpy(S.blob_image(512, 512, 3, 41)).cuda()
    small = torch.from_numpy(S.blob_image(97, 130, 1, 42)).cuda()
    for img, d, seed in ((big, 3.0, 501), (small, 1.7, 502)):
        print(f"noalloc {prec} {tuple(img.shape)} seed {seed}", flush=True)
        out = torch.full_like(img, float("nan"))
        p2s.simulate_noalloc(img, d, sim.basis, sim.net, seed, prec, out, sim.n_zernike)
        torch.cuda.synchronize()
        ref = solo(p2s, sim, img, d, seed, prec)
        assert torch.isfinite(out).all()
        assert torch.equal(out, ref), (prec, tuple(img.shape))


def test_noalloc_rejects_frames_beyond_the_scratch(p2s, sim):
    lib = p2s.lib()
    img = torch.zeros((3, 2048, 2048), dtype=torch.float32, device="cuda")
    out = torch.full_like(img, 7.0)
    rc = lib.p2s_simulate_noalloc(C.c_void_p(img.data_ptr()), 3, 2048, 2048, 2.0, sim.n_zernike, sim.basis.handle,
                                  sim.net.handle, 1, p2s.BF16, None, C.c_void_p(out.data_ptr()), None)
    assert rc == p2s.P2S_EINVAL
    assert b"scratch" in lib.p2s_last_error()
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
