"""CPU tests of the C-ABI library: it loads, exports every function the public
header declares, its host-side arithmetic agrees with the oracle, and argument
validation rejects bad calls before touching a device (so these run without a
GPU)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from oracle import basis as obasis
from oracle import fields as ofields
from oracle import noll as onoll

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "p2s.h")


@pytest.fixture(scope="module")
def p2s():
    from paper_2107_11627_amd import p2s as mod
    mod.lib()
    return mod


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(p2s_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_function(p2s):
    names = declared_functions()
    assert len(names) >= 18
    lib = p2s.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(p2s.EXPORTS)
    assert p2s.version() == 1


def test_noll_variance_matches_oracle(p2s):
    for j in range(2, 66):
        assert abs(p2s.noll_variance(j) - onoll.noll_variance(j)) < 1e-12 * onoll.noll_variance(j)
    with pytest.raises(p2s.P2SError):
        p2s.noll_variance(1)


def test_field_grid_matches_oracle(p2s):
    for n in (1, 2, 7, 64, 100, 128, 192, 255, 256, 320, 384, 512, 768, 1000, 1024, 2048):
        for ell in (1.0, 4.0, 16.0, 2.5):
            assert p2s.field_grid(n, ell) == ofields.grid_size(n, ell), (n, ell)


def test_workspace_sizes(p2s):
    nf = p2s.field_grid(512)
    # band of the Gaussian filter kept by the generator: exp(-pi^2 l^2 (k/N)^2) >= 1e-9
    kc = max(k for k in range(nf // 2 + 1) if k == 0 or math.exp(-(math.pi * 16.0 * k / nf) ** 2) >= 1e-9)
    mx = min(nf, 2 * kc + 1)
    assert kc == 52 and mx == 105
    v = (18 * 512 * mx + nf) * 8
    assert p2s.fields_workspace_bytes(512, 512, 35) == ((v + 255) // 256) * 256
    ws = p2s.workspace_bytes(1, 512, 512, 35, 100)
    need = 35 * 512 * 512 * 4 + max(v, 512 * 512 * 100 * 4) + 512 * 512 * 4
    assert need <= ws <= need + 3 * 256
    assert p2s.workspace_bytes(0, 512, 512, 35, 100) == 0
    assert p2s.workspace_bytes(1, 512, 512, 35, 200) == 0


def test_batch_workspace_sizes(p2s):
    shapes = [(1, 512, 512), (3, 128, 100), (2, 1, 1)]
    per = sum(p2s.workspace_bytes(c, h, w, 35, 100) for c, h, w in shapes)
    got = p2s.batch_workspace_bytes(shapes, 35, 100)
    plan = got - per                    # frame table + per-stage prefix sums, 256-byte pieces
    assert 0 < plan and plan % 256 == 0 and plan <= 3 * 2048 + 256
    assert p2s.batch_workspace_bytes([], 35, 100) == 0
    assert p2s.batch_workspace_bytes([(5, 8, 8)], 35, 100) == 0
    assert p2s.batch_workspace_bytes([(1, 8, 8)], 35, 200) == 0


def test_batch_validation_without_device(p2s):
    lib = p2s.lib()
    vp = C.c_void_p
    h = vp()
    fr = (p2s.Frame * 1)(p2s.Frame(vp(0x1000), vp(0x2000), 1, 8, 8, 1.0, 0))
    assert lib.p2s_batch_create(fr, 1, 35, None, None, 1, None, None, vp(0x9000), 1 << 30, C.byref(h)) == p2s.P2S_EINVAL
    assert b"basis" in lib.p2s_last_error()
    assert lib.p2s_batch_create(fr, 1, 35, vp(1), vp(1), 1, None, None, vp(0x9000), 1 << 30, None) == p2s.P2S_EINVAL
    for name in ("p2s_batch_upload", "p2s_batch_launch"):
        assert getattr(lib, name)(None, None) == p2s.P2S_EINVAL
    assert lib.p2s_batch_info(None, None, None) == p2s.P2S_EINVAL
    assert lib.p2s_batch_destroy(None) == p2s.P2S_OK
    assert lib.p2s_simulate_batch(fr, 1, 35, None, None, 1, None, vp(0x9000), 1 << 30, None) == p2s.P2S_EINVAL


def test_validation_without_device(p2s):
    """Every check below fails before any HIP call, so no GPU is needed."""
    lib = p2s.lib()
    vp = C.c_void_p
    fake = vp(0x1000)
    # blur with a NULL basis handle
    assert lib.p2s_blur(fake, 1, 8, 8, None, fake, 0, fake, None) == p2s.P2S_EINVAL
    assert b"basis" in lib.p2s_last_error()
    # warp: bad sizes, overlapping buffers
    assert lib.p2s_warp(fake, 0, 8, 8, fake, None, vp(0x2000), None) == p2s.P2S_EINVAL
    assert lib.p2s_warp(fake, 1, 8, 8, vp(0x9000), None, vp(0x1010), None) == p2s.P2S_EINVAL
    assert b"overlap" in lib.p2s_last_error()
    # make_fields: negative D/r0, too many planes, small workspace
    assert lib.p2s_make_fields(8, 8, -1.0, 35, 1, None, fake, fake, 1 << 30, None) == p2s.P2S_EINVAL
    assert lib.p2s_make_fields(8, 8, 1.0, 65, 1, None, fake, fake, 1 << 30, None) == p2s.P2S_EINVAL
    assert lib.p2s_make_fields(8, 8, 1.0, 35, 1, None, fake, fake, 16, None) == p2s.P2S_EINVAL
    assert b"workspace" in lib.p2s_last_error()
    bad = p2s.Params(0.0, 2.0)
    assert lib.p2s_make_fields(8, 8, 1.0, 35, 1, C.byref(bad), fake, fake, 1 << 30, None) == p2s.P2S_EINVAL
    # noise grid too large for the single-workgroup FFT
    assert lib.p2s_make_fields(16000, 8, 1.0, 35, 1, None, fake, fake, 1 << 40, None) == p2s.P2S_EUNSUPPORTED
    # handles: even P, K too large, NULL weights
    h = vp()
    b = np.zeros((4, 6, 6))
    assert lib.p2s_basis_create(b.ctypes.data_as(vp), 4, 6, C.byref(h)) == p2s.P2S_EINVAL
    b = np.zeros((200, 5, 5))
    assert lib.p2s_basis_create(b.ctypes.data_as(vp), 200, 5, C.byref(h)) == p2s.P2S_EINVAL
    b = np.full((2, 5, 5), np.nan)
    assert lib.p2s_basis_create(b.ctypes.data_as(vp), 2, 5, C.byref(h)) == p2s.P2S_EINVAL
    dims = (C.c_int * 3)(33, 200, 16)
    W = (vp * 2)(fake, fake)
    assert lib.p2s_mlp_create(2, dims, W, None, C.byref(h)) == p2s.P2S_EINVAL
    dims = (C.c_int * 3)(70, 20, 16)
    assert lib.p2s_mlp_create(2, dims, W, None, C.byref(h)) == p2s.P2S_EINVAL
    # simulate with NULL handles
    assert lib.p2s_simulate(fake, 1, 8, 8, 1.0, 35, None, None, 1, 0, None, fake, fake, 1 << 30, None) == p2s.P2S_EINVAL
    # noise hook with a NULL buffer
    assert lib.p2s_debug_noise(4, 4, 0, 1, None, None, None) == p2s.P2S_EINVAL


def test_product_basis_learner_matches_oracle():
    """The package's one-time basis learner and the oracle's are independent
    implementations of Sec. 3.2 (Zernike via Jacobi polynomials vs the
    factorial sum; PCA via SVD vs eigh); on the same draws they agree."""
    from paper_2107_11627_amd import basis as pb
    z = np.random.default_rng(5).standard_normal((600, 33))
    d = np.random.default_rng(6).uniform(0.5, 4.0, 600)
    Bp, ep = pb.learn_basis(z, d, 12, 17)
    Bo, eo = obasis.pca_basis(obasis.dataset(z, d, P=17), 12)
    np.testing.assert_allclose(ep, eo, rtol=1e-10, atol=1e-16)
    gaps = np.abs(np.diff(eo)) / eo[0]
    for k in range(12):
        if (k == 0 or gaps[k - 1] > 1e-6) and (k == 11 or gaps[k] > 1e-6):
            np.testing.assert_allclose(Bp[k], Bo[k], atol=1e-9)


def test_anchor_validation_without_device(p2s):
    """p2s_anchor_create rejects a bad grid, a bad mode count and non-finite
    factor entries before any device allocation; NULL handles are refused by
    the compute calls; the workspace queries return 0 for NULL."""
    lib = p2s.lib()
    G, n = 3, 5
    Ls = np.eye(G * G)
    Lz = np.eye(n)
    h = C.c_void_p()
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    for g in (1, 0, 129):
        assert lib.p2s_anchor_create(g, n, ptr(np.eye(max(g, 1) ** 2)), ptr(Lz), C.byref(h)) == p2s.P2S_EINVAL
    for nz in (0, 65):
        assert lib.p2s_anchor_create(G, nz, ptr(Ls), ptr(np.eye(max(nz, 1))), C.byref(h)) == p2s.P2S_EINVAL
    bad = Ls.copy()
    bad[4, 2] = np.nan
    assert lib.p2s_anchor_create(G, n, ptr(bad), ptr(Lz), C.byref(h)) == p2s.P2S_EINVAL
    assert b"not finite" in lib.p2s_last_error()
    bad = Ls.copy()
    bad[2, 4] = np.nan                     # above the diagonal: ignored, so only the next check fails
    badz = Lz.copy()
    badz[3, 1] = np.inf
    assert lib.p2s_anchor_create(G, n, ptr(bad), ptr(badz), C.byref(h)) == p2s.P2S_EINVAL
    assert b"mode factor" in lib.p2s_last_error()
    assert lib.p2s_anchor_create(G, n, None, ptr(Lz), C.byref(h)) == p2s.P2S_EINVAL
    assert lib.p2s_make_fields_anchor(None, 8, 8, 1.0, 0, None, None, 0, None) == p2s.P2S_EINVAL
    assert lib.p2s_simulate_anchor(None, 1, 8, 8, 1.0, None, None, None, 0, 0, None, None, None, 0,
                                   None) == p2s.P2S_EINVAL
    assert lib.p2s_anchor_fields_workspace_bytes(None) == 0
    assert lib.p2s_workspace_bytes_anchor(None, 1, 8, 8, 16) == 0
    assert lib.p2s_anchor_destroy(None) == p2s.P2S_OK


def test_product_anchor_setup_matches_oracle():
    """The product's set-up of the anchor model (its own Noll indexing,
    covariance and correlation code) equals the oracle's matrices."""
    from oracle import anchors as oanch
    from oracle import zernike as ozern
    from paper_2107_11627_amd import anchors as panch
    assert all(panch._noll_nm(j) == ozern.noll_to_nm(j) for j in range(1, 500))
    for n in (1, 10, 35, 64):
        a, b = panch.mode_covariance(n), oanch.mode_covariance(n)
        assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))
    for G, l in ((2, 1.0), (7, 2.0), (12, 3.5)):
        assert np.max(np.abs(panch.anchor_correlation(G, l) - oanch.anchor_correlation(G, l))) < 1e-15


def test_product_psf_dataset_any_wavelength_matches_oracle():
    """The package's PSF dataset at a non-integer sampling and a scaled phase
    (another wavelength than the reference) equals the oracle's: the
    package's direct Fourier sum against the oracle's psf_from_phase_q."""
    from paper_2107_11627_amd import basis as pb
    z = np.random.default_rng(8).standard_normal((40, 33))
    d = np.random.default_rng(9).uniform(1.0, 4.0, 40)
    for q, s in ((2.0 * 450 / 525, 525 / 450), (2.0 * 570 / 525, 525 / 570)):
        a = pb.psf_dataset(z, d, 17, 35, Q=q, phase_scale=s)
        b = obasis.dataset(z, d, P=17, Q=q, phase_scale=s)
        assert np.max(np.abs(a - b)) < 1e-12


def test_spectral_validation_without_device(p2s):
    """p2s_simulate_spectral rejects NULL handle arrays, a bad channel count and
    a bad mode count before touching a device."""
    lib = p2s.lib()
    assert lib.p2s_simulate_spectral(None, 3, 8, 8, 1.0, 35, None, None, 0, 1, None, None, None, 0,
                                     None) == p2s.P2S_EINVAL
    assert lib.p2s_simulate_spectral(None, 0, 8, 8, 1.0, 35, None, None, 0, 1, None, None, None, 0,
                                     None) == p2s.P2S_EINVAL
    nulls = (C.c_void_p * 3)(None, None, None)
    assert lib.p2s_simulate_spectral(None, 3, 8, 8, 1.0, 35, nulls, nulls, 0, 1, None, None, None, 0,
                                     None) == p2s.P2S_EINVAL
    assert b"channel 0" in lib.p2s_last_error()
    assert lib.p2s_simulate_spectral(None, 3, 8, 8, 1.0, 2, nulls, nulls, 0, 1, None, None, None, 0,
                                     None) == p2s.P2S_EINVAL
