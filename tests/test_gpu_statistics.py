"""Statistical validation on the GPU path (paper Sec. 4.1) against the
oracle's statistics of the same model.

Evaluation 1 (tilt): the mean lag products of the tilt planes the field
generators produce, against the covariance their model fixes (the periodic
covariance of the Gaussian PSD; the interpolated anchor covariance), and the
tilt displacement variance against the Kolmogorov Z-tilt.  Sampling error: a
512^2 plane with a correlation length of about 16 pixels holds a few hundred
independent patches, so 2 planes x 48 frames estimate a covariance to about
0.5 % of the variance (rms; measured errors 0.003-0.006); the 256^2 anchor
frames with 8-pixel cells, 64 of them, to about 1 % (measured 0.009-0.014).
Bounds: 0.03 and 0.04, and 3 % on the displacement variance.

Evaluation 2 (exposures): point sources through the whole simulator (trained
network, BF16) against the oracle's model of the same point source with the
exact PSF in place of the network.  Both sides are Monte Carlo estimates of
4096 realisations; the measured differences are at most 0.004 at every
frequency (the network's error on the basis coefficients averages out in the
MTFs); bound 0.02.
"""
import numpy as np
import pytest

import p2s_synth as S
from oracle import basis as obasis
from oracle import statistics as ostat

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U = [0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8]


@pytest.fixture(scope="module")
def mods():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2107_11627_amd import anchors, p2s, validate
    p2s.lib()
    return p2s, anchors, validate


def test_tilt_statistics_fft_model(mods):
    p2s, _, validate = mods
    lags = list(range(0, 49, 4))
    r = validate.tilt_statistics(512, 512, 3.0, 48, lags)
    want = ostat.fft_model_correlation(512, lags)
    ex = np.max(np.abs(np.array(r["cov_along_x"]) - want))
    ey = np.max(np.abs(np.array(r["cov_along_y"]) - want))
    sv = r["shift_variance_px2"] / ostat.tilt_shift_variance(3.0)
    print(f"FFT tilt covariance: max |err| along x {ex:.3f}, along y {ey:.3f}; shift variance ratio {sv:.3f}")
    assert ex < 0.03 and ey < 0.03
    assert abs(sv - 1.0) < 0.03


def test_tilt_statistics_anchor_model(mods):
    p2s, anchors, validate = mods
    G, H, W = 32, 256, 256
    model = anchors.anchor_model(G, 35, 2.0)
    lags = list(range(0, 33, 4))
    r = validate.tilt_statistics(H, W, 3.0, 64, lags, anchors=model)
    wx = ostat.anchor_model_covariance(G, H, W, lags, 1, 2.0)
    wy = ostat.anchor_model_covariance(G, H, W, lags, 0, 2.0)
    ex = np.max(np.abs(np.array(r["cov_along_x"]) - wx))
    ey = np.max(np.abs(np.array(r["cov_along_y"]) - wy))
    print(f"anchor tilt covariance: max |err| along x {ex:.3f}, along y {ey:.3f}")
    assert ex < 0.04 and ey < 0.04


def test_exposure_mtfs_match_the_model(mods):
    p2s, _, validate = mods
    from paper_2107_11627_amd import train as ptrain
    wl = S.workload("single512")
    z, d = wl.basis_draws()
    basis, _ = obasis.pca_basis(obasis.dataset(z, d, P=wl.P), wl.K)
    Ws, bs, _ = ptrain.load("p2s_single512", basis)
    sim = p2s.Simulator(basis, Ws, bs, n_zernike=wl.n_zernike)
    r = validate.exposure_statistics(sim, 3.0, 64, U)
    le, se = ostat.simulator_model_mtfs(3.0, 4096, 9, U)
    gl, gs = np.array(r["long_exposure_mtf"]), np.array(r["short_exposure_mtf"])
    print("u       " + " ".join(f"{u:6.2f}" for u in U))
    print("LE gpu  " + " ".join(f"{v:6.3f}" for v in gl))
    print("LE model" + " ".join(f"{v:6.3f}" for v in le))
    print("SE gpu  " + " ".join(f"{v:6.3f}" for v in gs))
    print("SE model" + " ".join(f"{v:6.3f}" for v in se))
    assert np.max(np.abs(gl - le)) < 0.02
    assert np.max(np.abs(gs - se)) < 0.02
