"""Pins of the oracle's anchor-grid field model (paper Sec. 3.4 with Noll's
R_Z of Sec. 2.2) against what the mathematics fixes.

Each test checks the oracle against something other than itself: a second
route to the same integral, an exact algebraic identity of the draw, or
exactness properties of bilinear interpolation.  The mistakes each is meant
to catch are noted per test.
"""
import math

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss
from scipy import integrate, special

from oracle import anchors, noll, philox, zernike


def _weber_schafheitlin_quadrature(n, nn, x_max=200.0):
    """int_0^inf x^(-14/3) J_{n+1}(x) J_{n'+1}(x) dx by adaptive quadrature
    over unit intervals (the tail beyond x_max is below 1e-10 of it)."""
    f = lambda x: x ** (-14.0 / 3.0) * special.jv(n + 1, x) * special.jv(nn + 1, x)
    total, a = 0.0, 0.0
    for b in np.arange(1.0, x_max + 1.0):
        v, _ = integrate.quad(f, a, b, limit=200, epsabs=0.0, epsrel=1e-12)
        total += v
        a = b
    return total


def test_mode_covariance_radial_part_matches_bessel_quadrature():
    """Noll's Fourier form gives C_jj' proportional to
    sqrt((n+1)(n'+1)) int x^(-14/3) J_{n+1} J_{n'+1} dx for every covarying
    pair; the closed form's Gamma ratio must match the quadrature relative to
    the tilt variance (catches a wrong Gamma argument, a dropped sqrt((n+1)
    (n'+1)) or a wrong exponent), modes 2..36."""
    C = anchors.mode_covariance(35)
    cache = {}
    for p in range(35):
        n, _ = zernike.noll_to_nm(p + 2)
        for q in range(35):
            if C[p, q] == 0.0:
                continue
            nn, _ = zernike.noll_to_nm(q + 2)
            key = (min(n, nn), max(n, nn))
            if key not in cache:
                cache[key] = _weber_schafheitlin_quadrature(*key)
            if (1, 1) not in cache:
                cache[(1, 1)] = _weber_schafheitlin_quadrature(1, 1)
            want = math.sqrt((n + 1) * (nn + 1)) * cache[key] / (2.0 * cache[(1, 1)]) * C[0, 0]
            assert abs(abs(C[p, q]) - abs(want)) <= 1e-5 * abs(want), (p + 2, q + 2)


def _real_space_covariance(n_planes, nr=32, nt=64):
    """-(1/2) int int Z_j(r) Z_j'(r') |r - r'|^(5/3) over the unit disk twice,
    by a polar Gauss rule: for piston-free modes this is the modal
    covariance of a phase with structure function |r - r'|^(5/3), up to one
    constant factor."""
    x, w = leggauss(nr)
    rho = 0.5 * (x + 1.0)
    wr = 0.5 * w * rho
    th = (np.arange(nt) + 0.5) * 2.0 * np.pi / nt
    R, T = np.meshgrid(rho, th, indexing="ij")
    wgt = np.outer(wr, np.full(nt, 2.0 * np.pi / nt)).ravel()
    R, T = R.ravel(), T.ravel()
    X, Y = R * np.cos(T), R * np.sin(T)
    Z = np.stack([zernike.zernike(j, R, T) for j in range(2, n_planes + 2)]) * wgt[None, :]
    D = np.hypot(X[:, None] - X[None, :], Y[:, None] - Y[None, :]) ** (5.0 / 3.0)
    return -0.5 * Z @ D @ Z.T


def test_mode_covariance_signs_and_selection_rules_real_space():
    """The real-space double integral of the 5/3 structure function fixes the
    sign of every cross term and which pairs vanish (m = m', same cos/sin
    parity) without Noll's Fourier algebra: correlation coefficients agree
    within 2e-3 (catches a wrong sign rule, a cos/sin pairing mistake or a
    missing cross term).  With Kolmogorov's D(r) = 6.8839 (r/r0)^(5/3) the
    integral also fixes the absolute tilt variance, which must match K of the
    Noll module within 0.5 %."""
    C = anchors.mode_covariance(35)
    M = _real_space_covariance(35)
    dc, dm = np.sqrt(np.diag(C)), np.sqrt(np.diag(M))
    rc, rm = C / np.outer(dc, dc), M / np.outer(dm, dm)
    assert np.max(np.abs(rc - rm)) < 2e-3
    assert np.all(np.abs(rm[rc == 0.0]) < 2e-3)
    big = np.abs(rc) > 0.01
    assert np.all(np.sign(rc[big]) == np.sign(rm[big]))
    # radius R = D/2: (|r|R / r0)^(5/3) = (D/r0)^(5/3) 2^(-5/3) |r|^(5/3); a_j = (1/pi) int phi Z_j.
    kolmogorov = 2.0 * ((24.0 / 5.0) * special.gamma(6.0 / 5.0)) ** (5.0 / 6.0)
    tilt = kolmogorov * 2.0 ** (-5.0 / 3.0) / np.pi ** 2 * M[0, 0]
    assert abs(tilt / C[0, 0] - 1.0) < 5e-3


def test_mode_covariance_diagonal_and_definiteness():
    """The diagonal is the Noll variance (pinned to Noll's table elsewhere)
    and the matrix is positive definite, so its Cholesky factor exists."""
    C = anchors.mode_covariance(35)
    assert np.allclose(np.diag(C), [noll.noll_variance(j) for j in range(2, 37)], rtol=1e-12, atol=0.0)
    assert np.allclose(C, C.T, rtol=0.0, atol=0.0)
    assert np.linalg.eigvalsh(C).min() > 0.0


def test_anchor_correlation_values_and_definiteness():
    """rho(0) = 1, rho(l) = 1/e, rho at a diagonal neighbour
    exp(-(sqrt 2 / l)^(5/3)); positive definite for several grids and
    lengths (catches a squared distance or a swapped index)."""
    R = anchors.anchor_correlation(5, 2.0)
    assert np.all(np.diag(R) == 1.0)
    assert R[0, 2] == pytest.approx(math.exp(-1.0), rel=1e-14)
    assert R[0, 6] == pytest.approx(math.exp(-(math.sqrt(2.0) / 2.0) ** (5.0 / 3.0)), rel=1e-14)
    assert R[3, 7] == pytest.approx(math.exp(-(math.sqrt(2.0) / 2.0) ** (5.0 / 3.0)), rel=1e-14)
    for G, l in ((4, 0.5), (9, 2.0), (16, 4.0)):
        assert np.linalg.eigvalsh(anchors.anchor_correlation(G, l)).min() > 0.0


def test_draw_has_the_kronecker_covariance():
    """A(E) is linear in the normals, so Cov(vec A) = sum over unit inputs of
    A(e) A(e)^T exactly; it must equal R_s[p, q] C_Z[i, k] (D/r0)^(5/3)
    (catches L_Z applied from the wrong side, a transposed factor, or a wrong
    power of D/r0)."""
    G, n, dr = 3, 10, 2.5
    rows = []
    for r in range(G * G):
        for c in range(n):
            E = np.zeros((G * G, n))
            E[r, c] = 1.0
            rows.append(anchors.anchor_coefficients(E, G, dr, 1.5).ravel())
    M = np.array(rows)
    cov = M.T @ M
    want = np.einsum("pq,ik->piqk", anchors.anchor_correlation(G, 1.5),
                     anchors.mode_covariance(n)).reshape(G * G * n, G * G * n) * dr ** (5.0 / 3.0)
    assert np.max(np.abs(cov - want)) < 1e-13


def test_anchor_normals_moments_and_stream():
    """Standard normal moments over 64 x 64 anchors x 36 planes; the cosine
    and sine of one Box-Muller pair are uncorrelated; a new seed gives new
    numbers; the draws differ from the frequency-domain noise of the same
    seed (catches a mapping to (0, 1] lost, or counter words reused)."""
    E = anchors.anchor_normals(64, 36, 7)
    z = E.ravel()
    N = z.size
    assert abs(z.mean()) < 4.0 / math.sqrt(N)
    assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / N)
    assert abs(np.mean(z ** 4) - 3.0) < 4.0 * math.sqrt(96.0 / N)
    assert abs(np.corrcoef(E[:, 0::2].ravel(), E[:, 1::2].ravel())[0, 1]) < 4.0 / math.sqrt(N / 2)
    assert np.all(anchors.anchor_normals(64, 36, 8) != E)
    assert np.all(np.isfinite(E))
    fb = philox.complex_normal_bins(64, 64, 0, 7)
    assert not np.allclose(fb.real.ravel()[:100], E[:100, 0])


def test_interpolation_exact_at_anchors():
    """Where an anchor falls on a pixel (H - 1 and W - 1 multiples of G - 1)
    the field equals the anchor value (catches an off-by-one cell or swapped
    axes)."""
    G, H, W = 5, 9, 13
    rng = np.random.default_rng(3)
    A = rng.standard_normal((G * G, 4))
    F = anchors.interpolate(A, G, H, W)
    V = A.T.reshape(4, G, G)
    assert np.array_equal(F[:, ::2, ::3], V)


def test_interpolation_reproduces_bilinear_functions():
    """Bilinear interpolation is exact for f = c0 + c1 y + c2 x + c3 y x of
    the pixel coordinates, on a ragged non-square image and for a single
    row (catches a wrong cell, a weight on the wrong corner, or swapped
    fractions)."""
    G = 7
    for H, W in ((37, 23), (1, 29), (19, 1), (2, 2)):
        sy = (H - 1) / (G - 1)
        sx = (W - 1) / (G - 1)
        a, b = np.divmod(np.arange(G * G), G)
        y, x = a * sy, b * sx
        c = np.array([0.3, -1.2, 0.7, 0.05])
        A = np.stack([c[0] + c[1] * y + c[2] * x + c[3] * y * x, -2.0 + 0.5 * x], axis=1)
        F = anchors.interpolate(A, G, H, W)
        Y, X = np.meshgrid(np.arange(H, dtype=float), np.arange(W, dtype=float), indexing="ij")
        if H == 1:
            Y = np.zeros_like(Y)
        if W == 1:
            X = np.zeros_like(X)
        assert np.allclose(F[0], c[0] + c[1] * Y + c[2] * X + c[3] * Y * X, rtol=0.0, atol=1e-12)
        assert np.allclose(F[1], -2.0 + 0.5 * X, rtol=0.0, atol=1e-12)


def test_make_fields_at_anchor_pixels_is_the_draw():
    """make_fields composes draw and interpolation: at anchor pixels the
    planes are A = L_s E L_Z^T (D/r0)^(5/6) of the seed's normals."""
    G, H, W = 9, 17, 25
    F = anchors.make_fields(H, W, 3.0, 12, 11, G=G, corr_len=2.0)
    A = anchors.anchor_coefficients(anchors.anchor_normals(G, 12, 11), G, 3.0, 2.0)
    assert np.allclose(F[:, ::2, ::3], A.T.reshape(12, G, G), rtol=0.0, atol=1e-14)
    with pytest.raises(ValueError):
        anchors.make_fields(4, 4, 1.0, 3, 0, G=1)
