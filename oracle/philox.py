"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11) and the Box-Muller
normals the field generator draws from it.

Philox4x32: each of the 10 rounds multiplies words 0 and 2 of the counter by
two fixed 32-bit multipliers, and the new counter is
(hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, lo(M0*x0)); between
rounds the key is advanced by the two Weyl constants.

Noise layout (a reading; the paper does not fix a generator): the field
generator draws its white noise directly in the frequency domain.  Bin
(ky, kx) of plane pair q under frame seed s uses key (s mod 2^32, s >> 32) and
counter (kx, ky, q, 0); from outputs o0, o1, with u_a = ((o0 >> 8) + 1) 2^-24
in (0, 1] and u_b = (o1 >> 8) 2^-24 in [0, 1), the bin's complex normal is
sqrt(-2 ln u_a) (cos(2 pi u_b) + i sin(2 pi u_b)) -- a Box-Muller pair, so
real and imaginary parts are independent N(0, 1).  Outputs o2, o3 are unused.

Parity: pinned by published known-answer vectors of Philox4x32-10 and by
moment tests of the normals.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Vectorised Philox4x32-10 over broadcastable uint32 counter words."""
    x0, x1, x2, x3 = (np.asarray(v, dtype=np.uint64) & MASK for v in (c0, c1, c2, c3))
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    ka, kb = k0 & 0xFFFFFFFF, k1 & 0xFFFFFFFF
    for _ in range(10):
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        x0, x1, x2, x3 = hi1 ^ x1 ^ np.uint64(ka), lo1, hi0 ^ x3 ^ np.uint64(kb), lo0
        ka = (ka + W0) & 0xFFFFFFFF
        kb = (kb + W1) & 0xFFFFFFFF
    return tuple(v.astype(np.uint32) for v in (x0, x1, x2, x3))


def raw_bins(Nfy: int, Nfx: int, pair: int, seed: int):
    """The four Philox outputs of counter (kx, ky, pair, 0) for every bin:
    array [Nfy][Nfx][4] of uint32."""
    ky = np.arange(Nfy, dtype=np.uint64)[:, None]
    kx = np.arange(Nfx, dtype=np.uint64)[None, :]
    o = philox4x32_10(kx, ky, np.uint64(pair), np.uint64(0), seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return np.stack(o, axis=-1)


def complex_normal_bins(Nfy: int, Nfx: int, pair: int, seed: int) -> np.ndarray:
    """Complex white noise [Nfy][Nfx] (complex128): real and imaginary parts
    are independent standard normals."""
    raw = raw_bins(Nfy, Nfx, pair, seed)
    ua = (np.floor(raw[..., 0].astype(np.float64) / 256.0) + 1.0) * 2.0 ** -24
    ub = np.floor(raw[..., 1].astype(np.float64) / 256.0) * 2.0 ** -24
    rad = np.sqrt(-2.0 * np.log(ua))
    return rad * np.cos(2.0 * np.pi * ub) + 1j * rad * np.sin(2.0 * np.pi * ub)
