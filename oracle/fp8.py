"""FP8 E4M3 form of the fused blur (the precision variant of Sec. 3.1's
basis blur): the image and the basis enter the convolutions as OCP FP8 E4M3
values, each basis function with a power-of-two scale of its own; the
weighted sum over the basis and everything else stay exact here.

E4M3 (OCP 8-bit floating point, "fn" variant): 1 sign, 4 exponent (bias 7)
and 3 mantissa bits; normal values 2^-6 .. 448, subnormal spacing 2^-9, no
infinities.  Rounding is to nearest, ties to even.

Readings recorded with the design notes:
  * the image is quantised as given (no scale), after clamping to +-448;
  * basis function k is multiplied by 2^e_k before quantisation, e_k the
    largest integer with max_u |phi_k(u)| 2^e_k <= 448 (taken from the
    float32 copy of the basis), and divided by it again after;
  * both operands are rounded from their float32 values.

TEST INFRASTRUCTURE: only tests, the smoke check and the CPU baseline use
this package.  Parity: pinned (rounding against torch's independent
float8_e4m3fn cast; every E4M3 value is a fixed point; scale exponents
against their defining inequality; representable operands reduce to the
plain basis blur).
"""
import numpy as np

from .blur import basis_blur

E4M3_MAX = 448.0
E4M3_MIN_NORMAL = 2.0 ** -6
E4M3_SUB_STEP = 2.0 ** -9


def e4m3_round(x) -> np.ndarray:
    """Nearest E4M3 value (ties to even) of float32 inputs, as float64;
    inputs are clamped to +-448 first."""
    a = np.asarray(x, dtype=np.float32).astype(np.float64)
    a = np.clip(a, -E4M3_MAX, E4M3_MAX)
    mag = np.abs(a)
    _, e = np.frexp(mag)                     # mag = f 2^e, f in [0.5, 1)
    quantum = np.where(mag >= E4M3_MIN_NORMAL, np.ldexp(1.0, e - 4), E4M3_SUB_STEP)   # 3 mantissa bits
    r = np.rint(mag / quantum) * quantum     # rint: half to even; division by 2^n is exact
    return np.copysign(np.minimum(r, E4M3_MAX), a)


def scale_exponent(amax: float) -> int:
    """Largest e with amax * 2^e <= 448 (0 for amax = 0), limited to +-127."""
    amax = float(amax)
    if amax == 0.0:
        return 0
    f, E = np.frexp(amax)                    # amax = f 2^E, 448 = 0.875 * 2^9
    e = (9 - E) if f <= 0.875 else (8 - E)
    return int(min(127, max(-127, e)))


def quantize_basis(basis: np.ndarray):
    """Dequantised FP8 basis [K][P][P] (float64) and the exponents e_k."""
    b32 = np.asarray(basis, dtype=np.float32).astype(np.float64)
    K = b32.shape[0]
    out = np.empty_like(b32)
    ex = np.empty(K, dtype=np.int64)
    for k in range(K):
        e = scale_exponent(np.max(np.abs(b32[k])))
        out[k] = e4m3_round(np.ldexp(b32[k], e)) * 2.0 ** (-e)
        ex[k] = e
    return out, ex


def quantize_image(image: np.ndarray) -> np.ndarray:
    return e4m3_round(image)


def fp8_blur(image: np.ndarray, basis: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Eq. 5 on E4M3 operands: sum_k w_k(x) (q(phi_k) conv q(I))(x), one
    channel [H][W]."""
    qb, _ = quantize_basis(basis)
    return basis_blur(quantize_image(image), qb, w)
