"""OCP FP8 e4m3 ("E4M3FN"): 1 sign, 4 exponent (bias 7), 3 mantissa bits; no
infinities, S.1111.111 is NaN, largest finite 448, smallest subnormal 2^-9.
Plain numpy encoder/decoder written from that definition, and the block
quantisation the FP8 form of the products uses (test infrastructure)."""
import numpy as np


def decode(codes):
    c = np.asarray(codes, dtype=np.int64)
    s = np.where(c >> 7, -1.0, 1.0)
    e = (c >> 3) & 15
    mant = (c & 7).astype(np.float64)
    val = np.where(e == 0, np.ldexp(mant / 8.0, -6), np.ldexp(1.0 + mant / 8.0, e - 7))
    val = np.where((e == 15) & ((c & 7) == 7), np.nan, val)
    return s * val


def round_e4m3(x):
    """Nearest e4m3 value to x (ties to even), for |x| <= 448, as float64."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -6.0)                   # subnormal range shares the 2^-9 spacing
    quantum = np.ldexp(1.0, (e - 3).astype(np.int64))
    q = np.round(a / quantum) * quantum       # numpy rounds half to even
    return np.sign(x) * q


def pow2_scale(amax):
    """2^ceil(log2(amax / 448)), at least 2^-126 (the smallest scale the FP8
    matrix-core instruction's E8M0 byte takes from a normal FP32 value); 1 for
    amax == 0."""
    amax = np.asarray(amax, dtype=np.float64)
    r = np.where(amax > 0, amax / 448.0, 1.0)
    e = np.maximum(np.ceil(np.log2(r)), -126.0).astype(np.int64)
    return np.where(amax > 0, np.ldexp(1.0, e), 1.0)


def quantize_blocks(A, b=64):
    """A (float32 values) -> (dequantised FP8 values, scales) with one scale per
    b x b block; the division by the power-of-two scale is exact."""
    A = np.asarray(A, dtype=np.float32).astype(np.float64)
    m, n = A.shape
    out = np.empty_like(A)
    scales = np.empty(((m + b - 1) // b, (n + b - 1) // b))
    for ib in range(scales.shape[0]):
        for jb in range(scales.shape[1]):
            blk = A[ib * b:(ib + 1) * b, jb * b:(jb + 1) * b]
            s = float(pow2_scale(np.max(np.abs(blk))))
            scales[ib, jb] = s
            out[ib * b:(ib + 1) * b, jb * b:(jb + 1) * b] = round_e4m3(blk / s) * s
    return out, scales


def quantize_columns(X):
    """Panel (rows x cols) -> dequantised FP8 values with one scale per column."""
    X = np.asarray(X, dtype=np.float32).astype(np.float64)
    s = pow2_scale(np.max(np.abs(X), axis=0))
    return round_e4m3(X / s[None, :]) * s[None, :], s
