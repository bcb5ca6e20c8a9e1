"""SplitMix64 as a counter-based generator, and the sketch draws built on it.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014; the 64-bit finalizer published with it): the state
advances by the golden-ratio increment GAMMA and each output is the state
passed through two xor-shift-multiply rounds.  The i-th output (0-based) of
a generator whose state starts at ``key`` is therefore mix(key + (i+1)*GAMMA),
a pure function of (key, i): that is the counter-based form used here, so any
draw can be made independently of the others.

Draw conventions (shared with the GPU path as a written specification, not
as code):

* stream keys: key_t = output t of SplitMix64(seed), t = 0, 1, 2, 3;
* CountSketch / SJLT row i, block b (Section 4, bullets 2-3):
  x = draw(key_0, i*s + b); bucket = b*(m/s) + ((x >> 32) * (m/s)) >> 32;
  sign = +1 if bit 0 of x is 0 else -1;
* SRHT diagonal sign of row i: bit 0 of draw(key_1, i) (0 -> +1);
* SRHT sampled row k (with replacement): ((draw(key_2, k) >> 32) * n') >> 32;
* Gaussian entries by Box-Muller pairs (Box and Muller, 1958): pair p gives
  u1 = ((draw(key_3, 2p) >> 11) + 1) * 2^-53, u2 = (draw(key_3, 2p+1) >> 11)
  * 2^-53, and the two independent N(0, 1) values z_{2p} = rho cos(2 pi u2),
  z_{2p+1} = rho sin(2 pi u2), rho = sqrt(-2 ln u1); entry q = r*n + i of the
  m x n sketch is z_q / sqrt(m).
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_C1 = np.uint64(0xBF58476D1CE4E5B9)
_C2 = np.uint64(0x94D049BB133111EB)
_S30, _S27, _S31 = np.uint64(30), np.uint64(27), np.uint64(31)


def mix(z):
    """The SplitMix64 output function applied to a uint64 array (wrapping)."""
    z = np.asarray(z, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = (z ^ (z >> _S30)) * _C1
        z = (z ^ (z >> _S27)) * _C2
    return z ^ (z >> _S31)


def draw(key, i):
    """Output i (0-based) of SplitMix64 started at state ``key``."""
    i = np.asarray(i, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix(np.uint64(key) + (i + np.uint64(1)) * GAMMA)


def stream_key(seed: int, t: int) -> np.uint64:
    return np.uint64(draw(np.uint64(seed), np.uint64(t)))


def range32(x, bound: int):
    """Multiply-shift reduction of the top 32 bits of x into [0, bound)."""
    hi = np.asarray(x, dtype=np.uint64) >> np.uint64(32)
    with np.errstate(over="ignore"):
        return ((hi * np.uint64(bound)) >> np.uint64(32)).astype(np.int64)


def sign_bit(x):
    """+1 when bit 0 of x is clear, -1 when it is set."""
    return (1 - 2 * (np.asarray(x, dtype=np.uint64) & np.uint64(1)).astype(np.int64)).astype(np.int8)


def countsketch_draws(seed: int, n: int, m: int, s: int = 1):
    """Buckets int32[n, s] and signs int8[n, s] of an SJLT with s blocks.

    s = 1 is CountSketch.  Block b owns rows [b*m/s, (b+1)*m/s) of S.
    """
    if m % s:
        raise ValueError("m must be a multiple of s")
    key = stream_key(seed, 0)
    ctr = (np.arange(n, dtype=np.uint64)[:, None] * np.uint64(s)
           + np.arange(s, dtype=np.uint64)[None, :])
    x = draw(key, ctr)
    mb = m // s
    h = (np.arange(s, dtype=np.int64)[None, :] * mb + range32(x, mb)).astype(np.int32)
    return h, sign_bit(x)


def srht_draws(seed: int, n: int, m: int):
    """(signs int8[n], rows int32[m] in [0, n')) with n' = 2^ceil(log2 n)."""
    npad = 1 << max(0, int(n - 1).bit_length())
    signs = sign_bit(draw(stream_key(seed, 1), np.arange(n, dtype=np.uint64)))
    rows = range32(draw(stream_key(seed, 2), np.arange(m, dtype=np.uint64)), npad)
    return signs, rows.astype(np.int32), npad


def gaussian_draws(seed: int, m: int, n: int) -> np.ndarray:
    """The N(0, 1) draws z (m x n, float64) of the Gaussian sketch: entry q =
    r * n + k is the cosine (q even) or sine (q odd) value of Box-Muller
    pair q // 2, made from draws (2p, 2p + 1) of the stream."""
    key = stream_key(seed, 3)
    total = m * n
    p = np.arange((total + 1) // 2, dtype=np.uint64)
    x1 = draw(key, p * np.uint64(2))
    x2 = draw(key, p * np.uint64(2) + np.uint64(1))
    u1 = ((x1 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (x2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    rho = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * p.size)
    z[0::2] = rho * np.cos(2.0 * np.pi * u2)
    z[1::2] = rho * np.sin(2.0 * np.pi * u2)
    return z[:total].reshape(m, n)


def gaussian_matrix(seed: int, m: int, n: int) -> np.ndarray:
    """Dense S (m x n) with entries N(0, 1/m) by Box-Muller, float64."""
    return gaussian_draws(seed, m, n) / np.sqrt(m)


def round_bf16(x) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), through FP32 first:
    BF16(FP32(x)), returned as float64.  BF16 keeps the top 16 bits of an FP32
    number; rounding adds 0x7FFF plus the lowest kept bit before truncating."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gaussian_matrix_bf16(seed: int, m: int, n: int) -> np.ndarray:
    """The BF16 Gaussian sketch: BF16(FP32(z)) / sqrt(m) of the same draws."""
    return round_bf16(gaussian_draws(seed, m, n)) / np.sqrt(m)


def e4m3_values() -> np.ndarray:
    """The finite nonnegative values of the OCP FP8 e4m3 format (e4m3fn), by
    code 0..126: code = 8 e + f with 3 fraction bits f; e = 0 holds the
    subnormals f 2^-9, e >= 1 the normals (1 + f/8) 2^(e-7); code 127 is NaN
    (no infinities), so the largest value is 1.75 * 2^8 = 448."""
    e, f = np.divmod(np.arange(127), 8)
    return np.where(e == 0, f * 2.0 ** -9, (1.0 + f / 8.0) * 2.0 ** (e - 7.0))


def round_e4m3(x) -> np.ndarray:
    """Round to the nearest e4m3 value through FP32 first, E4M3(FP32(x)): ties
    to the even code, magnitudes beyond 448 saturate to 448.  Returned as
    float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    a = np.minimum(np.abs(f), 448.0)
    vals = e4m3_values()
    hi = np.clip(np.searchsorted(vals, a, side="left"), 1, 126)  # vals[hi-1] < a <= vals[hi]
    lo = hi - 1
    dlo, dhi = a - vals[lo], vals[hi] - a
    pick = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi, np.where(lo % 2 == 0, lo, hi)))
    return np.copysign(vals[pick], f)


def gaussian_matrix_fp8(seed: int, m: int, n: int) -> np.ndarray:
    """The FP8 Gaussian sketch: E4M3(FP32(z)) / sqrt(m) of the same draws."""
    return round_e4m3(gaussian_draws(seed, m, n)) / np.sqrt(m)
