"""Random sketches for GN, built on the CPU from their definitions (NumPy).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper asks for Gaussian sketches with i.i.d. zero-mean, unit-variance entries
(Section 3.1, the Marchenko-Pastur discussion) and names the SRHT as a structured
alternative (Section 1; Section 3.5.1 notes Gaussianity is not essential).  It does
not fix a random number generator, so both sides of the parity tests implement the
same published counter-based generator, Philox4x32-10 (Salmon, Moraes, Dror and
Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), each from that
definition.  Everything below the generator (the counter layout, the Gaussian
transform, the SRHT signs and column selection) is this project's convention and is
stated here.

Counter layout (prefix-stable in rows and columns):
  key      = (seed & 0xffffffff, seed >> 32)
  Gaussian : element (i, j) of a sketch drawn on stream s uses the Philox block at
             counter (i, j >> 1, s, 0); even j takes z0, odd j takes z1.
  SRHT sign: d_i is the top bit of word (i & 3) of counter (i >> 2, 0, 3, 0);
             d_i = +1 if that bit is 0, -1 otherwise.
  SRHT keys: key_j is the 64-bit integer (w[2b] << 32) | w[2b+1] with b = j & 1 of
             counter (j >> 1, 0, 4, 0); the sample is the r columns with the
             smallest (key_j, j), listed in ascending key order.
Streams: 1 = X, 2 = Y, 3 = SRHT signs, 4 = SRHT sample keys, 5 = loss weights G,
6 = start vectors of the power-method norm estimate.

Gaussian transform (Box-Muller in FP64): from words (w0, w1, w2, w3)
  ka = (w0 >> 5) * 2**26 + (w1 >> 6),  kb = (w2 >> 5) * 2**26 + (w3 >> 6)  (53 bits)
  u1 = 1 - ka * 2**-53 in (0, 1],       u2 = kb * 2**-53 in [0, 1)
  z0 = sqrt(-2 ln u1) cos(2 pi u2),     z1 = sqrt(-2 ln u1) sin(2 pi u2).
FP32 / BF16 sketches are the FP64 values rounded to nearest-even directly.

Pins: the raw Philox4x32-10 words reproduce the generator's published
known-answer vectors (Random123, SC'11; tests/golden/philox4x32_10_kat.json).  The
Gaussian and SRHT properties the paper relies on are checked in the CPU tests
(moments, a Kolmogorov-Smirnov test against the normal CDF, decorrelation, sign
balance, distinct sample indices, the Sylvester-Hadamard closed form against
scipy.linalg.hadamard, X^T X = n' I).
"""
from __future__ import annotations

import numpy as np

MASK32 = 0xFFFFFFFF
# Philox4x32 round multipliers and Weyl key increments (SC'11, Section 5).
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
PHILOX_ROUNDS = 10

STREAM_X = 1
STREAM_Y = 2
STREAM_SRHT_SIGN = 3
STREAM_SRHT_KEY = 4
STREAM_G = 5
STREAM_POWER = 6

TWO_PI = 6.283185307179586  # the double nearest to 2*pi
TWO_M53 = 2.0 ** -53


def philox4x32_10(c0, c1, c2, c3, seed: int):
    """Philox4x32-10 block function applied elementwise.

    c0..c3 are integer arrays (broadcastable) holding 32-bit counter words; seed is
    the 64-bit key.  Returns four uint32 arrays.  Each round multiplies counter
    words 0 and 2 by the two round constants, splits the 64-bit products into high
    and low halves and mixes in the other words and the key; the key is advanced
    by the Weyl constants between rounds.
    """
    m = np.uint64(MASK32)
    x0 = np.asarray(c0, dtype=np.uint64) & m
    x1 = np.asarray(c1, dtype=np.uint64) & m
    x2 = np.asarray(c2, dtype=np.uint64) & m
    x3 = np.asarray(c3, dtype=np.uint64) & m
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    k0 = seed & MASK32
    k1 = (seed >> 32) & MASK32
    for _ in range(PHILOX_ROUNDS):
        p0 = x0 * PHILOX_M0           # < 2**64, exact in uint64
        p1 = x2 * PHILOX_M1
        hi0, lo0 = p0 >> np.uint64(32), p0 & m
        hi1, lo1 = p1 >> np.uint64(32), p1 & m
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0)), lo1, (hi0 ^ x3 ^ np.uint64(k1)), lo0
        k0 = (k0 + PHILOX_W0) & MASK32
        k1 = (k1 + PHILOX_W1) & MASK32
    return (x0.astype(np.uint32), x1.astype(np.uint32),
            x2.astype(np.uint32), x3.astype(np.uint32))


def box_muller(w0, w1, w2, w3):
    """Two FP64 standard normals per Philox block (the transform in the header)."""
    w0 = np.asarray(w0, np.uint64)
    w1 = np.asarray(w1, np.uint64)
    w2 = np.asarray(w2, np.uint64)
    w3 = np.asarray(w3, np.uint64)
    ka = ((w0 >> np.uint64(5)) << np.uint64(26)) + (w1 >> np.uint64(6))
    kb = ((w2 >> np.uint64(5)) << np.uint64(26)) + (w3 >> np.uint64(6))
    u1 = 1.0 - ka.astype(np.float64) * TWO_M53
    u2 = kb.astype(np.float64) * TWO_M53
    rad = np.sqrt(-2.0 * np.log(u1))
    theta = TWO_PI * u2
    return rad * np.cos(theta), rad * np.sin(theta)


def gaussian(seed: int, stream: int, rows: int, cols: int,
             row0: int = 0, col0: int = 0, workers: int = 1) -> np.ndarray:
    """FP64 Gaussian sketch block G[row0:row0+rows, col0:col0+cols] (row-major).

    Every element depends on its own counter only, so blocks of rows can be drawn
    in any order: `workers` > 1 draws them on that many host threads (NumPy's
    integer and transcendental loops release the interpreter lock); the values
    are the same."""
    out = np.empty((rows, cols), dtype=np.float64)
    if rows == 0 or cols == 0:
        return out
    j = np.arange(col0, col0 + cols, dtype=np.int64)
    pair = (j >> 1).astype(np.uint64)
    odd = (j & 1).astype(bool)
    chunk = max(1, (1 << 20) // max(cols, 1))

    def block(r0):
        r1 = min(rows, r0 + chunk)
        i = np.arange(row0 + r0, row0 + r1, dtype=np.uint64)[:, None]
        w = philox4x32_10(i, pair[None, :], stream, 0, seed)
        z0, z1 = box_muller(*w)
        out[r0:r1] = np.where(odd[None, :], z1, z0)

    starts = range(0, rows, chunk)
    if workers > 1 and len(starts) > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(block, starts))
    else:
        for r0 in starts:
            block(r0)
    return out


def round_f16(x: np.ndarray) -> np.ndarray:
    """Round FP64 to IEEE binary16, nearest-even, in one step (NumPy converts
    double to half directly, subnormals included), returned as FP64."""
    return np.asarray(x, np.float64).astype(np.float16).astype(np.float64)


def round_fp32(x: np.ndarray) -> np.ndarray:
    """Round FP64 to FP32, nearest-even (returned as float32)."""
    return np.asarray(x, np.float64).astype(np.float32)


def round_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to bfloat16 (8-bit significand), nearest-even.

    Returns the 16-bit bfloat16 patterns as uint16.  Works on the FP64 bit pattern
    directly (one rounding, no detour through FP32).  Values must lie in the
    normal range of bfloat16 or be zero; sketches and scaled matrices do.
    """
    x = np.ascontiguousarray(x, dtype=np.float64)
    u = x.view(np.uint64)
    drop = np.uint64(45)                       # 52 - 7 stored mantissa bits
    lsb = (u >> drop) & np.uint64(1)
    bias = np.uint64((1 << 44) - 1) + lsb
    rounded = (u + bias) & ~np.uint64((1 << 45) - 1)
    f32 = rounded.view(np.float64).astype(np.float32)   # exact: <= 8 significant bits
    return (f32.view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def bf16_bits_to_f64(b: np.ndarray) -> np.ndarray:
    b = np.asarray(b, np.uint16)
    return (b.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def round_bf16(x: np.ndarray) -> np.ndarray:
    """FP64 values of the bfloat16 rounding of x."""
    return bf16_bits_to_f64(round_bf16_bits(x))


def next_pow2(n: int) -> int:
    p = 1
    while p < n:
        p <<= 1
    return p


def srht_signs(seed: int, npad: int) -> np.ndarray:
    """Rademacher signs d_0..d_{npad-1} as int8 (+1 / -1)."""
    i = np.arange(npad, dtype=np.int64)
    w = philox4x32_10((i >> 2).astype(np.uint64), 0, STREAM_SRHT_SIGN, 0, seed)
    words = np.stack(w, axis=-1)[np.arange(npad), i & 3]
    return (1 - 2 * (words >> np.uint32(31)).astype(np.int64)).astype(np.int8)


def srht_keys(seed: int, npad: int) -> np.ndarray:
    """64-bit sampling keys key_0..key_{npad-1} (uint64)."""
    j = np.arange(npad, dtype=np.int64)
    w = np.stack(philox4x32_10((j >> 1).astype(np.uint64), 0, STREAM_SRHT_KEY, 0, seed),
                 axis=-1).astype(np.uint64)
    b = (j & 1)
    hi = w[np.arange(npad), 2 * b]
    lo = w[np.arange(npad), 2 * b + 1]
    return (hi << np.uint64(32)) | lo


def srht_sample(seed: int, npad: int, r: int) -> np.ndarray:
    """Indices of the r sampled Hadamard columns, ascending in (key, index)."""
    keys = srht_keys(seed, npad)
    order = np.lexsort((np.arange(npad), keys))   # primary: key, secondary: index
    return order[:r].astype(np.int32)


def hadamard_entry_sign(i: np.ndarray, j: np.ndarray) -> np.ndarray:
    """(-1)**popcount(i & j): the Sylvester-ordered Walsh-Hadamard matrix entries."""
    v = np.bitwise_and(np.asarray(i, np.uint64), np.asarray(j, np.uint64))
    # popcount parity by folding the bits
    for s in (32, 16, 8, 4, 2, 1):
        v = v ^ (v >> np.uint64(s))
    return 1 - 2 * (v & np.uint64(1)).astype(np.int64)


def srht_matrix(seed: int, n: int, r: int) -> np.ndarray:
    """Explicit SRHT sketch X (n x r, FP64): X[i, c] = d_i * H[i, idx[c]].

    H is the Sylvester-ordered Walsh-Hadamard matrix of order n' = next power of
    two >= n; only its first n rows are used (A is zero-padded to n' columns).
    Entries are +-1, with no 1/sqrt(r) normalization (the GN approximant does not
    depend on the scale of X, Section 1, the note that P_{XM,YN} = P_{X,Y}).
    """
    npad = next_pow2(n)
    d = srht_signs(seed, npad)[:n].astype(np.int64)
    idx = srht_sample(seed, npad, r).astype(np.int64)
    h = hadamard_entry_sign(np.arange(n)[:, None], idx[None, :])
    return (d[:, None] * h).astype(np.float64)
