"""Counter-based random numbers for the oracle (test infrastructure only).

Philox-4x64-10 and Philox-4x32-10 are written out from their published
definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC 2011): ten rounds of two full-width multiplications (64x64->128
or 32x32->64 bits) with the constants below, the key bumped by two Weyl
increments after every round.  The paper under study
only says that the pilot rows and columns are chosen at random (Algorithm 2,
pilot sampling); the reading taken here is: uniform sampling without
replacement, rows and columns independent, realised with Floyd's algorithm on
top of this generator so that a GPU can reproduce every draw bit for bit.

Philox-4x64-10 stream layout (counter = (a, b, stream, 0), key = (seed, 0)):
  0 pilot rows, 1 pilot columns, 2/3 extra initial centres (rows/columns) when
  the follow-up size exceeds the pilot size.
The two high-volume draws use the cheaper Philox-4x32-10 (its 32-bit
products are what a GPU multiplies natively), key = the 32-bit halves of the
seed: the error-estimation samples (counter (lo t, hi t, 4, 0)) and the noise
of the low-rank generator, one draw per entry of A (counter = the 32-bit
halves of (i, j)).
"""
from __future__ import annotations

import numpy as np

_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)
PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
PHILOX_M1 = np.uint64(0xCA5A826395121157)
PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)

STREAM_PILOT_ROWS = 0
STREAM_PILOT_COLS = 1
STREAM_INIT_ROWS = 2
STREAM_INIT_COLS = 3
STREAM_ERROR = 4
STREAM_LEVERAGE_ROWS = 5
STREAM_LEVERAGE_COLS = 6
STREAM_TARGET_ROWS = 7   # target sampling of the bilateral resampling CUR (Algorithm 1)
STREAM_TARGET_COLS = 8

PHILOX32_M0 = np.uint64(0xD2511F53)
PHILOX32_M1 = np.uint64(0xCD9E8D57)
PHILOX32_W0 = np.uint64(0x9E3779B9)
PHILOX32_W1 = np.uint64(0xBB67AE85)


def _u64(x) -> np.ndarray:
    return np.asarray(x, dtype=np.uint64)


def mulhilo64(a, b):
    """Full 128-bit product of two uint64 arrays, as (high word, low word)."""
    a = _u64(a)
    b = _u64(b)
    al, ah = a & _M32, a >> _S32
    bl, bh = b & _M32, b >> _S32
    p0 = al * bl
    p1 = al * bh
    p2 = ah * bl
    p3 = ah * bh
    mid = (p0 >> _S32) + (p1 & _M32) + (p2 & _M32)
    hi = p3 + (p1 >> _S32) + (p2 >> _S32) + (mid >> _S32)
    with np.errstate(over="ignore"):
        lo = a * b
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1):
    """Philox-4x64-10 block function, vectorised over broadcastable uint64 arrays."""
    x = [_u64(c0), _u64(c1), _u64(c2), _u64(c3)]
    k0 = _u64(k0)
    k1 = _u64(k1)
    with np.errstate(over="ignore"):
        for _ in range(10):
            hi0, lo0 = mulhilo64(PHILOX_M0, x[0])
            hi1, lo1 = mulhilo64(PHILOX_M1, x[2])
            x = [hi1 ^ x[1] ^ k0, lo1, hi0 ^ x[3] ^ k1, lo0]
            k0 = k0 + PHILOX_W0
            k1 = k1 + PHILOX_W1
    return x


def mulhi64(x, bound):
    """Map uniform uint64 words to integers in [0, bound) as floor(x * bound / 2^64)."""
    hi, _ = mulhilo64(x, bound)
    return hi


def to_unit_open0(x) -> np.ndarray:
    """uint64 -> double in (0, 1]: ((x >> 11) + 1) * 2^-53."""
    return ((_u64(x) >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)


def to_unit_open1(x) -> np.ndarray:
    """uint64 -> double in [0, 1): (x >> 11) * 2^-53."""
    return (_u64(x) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def philox4x32(c0, c1, c2, c3, k0, k1):
    """Philox-4x32-10 block function on 32-bit words held in uint64 arrays.

    Each round multiplies words 0 and 2 by the round constants (32x32 -> 64
    bits, exact in uint64), then mixes the high halves with words 1 and 3 and
    the key: (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0).
    """
    x = [_u64(c0) & _M32, _u64(c1) & _M32, _u64(c2) & _M32, _u64(c3) & _M32]
    k0 = _u64(k0) & _M32
    k1 = _u64(k1) & _M32
    for _ in range(10):
        p0 = PHILOX32_M0 * x[0]
        p1 = PHILOX32_M1 * x[2]
        x = [(p1 >> _S32) ^ x[1] ^ k0, p1 & _M32, (p0 >> _S32) ^ x[3] ^ k1, p0 & _M32]
        k0 = (k0 + PHILOX32_W0) & _M32
        k1 = (k1 + PHILOX32_W1) & _M32
    return x


def normal_at(seed: int, i, j) -> np.ndarray:
    """Standard normal for entry (i, j) of the low-rank generator's noise.

    Philox-4x32-10 at counter (lo(i), hi(i), lo(j), hi(j)), key (lo(seed),
    hi(seed)); words 1:0 and 3:2 joined into 64-bit integers give u1 in (0, 1]
    and u2 in [0, 1), and Box-Muller gives sqrt(-2 ln u1) cos(2 pi u2).
    """
    i = _u64(i)
    j = _u64(j)
    sd = np.uint64(seed)
    w = philox4x32(i & _M32, i >> _S32, j & _M32, j >> _S32, sd & _M32, sd >> _S32)
    u1 = to_unit_open0((w[1] << _S32) | w[0])
    u2 = to_unit_open1((w[3] << _S32) | w[2])
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def floyd_sample(n: int, k: int, seed: int, stream: int) -> np.ndarray:
    """k distinct integers from [0, n), uniformly, by Floyd's algorithm; sorted.

    Draw t (t = 0..k-1) looks at j = n - k + t, takes v uniform in [0, j] from
    word 0 of the block at counter (t, 0, stream, 0), and adds v, or j when v
    was already taken.  Every k-subset is equally likely (Bentley & Floyd,
    CACM 30(9), 1987).
    """
    if not (0 <= k <= n):
        raise ValueError(f"cannot draw {k} distinct values from [0, {n})")
    if k == 0:
        return np.zeros(0, dtype=np.int64)
    t = np.arange(k, dtype=np.uint64)
    words = philox4x64(t, 0, stream, 0, seed, 0)[0]
    j = np.uint64(n - k) + t
    v = mulhi64(words, j + np.uint64(1))
    chosen: set[int] = set()
    for vi, ji in zip(v.tolist(), j.tolist()):
        chosen.add(ji if vi in chosen else vi)
    return np.array(sorted(chosen), dtype=np.int64)


def unit_draws(n: int, seed: int, stream: int) -> np.ndarray:
    """u_i in (0, 1] for i = 0..n-1: word 0 of the Philox-4x64-10 block at counter (i, 0, stream, 0),
    key (seed, 0), through to_unit_open0."""
    return to_unit_open0(philox4x64(np.arange(n, dtype=np.uint64), 0, stream, 0, seed, 0)[0])


def error_sample_indices(m: int, n: int, count: int, seed: int, start: int = 0):
    """The (i, j) entry positions used by the sampled error estimate.

    Sample t takes the Philox-4x32-10 block at counter (lo t, hi t, 4, 0),
    key (lo seed, hi seed); words 1:0 and 3:2 joined into 64-bit integers
    give i = mulhi64(word, m) and j = mulhi64(word, n).  Samples are i.i.d.
    uniform over the m*n entries, drawn with replacement.
    """
    t = np.arange(start, start + count, dtype=np.uint64)
    sd = np.uint64(seed)
    w = philox4x32(t & _M32, t >> _S32, STREAM_ERROR, 0, sd & _M32, sd >> _S32)
    wi = (w[1] << _S32) | w[0]
    wj = (w[3] << _S32) | w[2]
    return mulhi64(wi, np.uint64(m)).astype(np.int64), mulhi64(wj, np.uint64(n)).astype(np.int64)
