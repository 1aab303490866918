"""Pins for the oracle's counter-based generator and sampling (CPU only)."""
import math
import os
from itertools import combinations

import numpy as np
import pytest

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")
GOLDEN32 = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows(path=GOLDEN):
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    return rows


@pytest.mark.parametrize("row", _kat_rows())
def test_philox_known_answers(row):
    out = philox.philox4x64(*[np.uint64(v) for v in row[:6]])
    assert [int(v) for v in out] == row[6:]


@pytest.mark.parametrize("row", _kat_rows(GOLDEN32))
def test_philox4x32_known_answers(row):
    out = philox.philox4x32(*[np.uint64(v) for v in row[:6]])
    assert [int(v) for v in out] == row[6:]


def test_philox4x32_matches_a_plain_integer_round():
    # one block recomputed with Python integers (arbitrary precision), round by round
    c, k = [0x01234567, 0x89ABCDEF, 0xDEADBEEF, 0x00C0FFEE], [0x13579BDF, 0x2468ACE0]
    x, kk = list(c), list(k)
    for _ in range(10):
        p0, p1 = 0xD2511F53 * x[0], 0xCD9E8D57 * x[2]
        x = [(p1 >> 32) ^ x[1] ^ kk[0], p1 & 0xFFFFFFFF, (p0 >> 32) ^ x[3] ^ kk[1], p0 & 0xFFFFFFFF]
        kk = [(kk[0] + 0x9E3779B9) & 0xFFFFFFFF, (kk[1] + 0xBB67AE85) & 0xFFFFFFFF]
    got = philox.philox4x32(*[np.uint64(v) for v in c + k])
    assert [int(v) for v in got] == x


def test_philox_matches_numpy_bit_generator():
    # numpy's Philox advances its counter before producing a block, so the block
    # it returns for counter c is the block function at c + 1.
    rng = np.random.default_rng(123)
    for _ in range(20):
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
        ctr = rng.integers(0, 2**63, size=4, dtype=np.uint64)
        ctr[0] = ctr[0] & np.uint64(0x7FFFFFFFFFFFFFF0)  # no carry out of word 0
        bg = np.random.Philox(key=key, counter=ctr)
        want = bg.random_raw(8)
        got0 = philox.philox4x64(ctr[0] + np.uint64(1), ctr[1], ctr[2], ctr[3], key[0], key[1])
        got1 = philox.philox4x64(ctr[0] + np.uint64(2), ctr[1], ctr[2], ctr[3], key[0], key[1])
        assert [int(v) for v in got0 + got1] == [int(v) for v in want]


def test_mulhilo_against_python_integers():
    rng = np.random.default_rng(5)
    a = rng.integers(0, 2**64, size=2000, dtype=np.uint64)
    b = rng.integers(0, 2**64, size=2000, dtype=np.uint64)
    a[:4] = [0, 1, 2**64 - 1, 2**63]
    b[:4] = [2**64 - 1, 2**64 - 1, 2**64 - 1, 2]
    hi, lo = philox.mulhilo64(a, b)
    for x, y, h, l in zip(a.tolist(), b.tolist(), hi.tolist(), lo.tolist()):
        p = x * y
        assert h == p >> 64 and l == p & (2**64 - 1)


def test_mulhi_bound_is_floor_scaling():
    x = np.array([0, 2**63, 2**64 - 1, 12345678901234567890], dtype=np.uint64)
    for bound in (1, 7, 1000, 2**40 + 3):
        got = philox.mulhi64(x, np.uint64(bound)).tolist()
        assert got == [(int(v) * bound) >> 64 for v in x.tolist()]
        assert all(0 <= g < bound for g in got)


def test_unit_maps():
    assert philox.to_unit_open0(np.uint64(0)) == 2.0**-53
    assert philox.to_unit_open0(np.uint64(2**64 - 1)) == 1.0
    assert philox.to_unit_open1(np.uint64(0)) == 0.0
    assert philox.to_unit_open1(np.uint64(2**64 - 1)) == 1.0 - 2.0**-53


def test_normal_box_muller_value_and_moments():
    i = np.arange(200_000, dtype=np.uint64)
    g = philox.normal_at(99, i, np.uint64(3))
    assert abs(g.mean()) < 0.01 and abs(g.var() - 1.0) < 0.01
    assert abs((g**4).mean() - 3.0) < 0.05
    # One value recomputed by hand from the four 32-bit words (64-bit halves of i, j and the seed).
    i0, j0, sd = (5 << 32) + 17, 3, (7 << 32) + 99
    w = [int(v) for v in philox.philox4x32(np.uint64(17), np.uint64(5), np.uint64(3), np.uint64(0),
                                           np.uint64(99), np.uint64(7))]
    u1 = ((((w[1] << 32) | w[0]) >> 11) + 1) / 2.0**53
    u2 = (((w[3] << 32) | w[2]) >> 11) / 2.0**53
    want = math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)
    assert philox.normal_at(sd, np.uint64(i0), np.uint64(j0)) == pytest.approx(want, rel=1e-15)
    # entries that differ only in the high halves of i, j or the seed draw different values
    base = philox.normal_at(sd, np.uint64(i0), np.uint64(j0))
    assert base != philox.normal_at(sd, np.uint64(17), np.uint64(j0))
    assert base != philox.normal_at(sd, np.uint64(i0), np.uint64(j0 + (1 << 32)))
    assert base != philox.normal_at(99, np.uint64(i0), np.uint64(j0))


def test_floyd_basic_properties():
    for n, k in [(1, 1), (10, 10), (10, 0), (1000, 50), (2**40, 5), (97, 96)]:
        s = philox.floyd_sample(n, k, seed=3, stream=0)
        assert s.size == k and len(set(s.tolist())) == k
        assert np.all(np.diff(s) > 0) and (k == 0 or (s[0] >= 0 and s[-1] < n))
    assert philox.floyd_sample(10, 10, 1, 0).tolist() == list(range(10))
    with pytest.raises(ValueError):
        philox.floyd_sample(5, 6, 0, 0)
    # Streams and seeds give different samples.
    a = philox.floyd_sample(10**6, 20, 1, 0)
    assert not np.array_equal(a, philox.floyd_sample(10**6, 20, 1, 1))
    assert not np.array_equal(a, philox.floyd_sample(10**6, 20, 2, 0))


def test_floyd_is_uniform_over_subsets():
    """Chi-square over all C(10,3) = 120 subsets; Floyd gives each 1/120."""
    n, k, trials = 10, 3, 36_000
    index = {c: t for t, c in enumerate(combinations(range(n), k))}
    counts = np.zeros(len(index))
    for seed in range(trials):
        counts[index[tuple(philox.floyd_sample(n, k, seed, 0).tolist())]] += 1
    exp = trials / len(index)
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    # 119 degrees of freedom: mean 119, sd ~15.4; 200 is beyond 5 sd.
    assert chi2 < 200.0, chi2


def test_error_samples_are_uniform_and_in_range():
    i, j = philox.error_sample_indices(7, 11, 77_000, seed=4)
    assert i.min() >= 0 and i.max() < 7 and j.min() >= 0 and j.max() < 11
    counts = np.bincount(i * 11 + j, minlength=77)
    assert counts.min() > 800 and counts.max() < 1200
    i2, j2 = philox.error_sample_indices(7, 11, 100, seed=4, start=500)
    assert np.array_equal(i2, i[500:600]) and np.array_equal(j2, j[500:600])
    # one sample recomputed from its block with Python integers; a sample index past 2^32 and a
    # seed past 2^32 use the high halves of the counter and key
    t, sd, m, n = (3 << 32) + 5, (9 << 32) + 4, 10**6 + 3, 777
    w = [int(v) for v in philox.philox4x32(np.uint64(5), np.uint64(3), np.uint64(4), np.uint64(0), np.uint64(4),
                                           np.uint64(9))]
    i3, j3 = philox.error_sample_indices(m, n, 1, seed=sd, start=t)
    assert int(i3[0]) == ((((w[1] << 32) | w[0]) * m) >> 64)
    assert int(j3[0]) == ((((w[3] << 32) | w[2]) * n) >> 64)
