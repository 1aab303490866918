"""Pins for the oracle's end-to-end CABS driver and error metric (CPU only)."""
import math

import numpy as np
import pytest

import workloads
from oracle import cabs as oc
from oracle import philox
from oracle.matrices import Matrix


def _dense(spec):
    return Matrix(spec).full_rows(0, spec.m)


@pytest.mark.parametrize("name,scale,k", [("rbf2000", 0.1, 12), ("lowrank1e5s", 0.002, 10)])
def test_error_is_never_below_the_truncated_svd_optimum(name, scale, k):
    spec, _ = workloads.config(name, scale)
    res = oc.cabs(spec, oc.Params.square(k, seed=1))
    a = _dense(spec)
    s = np.linalg.svd(a, compute_uv=False)
    optimum = math.sqrt((s[k:] ** 2).sum() / (s**2).sum())
    err = oc.rel_error_exact(Matrix(spec), res.C, res.Umid, res.Rt)
    assert err >= optimum * (1 - 1e-12)
    assert err == pytest.approx(np.linalg.norm(a - oc.reconstruct(res)) / np.linalg.norm(a), rel=1e-10)


def test_exact_rank_input_is_recovered_in_pseudo_skeleton_mode():
    spec = workloads.exact_rank(80, 60, 5, seed=11)
    res = oc.cabs(spec, oc.Params.square(5, seed=2, sketch_kind="pseudo_skeleton"))
    assert oc.rel_error_exact(Matrix(spec), res.C, res.Umid, res.Rt) < 1e-11


def test_entries_touched_is_linear_and_matches_brute_force():
    spec, _ = workloads.config("rbf2000", 0.04)
    prm = oc.Params(6, 5, 4, 7, seed=3)
    res = oc.cabs(spec, prm, track=True)
    m, n = spec.m, spec.n
    formula = m * (5 + 7) + n * (6 + 4) - 6 * 5 - 4 * 7
    assert res.entries_touched == formula
    assert res.entries_touched < 2 * (m + n) * 7


def test_pilot_indices_and_determinism():
    spec, _ = workloads.config("lowrank1e5", 0.003)
    prm = oc.Params.square(8, seed=5)
    r1 = oc.cabs(spec, prm)
    r2 = oc.cabs(spec, prm)
    assert np.array_equal(r1.pilot_rows, philox.floyd_sample(spec.m, 8, 5, 0))
    assert np.array_equal(r1.pilot_cols, philox.floyd_sample(spec.n, 8, 5, 1))
    assert np.array_equal(r1.idx_r, r2.idx_r) and np.array_equal(r1.Umid, r2.Umid)
    assert np.all(np.diff(r1.idx_r) > 0) and np.all(np.diff(r1.idx_c) > 0)


def test_kmeans_starts_from_the_pilot_sample_and_lowers_the_encoding_error():
    spec, _ = workloads.config("rbf2000", 0.1)
    res = oc.cabs(spec, oc.Params.square(10, seed=0))
    # initial objective uses the pilot rows as representatives (Delta_e >= 0 premise)
    _, dmin, _ = oc.assign(res.P, res.P[res.pilot_rows])
    assert res.km_r.e_initial == pytest.approx(float(res.w_r @ dmin), rel=1e-12)
    assert res.km_r.e_final <= res.km_r.e_initial and res.km_c.e_final <= res.km_c.e_initial


def test_embedding_reproduces_the_pilot_sketch():
    spec, _ = workloads.config("rbf2000", 0.05)
    res = oc.cabs(spec, oc.Params.square(8, seed=4))
    pilot = res.pilot_C @ res.pilot.Umid @ res.pilot_Rt.T
    assert np.allclose(res.P @ res.Q.T, pilot, atol=1e-12 * np.abs(pilot).max())
    # P P^T is the positive square root of pilot pilot^T
    ppt = res.P @ res.P.T
    assert np.allclose(ppt @ ppt, pilot @ pilot.T, atol=1e-10 * np.abs(pilot).max() ** 2)


def test_unequal_sample_sizes_and_factor_form():
    spec, _ = workloads.config("lowrank1e5s", 0.002)
    prm = oc.Params(9, 7, 5, 6, seed=8, factors=True)
    res = oc.cabs(spec, prm)
    assert res.idx_r.size == 5 and res.idx_c.size == 6
    assert res.Umid.shape == (6, 5)
    u, s, v = res.factors
    assert np.allclose(u @ np.diag(s) @ v.T, oc.reconstruct(res), atol=1e-9 * np.abs(oc.reconstruct(res)).max())
    # more centres than pilot rows: initial centres come from stream 2 / 3
    res2 = oc.cabs(spec, oc.Params(4, 4, 6, 6, seed=8))
    assert res2.idx_r.size == 6


def test_initial_centres_with_more_centres_than_pilot_rows():
    """k2 > k1: the k-means start is k2 distinct rows of the embedding drawn uniformly (each row in
    with probability k2 / n, checked by counting over seeds), the rows and the columns from their
    own streams; k2 <= k1: the first k2 pilot rows."""
    rng = np.random.default_rng(0)
    emb = rng.normal(size=(12, 3))
    pilot = np.array([1, 4, 9])
    assert np.array_equal(oc.initial_centres(emb, pilot, 2, 12, 0, philox.STREAM_INIT_ROWS), emb[[1, 4]])
    counts = np.zeros(12)
    for seed in range(6000):
        z = oc.initial_centres(emb, pilot, 5, 12, seed, philox.STREAM_INIT_ROWS)
        # every centre is a row of emb, all distinct (brute-force match)
        hit = np.all(np.isclose(z[:, None, :], emb[None, :, :], rtol=0, atol=0), axis=2)
        assert np.all(hit.sum(1) == 1)
        rows = hit.argmax(1)
        assert np.unique(rows).size == 5
        counts[rows] += 1
    from scipy import stats
    assert stats.chisquare(counts, np.full(12, 6000 * 5 / 12)).pvalue > 1e-3
    zr = oc.initial_centres(emb, pilot, 5, 12, 3, philox.STREAM_INIT_ROWS)
    zc = oc.initial_centres(emb, pilot, 5, 12, 3, philox.STREAM_INIT_COLS)
    assert not np.array_equal(zr, zc)


def test_invalid_parameters_raise():
    spec, _ = workloads.config("rbf2000", 0.01)
    with pytest.raises(ValueError):
        oc.cabs(spec, oc.Params.square(spec.m + 1))
    with pytest.raises(ValueError):
        oc.cabs(spec, oc.Params(3, 3, 3, 3, weight_kind="nope"))


def test_sampled_error_against_brute_force_and_exact():
    spec, _ = workloads.config("lowrank1e5s", 0.002)
    res = oc.cabs(spec, oc.Params.square(6, seed=0))
    mat = Matrix(spec)
    a = _dense(spec)
    approx = oc.reconstruct(res)
    i, j = philox.error_sample_indices(spec.m, spec.n, 5000, seed=21)
    num = float(((a[i, j] - approx[i, j]) ** 2).sum())
    den = float((a[i, j] ** 2).sum())
    rel, n2, d2 = oc.rel_error_sampled(mat, res.C, res.Umid, res.Rt, 5000, 21, chunk=777)
    assert n2 == pytest.approx(num, rel=1e-10) and d2 == pytest.approx(den, rel=1e-12)
    exact = oc.rel_error_exact(mat, res.C, res.Umid, res.Rt)
    assert exact == pytest.approx(np.linalg.norm(a - approx) / np.linalg.norm(a), rel=1e-12)
    big, _, _ = oc.rel_error_sampled(mat, res.C, res.Umid, res.Rt, 400_000, 22)
    assert big == pytest.approx(exact, rel=0.05)


def test_hard_threshold_against_a_plain_sort():
    rng = np.random.default_rng(4)
    for m, k in [(1, 1), (10, 10), (50, 7), (300, 64)]:
        w = np.round(rng.exponential(size=m), 1)  # rounded, so that many weights tie
        got = oc.hard_threshold(w, k).tolist()
        want = sorted(sorted(range(m), key=lambda i: (-w[i], i))[:k])
        assert got == want
    # constant weights: every row ties, so the first k rows
    assert oc.hard_threshold(np.ones(20), 6).tolist() == list(range(6))
    # a NaN weight ranks below every number
    w = np.array([0.5, np.nan, 2.0, 0.1])
    assert oc.hard_threshold(w, 3).tolist() == [0, 2, 3]


def test_hard_threshold_follow_up_takes_the_largest_embedding_rows():
    spec = workloads.exact_rank(90, 70, 6, seed=5)
    prm = oc.Params.square(6, seed=3, weight_kind="pow", weight_param=2.0, follow_up="hard")
    res = oc.cabs(spec, prm)
    norms = np.linalg.norm(res.P, axis=1)
    assert res.idx_r.tolist() == sorted(np.argsort(-norms, kind="stable")[:6].tolist())
    assert res.km_r is None and res.km_c is None
    # the chosen rows and columns feed the follow-up round: on an exact-rank input with a
    # full-rank W the pseudo-skeleton form recovers A
    res2 = oc.cabs(spec, oc.Params.square(6, seed=3, weight_kind="pow", weight_param=2.0, follow_up="hard",
                                          sketch_kind="pseudo_skeleton"))
    wb = res2.C[res2.idx_r, :]
    assert np.linalg.matrix_rank(wb) == 6
    assert oc.rel_error_exact(Matrix(spec), res2.C, res2.Umid, res2.Rt) < 1e-10
    with pytest.raises(ValueError):
        oc.cabs(spec, oc.Params.square(6, follow_up="nope"))
