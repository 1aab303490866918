"""Pins for the oracle's leverage-score follow-up (Section 5's leverage variant; CPU only).

The scores are pinned by what fixes them independently of the oracle's own code path: an
orthonormal basis's squared row norms sum to its rank and equal the diagonal of the
orthogonal projector onto its span, which is computed here from a QR factorisation of the
sampled columns themselves.  The sampling law (exponential races) is pinned by its defining
property, checked by counting over seeds: each draw takes a row with probability proportional
to its score among the rows not yet drawn.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

import workloads
from oracle import cabs as oc
from oracle import philox
from oracle.matrices import Matrix


def test_scores_of_an_orthonormal_basis():
    rng = np.random.default_rng(0)
    q, _ = np.linalg.qr(rng.normal(size=(50, 7)))
    s = np.linspace(3.0, 1.0, 7)
    lev = oc.leverage_scores(q, s, 7)
    assert lev.sum() == pytest.approx(7.0, rel=1e-13)
    assert np.all(lev >= 0.0) and np.all(lev <= 1.0 + 1e-13)
    # the projector's diagonal from a different basis of the same span
    b = q @ rng.normal(size=(7, 7))
    u, _, _ = np.linalg.svd(b, full_matrices=False)
    assert np.allclose(lev, (u * u).sum(1), rtol=1e-12, atol=1e-15)
    # coordinate basis: 1 on its rows, 0 elsewhere
    e = np.zeros((9, 3))
    e[[1, 4, 6], [0, 1, 2]] = 1.0
    assert np.array_equal(oc.leverage_scores(e, np.ones(3), 3), np.isin(np.arange(9), [1, 4, 6]).astype(float))


def test_components_below_the_cut_do_not_count():
    e = np.eye(4)[:, :2]
    lev = oc.leverage_scores(e, np.array([1.0, 1e-20]), 2)
    assert np.array_equal(lev, np.array([1.0, 0.0, 0.0, 0.0]))
    assert np.array_equal(oc.leverage_scores(e, np.zeros(2), 2), np.zeros(4))


@pytest.mark.parametrize("ortho", [True, False])
def test_pilot_scores_are_the_projector_onto_the_sampled_columns(ortho):
    """With every pilot component kept, span(U) = span(C(:, I_c)); the leverage scores the
    follow-up uses are then the diagonal of the projector onto the sampled columns (QR of C)."""
    spec, _ = workloads.config("rbf2000", 0.1)
    k = 12
    res = oc.cabs(spec, oc.Params.square(k, seed=3, follow_up="leverage", orthogonalize=ortho))
    assert res.pilot.keep.all()
    so = res.pilot_sigma
    lev_r = ((res.P ** 2) / so).sum(1)
    lev_c = ((res.Q ** 2) / so).sum(1)
    qc, _ = np.linalg.qr(res.pilot_C)
    qr_, _ = np.linalg.qr(res.pilot_Rt)
    if ortho:
        assert np.allclose(lev_r, (qc * qc).sum(1), rtol=1e-9, atol=1e-13)
        assert np.allclose(lev_c, (qr_ * qr_).sum(1), rtol=1e-9, atol=1e-13)
        assert lev_r.sum() == pytest.approx(k, rel=1e-11)
    else:
        # unit-norm columns that are not orthogonal: scores sum to k, span unchanged
        assert lev_r.sum() == pytest.approx(k, rel=1e-11)
        assert np.all(lev_r <= (qc * qc).sum(1) * (1 + 1e-9) * k)


def test_sample_takes_exactly_the_rows_with_positive_score():
    sc = np.zeros(40)
    sc[[3, 9, 20, 33]] = [0.1, 5.0, 1.0, 2.0]
    for seed in range(20):
        assert np.array_equal(oc.leverage_sample(sc, 4, seed, 5), np.array([3, 9, 20, 33]))
    # more rows than positive scores: zero-score rows follow in index order
    assert np.array_equal(oc.leverage_sample(sc, 6, 0, 5), np.array([0, 1, 3, 9, 20, 33]))


def test_first_draw_is_proportional_to_the_score():
    sc = np.array([1.0, 2.0, 3.0, 4.0])
    counts = np.zeros(4)
    for seed in range(20000):
        counts[oc.leverage_sample(sc, 1, seed, 6)[0]] += 1
    p = stats.chisquare(counts, 20000 * sc / sc.sum()).pvalue
    assert p > 1e-3, counts


def test_pairs_follow_successive_sampling_without_replacement():
    """P({i, j}) = p_i p_j / (1 - p_i) + p_j p_i / (1 - p_j) for two draws without replacement."""
    sc = np.array([1.0, 2.0, 3.0, 4.0, 6.0])
    pr = sc / sc.sum()
    pairs = list(itertools.combinations(range(5), 2))
    want = np.array([pr[i] * pr[j] / (1 - pr[i]) + pr[j] * pr[i] / (1 - pr[j]) for i, j in pairs])
    assert want.sum() == pytest.approx(1.0)
    counts = np.zeros(len(pairs))
    n = 30000
    for seed in range(n):
        got = tuple(oc.leverage_sample(sc, 2, seed, 5).tolist())
        counts[pairs.index(got)] += 1
    assert stats.chisquare(counts, n * want).pvalue > 1e-3, counts


def test_uniform_scores_give_uniform_subsets():
    counts = {}
    n = 15000
    for seed in range(n):
        key = tuple(oc.leverage_sample(np.ones(6), 2, seed, 6).tolist())
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 15
    assert stats.chisquare(np.array(list(counts.values())), np.full(15, n / 15)).pvalue > 1e-3


def test_draws_are_the_counter_based_generator():
    u = philox.unit_draws(5, 7, 5)
    w = philox.philox4x64(np.arange(5, dtype=np.uint64), 0, 5, 0, 7, 0)[0]
    assert np.array_equal(u, ((w >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53)
    assert np.all((u > 0.0) & (u <= 1.0))


def test_leverage_follow_up_recovers_an_exact_rank_input():
    spec = workloads.exact_rank(90, 70, 6, seed=4)
    res = oc.cabs(spec, oc.Params.square(6, seed=1, follow_up="leverage", sketch_kind="pseudo_skeleton"))
    assert oc.rel_error_exact(Matrix(spec), res.C, res.Umid, res.Rt) < 1e-10
    res2 = oc.cabs(spec, oc.Params.square(6, seed=1, follow_up="leverage", sketch_kind="pseudo_skeleton"))
    assert np.array_equal(res.idx_r, res2.idx_r) and np.array_equal(res.idx_c, res2.idx_c)


def test_leverage_follow_up_error_is_above_the_optimum():
    spec, _ = workloads.config("lowrank1e5s", 0.002)
    k = 10
    res = oc.cabs(spec, oc.Params.square(k, seed=2, follow_up="leverage"))
    a = Matrix(spec).full_rows(0, spec.m)
    s = np.linalg.svd(a, compute_uv=False)
    optimum = math.sqrt((s[k:] ** 2).sum() / (s ** 2).sum())
    err = oc.rel_error_exact(Matrix(spec), res.C, res.Umid, res.Rt)
    assert optimum * (1 - 1e-12) <= err < 1.0
