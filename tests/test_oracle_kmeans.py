"""Pins for the oracle's weighted k-means, snapping and weights (CPU only)."""
import numpy as np
import pytest
from sklearn.cluster import KMeans

from oracle import cabs as oc


def _blobs(seed, m=300, d=4, k=6):
    rng = np.random.default_rng(seed)
    centers = rng.normal(scale=4.0, size=(k, d))
    lab = rng.integers(0, k, size=m)
    return centers[lab] + rng.normal(size=(m, d))


@pytest.mark.parametrize("iters", [1, 3])
def test_unweighted_kmeans_matches_sklearn_lloyd(iters):
    p = _blobs(0)
    z0 = p[[3, 50, 100, 150, 200, 250]]
    w = oc.upsilon(np.linalg.norm(p, axis=1), "const", 0.0)
    ours = oc.weighted_kmeans(p, w, z0, iters)
    ref = KMeans(n_clusters=6, init=z0, n_init=1, max_iter=iters, algorithm="lloyd", tol=0.0).fit(p)
    assert np.allclose(ours.Z, ref.cluster_centers_, atol=1e-12)
    assert np.array_equal(ours.labels, ref.labels_)
    assert ours.e_final == pytest.approx(ref.inertia_, rel=1e-12)


def test_weighted_kmeans_matches_sklearn_sample_weight():
    p = _blobs(1)
    z0 = p[[1, 2, 3, 4, 5, 6]]
    w = oc.upsilon(np.linalg.norm(p, axis=1), "pow", 2.0)
    assert np.allclose(w, (p * p).sum(1))
    ours = oc.weighted_kmeans(p, w, z0, 2)
    ref = KMeans(n_clusters=6, init=z0, n_init=1, max_iter=2, algorithm="lloyd", tol=0.0).fit(p, sample_weight=w)
    assert np.allclose(ours.Z, ref.cluster_centers_, atol=1e-10)
    assert np.array_equal(ours.labels, ref.labels_)


def test_objective_never_increases_and_max_cluster():
    p = _blobs(2, m=500, d=6, k=9)
    w = oc.upsilon(np.linalg.norm(p, axis=1), "sigmoid", 0.7)
    ours = oc.weighted_kmeans(p, w, p[:9], 8)
    obj = np.array(ours.objective)
    assert np.all(np.diff(obj) <= 1e-9 * obj[0])
    assert ours.e_final <= ours.e_initial
    assert ours.max_cluster == np.bincount(ours.labels).max()


def test_empty_cluster_keeps_centre_and_ties_go_to_lowest_index():
    p = np.array([[0.0, 0.0], [0.0, 1.0], [10.0, 0.0], [10.0, 1.0]])
    z0 = np.array([[0.0, 0.5], [10.0, 0.5], [100.0, 100.0], [0.0, 0.5]])  # centre 2 far away, 3 duplicates 0
    res = oc.weighted_kmeans(p, np.ones(4), z0, 3)
    assert np.array_equal(res.Z[2], z0[2])        # never gets a point
    assert np.array_equal(res.Z[3], z0[3])        # always loses the tie to centre 0
    assert res.labels.tolist() == [0, 0, 1, 1]
    assert np.allclose(res.Z[0], [0.0, 0.5]) and np.allclose(res.Z[1], [10.0, 0.5])


def test_zero_weight_cluster_keeps_centre():
    p = np.array([[0.0], [0.1], [5.0], [5.2]])
    w = oc.upsilon(np.abs(p[:, 0]), "step", 1.0)   # the two small rows weigh 0
    res = oc.weighted_kmeans(p, w, np.array([[0.05], [4.0]]), 2)
    assert res.Z[0, 0] == 0.05 and res.Z[1, 0] == pytest.approx(5.1)


def test_snap_by_brute_force():
    rng = np.random.default_rng(3)
    p = rng.normal(size=(40, 3))
    p[7] = p[8]                   # exact duplicate rows force a tie
    z = np.vstack([p[8] + 1e-9, p[8], rng.normal(size=(5, 3))])
    got = oc.snap(p, z)
    taken, want = set(), []
    for j in range(z.shape[0]):
        best, bd = None, np.inf
        for l in range(40):
            if l in taken:
                continue
            dd = float(((p[l] - z[j]) ** 2).sum())
            if dd < bd:
                best, bd = l, dd
        taken.add(best)
        want.append(best)
    assert got.tolist() == sorted(want)
    assert 7 in got and 8 in got          # both duplicates taken, lowest first
    assert len(set(got.tolist())) == z.shape[0]


def test_snap_midpoint_tie_goes_to_the_lowest_row():
    """A two-row cluster's centre is the midpoint: both rows are nearest."""
    rng = np.random.default_rng(4)
    p = rng.normal(size=(50, 6))
    z = oc.centroid_update(p, np.ones(50), np.where(np.arange(50) == 17, 0, np.where(np.arange(50) == 31, 0, 1)),
                           np.zeros((2, 6)))
    assert oc.snap(p, z[:1]).tolist() == [17]
    # without the tie window the choice would follow floating-point rounding
    d = ((p[[17, 31]] - z[0]) ** 2).sum(1)
    assert abs(d[0] - d[1]) <= 1e-12 * d.max()
    # a real gap well above the window is not a tie
    z2 = 0.6 * p[17] + 0.4 * p[31]
    assert oc.snap(p, z2[None]).tolist() == [17]
    z3 = 0.4 * p[17] + 0.6 * p[31]
    assert oc.snap(p, z3[None]).tolist() == [31]


def test_upsilon_kinds():
    x = np.array([0.0, 0.5, 2.0])
    assert oc.upsilon(x, "const", 3.0).tolist() == [1.0, 1.0, 1.0]
    assert np.allclose(oc.upsilon(x, "pow", 1.5), x**1.5)
    assert np.allclose(oc.upsilon(x, "sigmoid", 2.0), 1 / (1 + np.exp(-2 * x)))
    assert oc.upsilon(x, "step", 0.5).tolist() == [0.0, 1.0, 1.0]
    for kind in ("pow", "sigmoid", "step"):
        assert np.all(np.diff(oc.upsilon(np.linspace(0, 3, 20), kind, 1.0)) >= 0)
