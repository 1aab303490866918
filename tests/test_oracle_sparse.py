"""Pins for the sparse (CSR) source and its stand-ins (CPU only).

The oracle's CSR accessor is pinned by brute force against the dense array of the same
matrix (scipy.sparse toarray); the stand-ins by their defining statistics; the method on a
sparse input by the invariants that hold for any input (error never below the truncated-SVD
optimum, exact recovery of an exact-rank input in pseudo-skeleton mode)."""
import math

import numpy as np
import pytest

import workloads
from oracle import cabs as oc
from oracle.matrices import Matrix


def _small(seed=0, m=300, n=420, density=0.03):
    return workloads.movie_like(m, n, density, seed=seed)


def test_csr_entries_cols_rows_equal_the_dense_array():
    spec = _small()
    a = spec.sp.toarray()
    mat = Matrix(spec)
    rng = np.random.default_rng(1)
    i = rng.integers(0, spec.m, 5000)
    j = rng.integers(0, spec.n, 5000)
    # half the probes on listed nonzeros
    nz = rng.integers(0, spec.nnz, 2500)
    rows = np.repeat(np.arange(spec.m), np.diff(spec.sp.indptr))
    i[:2500], j[:2500] = rows[nz], spec.sp.indices[nz]
    assert np.array_equal(mat.entries(i, j), a[i, j])
    cols = np.array([0, 7, 33, 419])
    assert np.array_equal(mat.cols(cols), a[:, cols])
    rws = np.array([2, 150, 299])
    assert np.array_equal(mat.rows_t(rws), a[rws].T)
    assert np.array_equal(mat.full_rows(10, 20), a[10:20])


def test_movie_like_statistics():
    spec = workloads.movie_like(2000, 3000, 0.01, seed=3)
    assert spec.nnz == round(0.01 * 2000 * 3000)
    v = spec.sp.data
    assert set(np.unique(v)) <= {1.0, 2.0, 3.0, 4.0, 5.0}
    deg = np.diff(spec.sp.indptr)
    assert deg.max() > 8 * np.median(deg)  # heavy-tailed degrees
    # canonical CSR: strictly ascending columns within every row
    d = np.diff(spec.sp.indices.astype(np.int64))
    starts = spec.sp.indptr[1:-1]
    mask = np.ones(d.size, dtype=bool)
    mask[starts[(starts > 0) & (starts < spec.nnz)] - 1] = False
    assert np.all(d[mask] > 0)


def test_newsgroup_like_statistics():
    spec = workloads.newsgroup_like(1500, 4000, 0.005, seed=2)
    assert spec.nnz == round(0.005 * 1500 * 4000)
    assert np.all(spec.sp.data >= 1.0) and np.all(spec.sp.data == np.rint(spec.sp.data))


@pytest.mark.parametrize("follow_up,weight,wp", [("kmeans", "const", 0.0), ("hard", "pow", 2.0), ("leverage", "const", 0.0)])
def test_sparse_sketch_is_above_the_optimum(follow_up, weight, wp):
    spec = _small(seed=4)
    k = 12
    res = oc.cabs(spec, oc.Params.square(k, seed=1, follow_up=follow_up, weight_kind=weight, weight_param=wp))
    a = spec.sp.toarray()
    s = np.linalg.svd(a, compute_uv=False)
    optimum = math.sqrt((s[k:] ** 2).sum() / (s ** 2).sum())
    err = oc.rel_error_exact(Matrix(spec), res.C, res.Umid, res.Rt)
    assert err == pytest.approx(np.linalg.norm(a - oc.reconstruct(res)) / np.linalg.norm(a), rel=1e-10)
    assert err >= optimum * (1 - 1e-12)


def test_sparse_exact_rank_input_is_recovered():
    rng = np.random.default_rng(5)
    g = rng.normal(size=(60, 4)) * (rng.random((60, 1)) < 0.5)
    h = rng.normal(size=(80, 4)) * (rng.random((80, 1)) < 0.5)
    a = g @ h.T
    r, c = np.nonzero(a)
    spec = workloads.sparse_matrix(r, c, a[r, c], 60, 80, "rank4-sparse")
    # pilot of 12 (half the rows and columns are zero), follow-up of the 6 heaviest rows and columns
    res = oc.cabs(spec, oc.Params(12, 12, 6, 6, seed=0, sketch_kind="pseudo_skeleton", follow_up="hard",
                                  weight_kind="pow", weight_param=2.0))
    assert oc.rel_error_exact(Matrix(spec), res.C, res.Umid, res.Rt) < 1e-10
