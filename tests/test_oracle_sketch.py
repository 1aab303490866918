"""Pins for the oracle's entry access, sketching routine and orthogonalisation (CPU only)."""
import math

import numpy as np
import pytest

import workloads
from oracle import cabs as oc
from oracle import philox
from oracle.matrices import Matrix


def test_lowrank_entries_by_brute_force():
    spec = workloads.lowrank_noise(9, 7, 4, seed=1, noise_std=0.25)
    mat = Matrix(spec)
    cols = np.array([0, 3, 6])
    c = mat.cols(cols)
    for i in range(9):
        for a, j in enumerate(cols):
            sig = sum(spec.pf[i, t] * spec.s[t] * spec.qf[j, t] for t in range(4))
            sd = int(spec.noise_seed)
            w = [int(v) for v in philox.philox4x32(np.uint64(i), np.uint64(0), np.uint64(j), np.uint64(0),
                                                   np.uint64(sd & 0xFFFFFFFF), np.uint64(sd >> 32))]
            u1 = ((((w[1] << 32) | w[0]) >> 11) + 1) / 2.0**53
            u2 = (((w[3] << 32) | w[2]) >> 11) / 2.0**53
            g = math.sqrt(-2 * math.log(u1)) * math.cos(2 * math.pi * u2)
            assert c[i, a] == pytest.approx(sig + 0.25 * g, rel=1e-13, abs=1e-15)
    rt = mat.rows_t(np.array([2, 5]))
    assert rt.shape == (7, 2)
    assert np.allclose(rt[:, 1], mat.entries(np.full(7, 5), np.arange(7)), rtol=1e-14)


def test_rbf_entries_by_brute_force():
    spec = workloads.rbf_mixture(12, 3, 2, 1.0, 0.5, seed=2)
    mat = Matrix(spec)
    c = mat.cols(np.array([1, 4]))
    for i in range(12):
        for a, j in enumerate([1, 4]):
            d2 = sum((spec.x[i, t] - spec.y[j, t]) ** 2 for t in range(3))
            assert c[i, a] == pytest.approx(math.exp(-d2 / (2 * spec.sigma**2)), rel=1e-14)
    assert np.allclose(np.diag(mat.full_rows(0, 12)), 1.0)


def test_entry_counter_counts_rows_and_columns():
    spec = workloads.exact_rank(20, 30, 3, seed=0)
    mat = Matrix(spec, track=True)
    mat.cols(np.array([1, 2]))
    mat.rows_t(np.array([5, 6, 7]))
    assert mat.entries_read == 20 * 2 + 30 * 3
    assert mat.mask.sum() == 20 * 2 + 30 * 3 - 2 * 3


def _sample(spec, ir, ic):
    mat = Matrix(spec)
    c = mat.cols(ic)
    rt = mat.rows_t(ir)
    return mat, c, rt, c[ir, :]


def test_pseudo_skeleton_recovers_exact_rank_input():
    spec = workloads.exact_rank(60, 45, 6, seed=3)
    ir = philox.floyd_sample(60, 6, 0, 0)
    ic = philox.floyd_sample(45, 6, 0, 1)
    _, c, rt, w = _sample(spec, ir, ic)
    sk = oc.sketching(c, rt, w, 60, 45, kind="pseudo_skeleton")
    approx = c @ sk.Umid @ rt.T
    assert np.linalg.norm(spec.a - approx) / np.linalg.norm(spec.a) < 1e-12
    # the factor form describes the same matrix
    assert np.allclose(sk.U @ np.diag(sk.S) @ sk.V.T, approx, atol=1e-10 * np.abs(approx).max())


def test_pseudo_skeleton_truncates_rank_deficient_w():
    # rank 4 input, 7 samples: W has rank 4, the rest is dropped, still exact.
    spec = workloads.exact_rank(50, 40, 4, seed=9)
    ir = philox.floyd_sample(50, 7, 1, 0)
    ic = philox.floyd_sample(40, 7, 1, 1)
    _, c, rt, w = _sample(spec, ir, ic)
    sk = oc.sketching(c, rt, w, 50, 40, kind="pseudo_skeleton")
    assert sk.keep.sum() == 4
    assert np.linalg.norm(spec.a - c @ sk.Umid @ rt.T) / np.linalg.norm(spec.a) < 1e-10


def test_stabilized_recovers_block_replicated_input():
    """A = B kron 1: one row and column per block gives C v_i = sigma_i (u_i kron 1),
    so N_c = sigma sqrt(t_r), N_r = sigma sqrt(t_c), S = sigma sqrt(mn)/k and the
    stabilised product equals A exactly."""
    k, tr, tc = 5, 4, 3
    spec = workloads.block_replicated(k, tr, tc, seed=4)
    ir = np.arange(k) * tr + np.array([0, 1, 3, 2, 0])
    ic = np.arange(k) * tc + np.array([2, 0, 1, 1, 0])
    m, n = k * tr, k * tc
    _, c, rt, w = _sample(spec, ir, ic)
    sk = oc.sketching(c, rt, w, m, n)
    approx = c @ sk.Umid @ rt.T
    assert np.linalg.norm(spec.a - approx) / np.linalg.norm(spec.a) < 1e-13
    assert np.allclose(sk.nc, sk.sw * math.sqrt(tr), rtol=1e-12)
    assert np.allclose(sk.nr, sk.sw * math.sqrt(tc), rtol=1e-12)


def test_stabilized_rank_one_closed_form():
    """A = x y^T: the sketch is A |x_I| |y_J| sqrt(mn) / (k |x| |y|)."""
    rng = np.random.default_rng(0)
    m, n, k = 40, 30, 5
    x = rng.normal(size=m)
    y = rng.normal(size=n)
    spec = workloads.dense_matrix(np.outer(x, y))
    ir = philox.floyd_sample(m, k, 7, 0)
    ic = philox.floyd_sample(n, k, 7, 1)
    _, c, rt, w = _sample(spec, ir, ic)
    sk = oc.sketching(c, rt, w, m, n)
    assert sk.keep.sum() == 1
    factor = np.linalg.norm(x[ir]) * np.linalg.norm(y[ic]) * math.sqrt(m * n) / (k * np.linalg.norm(x) * np.linalg.norm(y))
    assert np.allclose(c @ sk.Umid @ rt.T, factor * spec.a, rtol=1e-12, atol=1e-14)
    assert sk.S[0] == pytest.approx(sk.sw[0] * math.sqrt(m * n) / k, rel=1e-14)


def test_stabilized_factors_and_scale_rectangular_samples():
    spec = workloads.config("rbf2000", scale=0.05)[0]
    m = spec.m
    ir = philox.floyd_sample(m, 8, 2, 0)
    ic = philox.floyd_sample(m, 5, 2, 1)
    _, c, rt, w = _sample(spec, ir, ic)
    sk = oc.sketching(c, rt, w, m, m)
    assert np.allclose(np.linalg.norm(sk.U, axis=0), 1.0) and np.allclose(np.linalg.norm(sk.V, axis=0), 1.0)
    assert np.allclose(sk.S, sk.sw[sk.keep] * math.sqrt(m * m / (8 * 5)), rtol=1e-14)
    assert np.allclose(sk.U @ np.diag(sk.S) @ sk.V.T, c @ sk.Umid @ rt.T, atol=1e-12)
    # U lies in the span of C, V in the span of R^T
    for basis, f in ((c, sk.U), (rt, sk.V)):
        coef, *_ = np.linalg.lstsq(basis, f, rcond=None)
        assert np.allclose(basis @ coef, f, atol=1e-10)


def test_zero_matrix_raises_rank_error():
    spec = workloads.dense_matrix(np.zeros((10, 8)))
    _, c, rt, w = _sample(spec, np.arange(3), np.arange(3))
    with pytest.raises(oc.RankError):
        oc.sketching(c, rt, w, 10, 8)


def test_svd_canonical_signs_and_order():
    rng = np.random.default_rng(1)
    w = rng.normal(size=(6, 4))
    u, s, v = oc.svd_canonical(w)
    assert np.allclose(u * s @ v.T, w)
    assert np.all(np.diff(s) <= 0)
    piv = np.argmax(np.abs(u), axis=0)
    assert np.all(u[piv, np.arange(4)] > 0)
    u2, s2, v2 = oc.svd_canonical(-w)
    assert np.allclose(u2, u) and np.allclose(v2, -v)


def test_orthogonalize_is_exact_svd_of_the_product():
    rng = np.random.default_rng(2)
    m, n, k = 70, 50, 6
    u = rng.normal(size=(m, k))
    u /= np.linalg.norm(u, axis=0)
    v = rng.normal(size=(n, k))
    v /= np.linalg.norm(v, axis=0)
    s = np.sort(rng.uniform(0.5, 3.0, size=k))[::-1]
    uo, so, vo = oc.orthogonalize(u, s, v)
    dense = u @ np.diag(s) @ v.T
    assert np.allclose(uo.T @ uo, np.eye(k), atol=1e-13)
    assert np.allclose(vo.T @ vo, np.eye(k), atol=1e-13)
    assert np.allclose(uo @ np.diag(so) @ vo.T, dense, atol=1e-13)
    assert np.allclose(so, np.linalg.svd(dense, compute_uv=False)[:k], rtol=1e-13)
