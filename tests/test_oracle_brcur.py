"""Pins for the oracle's bilateral resampling CUR (Algorithm 1) and its special cases (CPU only).

What fixes these results independently of the oracle's own arithmetic:
* the minimiser of |M - Cbar U Rbar|_F is the minimum-norm least-squares solution of the
  Kronecker system (Rbar^T kron Cbar) vec(U) = vec(M), computed here by LAPACK's lstsq;
* the pseudo-inverse meets the four Penrose conditions, and lstsq against the identity gives it;
* with one sample for both rounds the method is Eq. (W), whose middle factor the oracle's
  sketching routine (pseudo-skeleton kind) also computes, by another route;
* exact recovery of an exactly rank-r input from base samples of rank r (any method of the
  family), and of a rank-r positive semi-definite input by the Nystrom method;
* on a positive semi-definite input the Nystrom residual A - C W^+ C^T is a Schur complement:
  positive semi-definite, zero on the sampled rows and columns, and, as fewer singular vectors
  of W are used, larger in the Loewner order, so its Frobenius norm falls monotonically as the
  number used grows (the stability the supplementary material reports for Nystrom).
"""
import math

import numpy as np
import pytest

import workloads
from oracle import brcur as ob
from oracle import cabs as oc
from oracle import philox
from oracle.matrices import Matrix


def _rank_deficient(rng, m, n, r):
    return rng.normal(size=(m, r)) @ rng.normal(size=(r, n))


@pytest.mark.parametrize("shape,r", [((9, 4), 4), ((7, 7), 3), ((5, 12), 2)])
def test_pinv_penrose_conditions_and_lstsq(shape, r):
    rng = np.random.default_rng(1)
    a = _rank_deficient(rng, *shape, r)
    x, rank, s1 = ob.pinv(a)
    assert rank == r
    assert s1 == pytest.approx(np.linalg.norm(a, 2), rel=1e-12)
    sc = np.abs(a).max()
    assert np.allclose(a @ x @ a, a, atol=1e-11 * sc)
    assert np.allclose(x @ a @ x, x, atol=1e-11 * np.abs(x).max())
    assert np.allclose((a @ x).T, a @ x, atol=1e-11)
    assert np.allclose((x @ a).T, x @ a, atol=1e-11)
    want = np.linalg.lstsq(a, np.eye(shape[0]), rcond=1e-10)[0]
    assert np.allclose(x, want, atol=1e-10 * np.abs(want).max())


def test_pinv_rank_cap_is_the_top_eigenpair():
    rng = np.random.default_rng(2)
    g = rng.normal(size=(6, 6))
    w = g @ g.T
    x, rank, _ = ob.pinv(w, rank_cap=1)
    lam, vec = np.linalg.eigh(w)
    assert rank == 1
    assert np.allclose(x, np.outer(vec[:, -1], vec[:, -1]) / lam[-1], atol=1e-14 / lam[-1] * 10)


def test_general_middle_factor_is_the_min_norm_least_squares_solution():
    spec = workloads.lowrank_noise(60, 50, 5, seed=3, noise_std=0.05)
    br, bc = ob.base_sample(spec, 4, 6, seed=2)
    tr, tc = ob.target_sample(spec, 9, 8, seed=2)
    res = ob.br_cur(spec, br, bc, tr, tc)
    a = Matrix(spec).full_rows(0, spec.m)
    cbar = a[np.ix_(tr, bc)]
    rbar = a[np.ix_(br, tc)]
    m_blk = a[np.ix_(tr, tc)]
    # vec(Cbar U Rbar) = (Rbar^T kron Cbar) vec(U), column-major vec
    sol = np.linalg.lstsq(np.kron(rbar.T, cbar), m_blk.ravel(order="F"), rcond=None)[0]
    want = sol.reshape(bc.size, br.size, order="F")
    assert np.allclose(res.Umid, want, rtol=1e-9, atol=1e-11 * np.abs(want).max())
    # the bases are the sampled columns and rows
    assert np.array_equal(res.C, a[:, bc]) and np.array_equal(res.Rt, a[br, :].T)
    assert res.entries == spec.m * 6 + spec.n * 4 + 9 * 8


def test_same_sample_is_eq_w():
    spec, _ = workloads.config("lowrank1e5s", 0.002)
    res = ob.pseudo_skeleton(spec, 8, 11, seed=4)
    sk = oc.sketching(res.C, res.Rt, res.C[res.base_r, :], spec.m, spec.n, "pseudo_skeleton")
    assert np.allclose(res.Umid, sk.Umid, rtol=1e-9, atol=1e-12 * np.abs(sk.Umid).max())
    # the general formula on explicit copies of the base sample gives the same factor
    gen = ob.br_cur(spec, res.base_r, res.base_c, res.base_r.copy(), res.base_c.copy())
    assert np.allclose(gen.Umid, res.Umid, rtol=1e-8, atol=1e-10 * np.abs(res.Umid).max())
    assert res.entries == spec.m * 11 + spec.n * 8


def test_distinct_entries_read():
    spec = workloads.lowrank_noise(40, 30, 3, seed=1)
    br, bc = ob.base_sample(spec, 5, 4, seed=0)
    tr, tc = ob.target_sample(spec, 15, 12, seed=0)
    mat = Matrix(spec, track=True)
    mat.cols(bc)
    mat.rows_t(br)
    mat.block(tr, tc)
    want = np.zeros((40, 30), bool)
    want[:, bc] = True
    want[br, :] = True
    want[np.ix_(tr, tc)] = True
    assert np.array_equal(mat.mask, want)


@pytest.mark.parametrize("method", ["sketch_cur", "pseudo_skeleton"])
def test_exact_rank_input_is_recovered(method):
    """(The stabilised pilot sketch rescales the singular values by sqrt(mn / (kr kc)) and is not
    exact on such input, so it is not in this list.)"""
    spec = workloads.exact_rank(80, 64, 5, seed=7)
    if method == "sketch_cur":
        res = ob.sketch_cur(spec, 6, 7, seed=1)
    else:
        res = ob.pseudo_skeleton(spec, 6, 7, seed=1)
    assert res.rank_c == 5 and res.rank_r == 5
    assert oc.rel_error_exact(Matrix(spec), res.C, res.Umid, res.Rt) < 1e-10


def test_nystrom_recovers_a_rank_r_psd_matrix():
    rng = np.random.default_rng(5)
    g = rng.normal(size=(70, 4))
    spec = workloads.dense_matrix(g @ g.T)
    res = ob.nystrom(spec, 9, seed=3)
    assert res.rank_c == 4
    assert np.array_equal(res.base_r, res.base_c)
    assert oc.rel_error_exact(Matrix(spec), res.C, res.Umid, res.Rt) < 1e-10
    with pytest.raises(ValueError):
        ob.nystrom(workloads.exact_rank(10, 12, 2, seed=0), 3, seed=0)


def test_nystrom_residual_is_a_schur_complement():
    spec, _ = workloads.config("rbf2000", 0.1)
    a = Matrix(spec).full_rows(0, spec.m)
    k = 25
    res = ob.nystrom(spec, k, seed=6, pinv_rtol=1e-10)
    resid = a - res.C @ res.Umid @ res.Rt.T
    i = res.base_c
    assert np.abs(resid[i, :]).max() < 1e-8 and np.abs(resid[:, i]).max() < 1e-8
    ev = np.linalg.eigvalsh(0.5 * (resid + resid.T))
    assert ev.min() > -1e-8 * np.abs(ev).max()
    # fewer singular vectors: a residual larger in the Loewner order, so a larger Frobenius norm
    errs = []
    for r in range(1, res.rank_c + 1):
        rr = ob.nystrom(spec, k, seed=6, pinv_rtol=1e-10, rank_cap=r)
        errs.append(np.linalg.norm(a - rr.C @ rr.Umid @ rr.Rt.T))
    assert all(e1 <= e0 * (1 + 1e-9) for e0, e1 in zip(errs, errs[1:])), errs


def test_every_method_is_above_the_optimum():
    spec, _ = workloads.config("lowrank1e5s", 0.002)
    a = Matrix(spec).full_rows(0, spec.m)
    s = np.linalg.svd(a, compute_uv=False)
    k = 12
    optimum = math.sqrt((s[k:] ** 2).sum() / (s ** 2).sum())
    for res in (ob.sketch_cur(spec, k, k, 0), ob.pseudo_skeleton(spec, k, k, 0), ob.pilot_sketch(spec, k, k, 0)):
        err = oc.rel_error_exact(Matrix(spec), res.C, res.Umid, res.Rt)
        assert optimum * (1 - 1e-12) <= err < 10.0


def test_sample_streams():
    spec = workloads.lowrank_noise(500, 400, 3, seed=0)
    res = ob.sketch_cur(spec, 20, 30, seed=9)
    assert np.array_equal(res.base_r, philox.floyd_sample(500, 20, 9, philox.STREAM_PILOT_ROWS))
    assert np.array_equal(res.base_c, philox.floyd_sample(400, 30, 9, philox.STREAM_PILOT_COLS))
    assert np.array_equal(res.tgt_r, philox.floyd_sample(500, 60, 9, philox.STREAM_TARGET_ROWS))
    assert np.array_equal(res.tgt_c, philox.floyd_sample(400, 90, 9, philox.STREAM_TARGET_COLS))
    # the pilot sketch uses the same base sample as the other one-shot methods
    pil = ob.pilot_sketch(spec, 20, 30, seed=9)
    assert np.array_equal(pil.base_r, res.base_r) and np.array_equal(pil.base_c, res.base_c)
    # the target size saturates at the dimension
    small = workloads.lowrank_noise(50, 40, 3, seed=0)
    r2 = ob.sketch_cur(small, 20, 15, seed=1)
    assert r2.tgt_r.size == 50 and r2.tgt_c.size == 40


def test_pilot_follow_up_is_step_two():
    spec, _ = workloads.config("rbf2000", 0.1)
    res = oc.cabs(spec, oc.Params.square(15, seed=2, follow_up="pilot"))
    full = oc.cabs(spec, oc.Params.square(15, seed=2))
    assert np.array_equal(res.idx_r, full.pilot_rows) and np.array_equal(res.idx_c, full.pilot_cols)
    assert np.array_equal(res.Umid, full.pilot.Umid)
    with pytest.raises(ValueError):
        oc.cabs(spec, oc.Params(15, 15, 16, 15, follow_up="pilot"))
