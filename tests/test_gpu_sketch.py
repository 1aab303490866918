"""End-to-end GPU parity of cabs_sketch / cabs_error against the FP64 oracle."""
import math

import numpy as np
import pytest

import workloads
from oracle import cabs as oc
from oracle import philox
from oracle.matrices import Matrix
from sketch_checks import approx_at as _approx_at
from sketch_checks import compare_f64 as _compare_f64
from sketch_checks import oracle_params as _oracle_params
from sketch_checks import run as _run

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    from paper_1607_07395_amd import api as a
    return a


@pytest.mark.parametrize("name,scale,k,wp,seed", [("rbf2000", 1.0, 50, 2.0, 1), ("lowrank1e5s", 0.05, 40, 1.0, 2),
                                                  ("lowrank1e5s", 0.03, 64, 2.0, 4), ("rbf2000", 0.5, 30, 1.0, 3),
                                                  ("lowrank1e5s", 1.0, 24, 2.0, 5)])
def test_sketch_f64_hard_threshold(api, name, scale, k, wp, seed):
    """Hard-threshold follow-up (Section 5 variant) with POW weights: indices bit-exact with the
    oracle (the k-th and (k+1)-th weights differ by > 1e-9 of the largest, so FP64 rounding on
    either side cannot change the choice; 1000-5000 rows cover the LDS-only and the first global
    merge passes of the selection, 10^5 rows (padded to 2^17) six levels of them), the CUR
    product to 1e-10."""
    spec, _ = workloads.config(name, scale)
    kw = dict(k1_rows=k, k1_cols=k, k2_rows=k, k2_cols=k, seed=seed, weight="pow", weight_param=wp)
    mat, prm, res = _run(api, spec, dict(kw, follow_up="hard"), "f64")
    okw = _oracle_params(kw)
    okw.follow_up = "hard"
    ref = oc.cabs(spec, okw)
    for w in (ref.w_r, ref.w_c):
        s = np.sort(w)[::-1]
        assert s[k - 1] - s[k] > 1e-9 * s[0]
    d = res.diagnostics()
    assert d["status"] == 0
    assert np.array_equal(res.idx_r.cpu().numpy(), ref.idx_r)
    assert np.array_equal(res.idx_c.cpu().numpy(), ref.idx_c)
    assert d["enc_r_final"] == 0.0 and d["enc_c_final"] == 0.0
    C, Rt, Umid = res.C.cpu().numpy(), res.Rt.cpu().numpy(), res.Umid.cpu().numpy()
    i, j = philox.error_sample_indices(spec.m, spec.n, 20000, seed=98)
    scale_a = np.sqrt(np.mean(Matrix(spec).entries(i, j) ** 2))
    assert np.abs(_approx_at(C, Umid, Rt, i, j) - _approx_at(ref.C, ref.Umid, ref.Rt, i, j)).max() <= 1e-10 * scale_a
    assert d["rank_final"] == int(ref.final.keep.sum())


@pytest.mark.parametrize("scale,k,seed", [(0.1, 12, 0), (0.2, 20, 3), (0.137, 17, 5)])
def test_sketch_f64_rbf_small(api, scale, k, seed):
    spec, _ = workloads.config("rbf2000", scale)
    _compare_f64(api, spec, dict(k1_rows=k, k1_cols=k, k2_rows=k, k2_cols=k, seed=seed))


def test_sketch_f64_rbf_full_config(api):
    """RBF 2000 x 2000, d = 10, 20 clusters, k = 50, c = 5, FP64, exact error."""
    spec, c = workloads.config("rbf2000")
    kw = dict(k1_rows=50, k1_cols=50, k2_rows=50, k2_cols=50, kmeans_iters=5, seed=0)
    mat, prm, res, ref = _compare_f64(api, spec, kw)
    e = api.error(mat, prm, res, 0).cpu().numpy()
    want = oc.rel_error_exact(Matrix(spec), ref.C, ref.Umid, ref.Rt)
    assert e[2] == pytest.approx(want, rel=1e-10)


def test_sketch_f64_large_p_orthogonalisation(api):
    """p = 256 > 204 components: the orthogonalisation factors both Grams with the step-per-launch
    pivoted Cholesky (the one the 1e6 x 1e6 RBF configuration's k = 500 takes) instead of the
    register-resident one; 3000-point RBF kernel, FP64, follow-up indices bit-exact with the oracle."""
    spec, _ = workloads.config("rbf2000", 1.5)
    _compare_f64(api, spec, dict(k1_rows=256, k1_cols=256, k2_rows=256, k2_cols=256, seed=2))


def test_sketch_f64_qr_preconditioned_svds(api):
    """k = 420 >= 384: the SVDs of W (both rounds) and of K take the QR-preconditioned path
    (Householder QR with column pivoting, then the block-Jacobi SVD of R^T); 3000-point RBF kernel,
    FP64, follow-up indices bit-exact with the oracle."""
    spec, _ = workloads.config("rbf2000", 1.5)
    _compare_f64(api, spec, dict(k1_rows=420, k1_cols=420, k2_rows=420, k2_cols=420, seed=5))


def test_sketch_f64_large_p_rectangular(api):
    """The same with different row and column sample sizes (p = min = 230)."""
    spec = workloads.lowrank_noise(4000, 2500, 260, seed=6, noise_std=1e-2, s_kind="scaled")
    _compare_f64(api, spec, dict(k1_rows=240, k1_cols=230, k2_rows=235, k2_cols=250, seed=4))


@pytest.mark.parametrize("kw", [
    dict(k1_rows=9, k1_cols=7, k2_rows=6, k2_cols=8, seed=2),
    dict(k1_rows=10, k1_cols=10, k2_rows=10, k2_cols=10, orthogonalize=False, seed=1),
    dict(k1_rows=10, k1_cols=10, k2_rows=10, k2_cols=10, sketch="pseudo_skeleton", seed=4),
    dict(k1_rows=12, k1_cols=12, k2_rows=12, k2_cols=12, weight="pow", weight_param=2.0, seed=6),
    dict(k1_rows=8, k1_cols=8, k2_rows=8, k2_cols=8, kmeans_iters=0, seed=7),
])
def test_sketch_f64_options(api, kw):
    spec = workloads.lowrank_noise(700, 400, 15, seed=1, noise_std=1e-2, s_kind="scaled")
    _compare_f64(api, spec, kw)


def test_sketch_dense_source_and_exact_recovery(api):
    spec = workloads.exact_rank(300, 220, 6, seed=4)
    kw = dict(k1_rows=6, k1_cols=6, k2_rows=6, k2_cols=6, sketch="pseudo_skeleton", seed=3)
    mat, prm, res, ref = _compare_f64(api, spec, kw)
    e = api.error(mat, prm, res, 0).cpu().numpy()
    assert e[2] < 1e-11


def test_factor_form_f64(api):
    spec, _ = workloads.config("rbf2000", 0.15)
    kw = dict(k1_rows=14, k1_cols=14, k2_rows=14, k2_cols=14, factors=True, seed=8)
    mat, prm, res, ref = _compare_f64(api, spec, kw)
    u, s, v = ref.factors
    S = res.S.cpu().numpy()
    kept = int(ref.final.keep.sum())
    assert np.allclose(S[:kept], s[:kept], rtol=0, atol=1e-10 * s[0])
    Uf, Vf = res.Uf.cpu().numpy(), res.Vf.cpu().numpy()
    assert np.abs(Uf[:, :kept].T @ Uf[:, :kept] - np.eye(kept)).max() < 1e-9
    gaps = np.abs(np.diff(s[:kept]))
    for j in range(kept):
        g = min(gaps[j - 1] if j > 0 else np.inf, gaps[j] if j < kept - 1 else np.inf)
        if g > 1e-3 * s[0]:
            assert np.abs(Uf[:, j] - u[:, j]).max() < 1e-8, j
            assert np.abs(Vf[:, j] - v[:, j]).max() < 1e-8, j


@pytest.mark.parametrize("m,n,ns", [(900, 500, 100_000),    # bucketed by row, one row per bucket
                                    (900, 500, 600),        # fewer samples than rows: direct gather
                                    (20000, 300, 50_000)])  # bucketed, three rows per bucket
def test_error_sampled_matches_oracle(api, m, n, ns):
    spec = workloads.lowrank_noise(m, n, 20, seed=2, noise_std=1e-2, s_kind="scaled")
    kw = dict(k1_rows=15, k1_cols=15, k2_rows=15, k2_cols=15, seed=1)
    mat, prm, res, ref = _compare_f64(api, spec, kw)
    e = api.error(mat, prm, res, ns, seed=5).cpu().numpy()
    rel, num, den = oc.rel_error_sampled(Matrix(spec), ref.C, ref.Umid, ref.Rt, ns, 5)
    assert e[0] == pytest.approx(num, rel=1e-8) and e[1] == pytest.approx(den, rel=1e-12)
    assert e[2] == pytest.approx(rel, rel=1e-8)


@pytest.mark.parametrize("k,seed", [(270, 7), (288, 8)])
def test_error_exact_with_wide_samples(api, k, seed):
    """k > 256: C U is formed by the FP64 product kernel for rows wider than the register-resident
    one takes (K in stages of 16: 270 gives 17, the last one partial, 288 eighteen full ones); 3000
    rows (23 full 128-row tiles and a ragged one) and k columns (ragged 128-column tiles); the
    exact error against the oracle's."""
    spec, _ = workloads.config("rbf2000", 1.5)
    kw = dict(k1_rows=k, k1_cols=k, k2_rows=k, k2_cols=k, seed=seed)
    mat, prm, res, ref = _compare_f64(api, spec, kw)
    e = api.error(mat, prm, res, 0).cpu().numpy()
    want = oc.rel_error_exact(Matrix(spec), ref.C, ref.Umid, ref.Rt)
    assert e[2] == pytest.approx(want, rel=1e-9)


def test_zero_matrix_reports_rank_loss(api):
    spec = workloads.dense_matrix(np.zeros((100, 80)))
    mat, prm, res = _run(api, spec, dict(k1_rows=5, k1_cols=5, k2_rows=5, k2_cols=5))
    d = res.diagnostics()
    assert d["status"] == -3 and d["rank_pilot"] == 0
    assert np.all(np.isfinite(res.Umid.cpu().numpy()))


def test_determinism_bitwise(api):
    spec, _ = workloads.config("rbf2000", 0.1)
    kw = dict(k1_rows=12, k1_cols=12, k2_rows=12, k2_cols=12, seed=0)
    _, _, r1 = _run(api, spec, kw, "f32")
    _, _, r2 = _run(api, spec, kw, "f32")
    for a, b in [(r1.C, r2.C), (r1.Rt, r2.Rt), (r1.Umid, r2.Umid), (r1.idx_r, r2.idx_r), (r1.diag, r2.diag)]:
        assert torch.equal(a, b)


# Bound on the deviation of the reduced-precision CUR product from the FP64 sketching routine run on
# the same follow-up samples, relative to |A| at the sampled entries, in unit roundoffs of the compute
# type.  In 16-bit compute the stored C-bar and R-bar carry one rounding of the compute type per entry
# (test_eval_cols_and_rows), which dominates: measured 0.82-0.88 roundoffs, bound 4.  In FP32 the
# entry rounding is as small as the rounding of every FP32 product and sum downstream (the k-term
# evaluation sums, the embedding products), and the deviation collects them: measured 7.3-8.1
# roundoffs, bound 32.
U_C = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}
DEV_UNITS = {"f32": 32.0, "bf16": 4.0, "f16": 4.0}


@pytest.mark.parametrize("compute", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("seed", [3, 8])
def test_reduced_precision_against_oracle(api, compute, seed):
    """Reduced precision, end to end on the scaled-signal low-rank workload (3000 x 600, k = 32, so
    that the FP32 and 16-bit fast k-means kernels run):
    * pilot indices bit-exact with the oracle;
    * the CUR product against the oracle's sketching routine (Section 4.1) on the GPU's own
      follow-up samples, within DEV_UNITS[compute] roundoffs of the compute type relative to |A|;
    * the GPU's sampled error estimate against the same ratio recomputed from its factors;
    * the error relative to the oracle's own sketch (its own follow-up samples) is printed: the
      follow-up choice in reduced precision may differ where distances tie within rounding."""
    spec, _ = workloads.config("lowrank1e5s", 0.03)
    k = 32
    kw = dict(k1_rows=k, k1_cols=k, k2_rows=k, k2_cols=k, seed=seed)
    mat, prm, res = _run(api, spec, kw, compute)
    ref = oc.cabs(spec, _oracle_params(kw))
    assert np.array_equal(res.pilot_r.cpu().numpy(), ref.pilot_rows)
    assert np.array_equal(res.pilot_c.cpu().numpy(), ref.pilot_cols)
    ir, ic = res.idx_r.cpu().numpy(), res.idx_c.cpu().numpy()
    om = Matrix(spec)
    cb, rtb = om.cols(ic), om.rows_t(ir)
    sk = oc.sketching(cb, rtb, cb[ir], spec.m, spec.n)
    ns = 200_000
    i, j = philox.error_sample_indices(spec.m, spec.n, ns, 1)
    a = om.entries(i, j)
    na = float(np.linalg.norm(a))
    C = res.C.double().cpu().numpy()
    Rt = res.Rt.double().cpu().numpy()
    a_gpu = _approx_at(C, res.Umid.cpu().numpy(), Rt, i, j)
    a_or = _approx_at(cb, sk.Umid, rtb, i, j)
    dev = float(np.linalg.norm(a_gpu - a_or)) / na
    e_host = float(np.linalg.norm(a - a_gpu)) / na
    e_same = float(np.linalg.norm(a - a_or)) / na
    e = api.error(mat, prm, res, ns, seed=1).cpu().numpy()[2]
    want, _, _ = oc.rel_error_sampled(Matrix(spec), ref.C, ref.Umid, ref.Rt, ns, 1)
    agree = float(np.mean(np.isin(ir, ref.idx_r)))
    print(f"{compute} seed {seed}: deviation {dev:.3e} = {dev / U_C[compute]:.2f} roundoffs; error {e:.5f}, "
          f"oracle on the same samples {e_same:.5f}, oracle's own sketch {want:.5f}; row agreement {agree:.2f}")
    assert dev <= DEV_UNITS[compute] * U_C[compute], dev
    assert e == pytest.approx(e_host, rel=1e-4)
