"""GPU parity of the sparse (CSR) source against the FP64 oracle (through the C ABI).

* Gathers: C = A(:, J) and R^T = A(I, :)^T are copies of stored values, so they equal the
  oracle's bit for bit in FP64 and up to the one rounding of each value in FP32.
* Sketches (FP64): for the hard-threshold and leverage variants of Section 5 (the paper
  recommends the hard threshold on sparse inputs), pilot and follow-up indices bit-exact and the
  CUR product to 1e-10 of the rms entry; for the k-means follow-up (Section 3.2), whose ties on
  sparse embeddings are decided by rounding, the pilot stage exactly and the rest as a valid
  sample (the k-means steps are checked one by one in test_gpu_kmeans_paths).
* Errors: the exact error over every entry and the sampled estimate against the oracle's on the
  same entries, to 1e-10.
"""
import numpy as np
import pytest

import workloads
from oracle import cabs as oc
from oracle import philox
from oracle.matrices import Matrix
from sketch_checks import approx_at, oracle_params, run

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    from paper_1607_07395_amd import api as a
    return a


def _np(t):
    return t.detach().float().cpu().numpy() if t.dtype in (torch.bfloat16, torch.float16) else t.detach().cpu().numpy()


# small stand-ins, dense enough (8-10 %) that a pilot sample of 30-40 rows and columns keeps
# most components; the full movie-like shape is the last test
SPARSE = {
    "movie": lambda: workloads.movie_like(3000, 4600, 0.08, seed=1),
    "news": lambda: workloads.newsgroup_like(1877, 6118, 0.1, seed=2),
}


@pytest.mark.parametrize("kind", list(SPARSE))
@pytest.mark.parametrize("compute", ["f64", "f32", "bf16"])
def test_sparse_gathers(api, kind, compute):
    spec = SPARSE[kind]()
    mat = api.DeviceMatrix(spec, storage="f64" if compute == "f64" else "f32")
    om = Matrix(spec)
    rng = np.random.default_rng(3)
    for k in (1, 37, 300):
        ic = np.sort(rng.choice(spec.n, k, replace=False)).astype(np.int64)
        ir = np.sort(rng.choice(spec.m, k, replace=False)).astype(np.int64)
        c = _np(api.eval_cols(mat, torch.from_numpy(ic).cuda(), compute))
        rt = _np(api.eval_rows_t(mat, torch.from_numpy(ir).cuda(), compute))
        cw, rw = om.cols(ic), om.rows_t(ir)
        if compute == "f64":
            assert np.array_equal(c, cw) and np.array_equal(rt, rw)
        else:
            dt = {"f32": torch.float32, "bf16": torch.bfloat16}[compute]
            rc = torch.from_numpy(cw).to(dt).double().numpy()
            rr = torch.from_numpy(rw).to(dt).double().numpy()
            assert np.array_equal(c, rc) and np.array_equal(rt, rr)


@pytest.mark.parametrize("kind,k,seed", [("movie", 40, 0), ("news", 32, 3)])
def test_sparse_sketch_f64_kmeans(api, kind, k, seed):
    """The k-means follow-up on sparse input, end to end in FP64.  Zero embedding rows and
    coinciding pilot rows give exact distance ties that rounding decides (the k-means and snap
    steps are checked with those ties allowed in test_gpu_kmeans_paths), so here: the pilot
    indices and the pilot sketch bit-exact / to 1e-12, a valid follow-up sample (distinct,
    sorted, in range) sharing at least half its rows with the oracle's (trajectories that take a
    tie differently drift apart), and the exact error within 10 % of the oracle's."""
    spec = SPARSE[kind]()
    kw = dict(k1_rows=k, k1_cols=k, k2_rows=k, k2_cols=k, kmeans_iters=5, seed=seed, count_entries=True)
    ref = oc.cabs(spec, oracle_params(kw))
    mat, prm, res = run(api, spec, kw, "f64")
    d = res.diagnostics()
    assert d["status"] == 0
    assert np.array_equal(res.pilot_r.cpu().numpy(), ref.pilot_rows)
    assert np.array_equal(res.pilot_c.cpu().numpy(), ref.pilot_cols)
    assert d["rank_pilot"] == int(ref.pilot.keep.sum())
    assert d["sigma1_pilot"] == pytest.approx(ref.pilot.sw[0], rel=1e-12)
    assert d["enc_r_pilot"] == pytest.approx(ref.km_r.e_initial, rel=1e-9)
    assert d["enc_c_pilot"] == pytest.approx(ref.km_c.e_initial, rel=1e-9)
    assert d["entries"] == ref.entries_touched + 2 * k * k
    for got, want, n in ((res.idx_r, ref.idx_r, spec.m), (res.idx_c, ref.idx_c, spec.n)):
        g = got.cpu().numpy()
        assert np.all(np.diff(g) > 0) and g[0] >= 0 and g[-1] < n
        assert np.isin(g, want).mean() >= 0.5
    e = float(api.error(mat, prm, res, 0)[2].item())
    want = oc.rel_error_exact(Matrix(spec), ref.C, ref.Umid, ref.Rt)
    assert abs(e - want) <= 0.1 * want, (e, want)


@pytest.mark.parametrize("kind,follow_up,k,seed", [("movie", "hard", 40, 1), ("news", "hard", 30, 2),
                                                   ("movie", "leverage", 40, 4), ("news", "leverage", 30, 5)])
def test_sparse_sketch_f64_variants(api, kind, follow_up, k, seed):
    """Section 5's variants on sparse input, POW(2) weights for the hard threshold: indices
    bit-exact (after checking that the k-th and (k+1)-th oracle weights or keys differ by more
    than 1e-9 relative), the CUR product to 1e-10, exact and sampled errors to 1e-10."""
    spec = SPARSE[kind]()
    kw = dict(k1_rows=k, k1_cols=k, k2_rows=k, k2_cols=k, seed=seed)
    if follow_up == "hard":
        kw.update(weight="pow", weight_param=2.0)
    prm = oracle_params(kw)
    prm.follow_up = follow_up
    ref = oc.cabs(spec, prm)
    if follow_up == "hard":
        for w in (ref.w_r, ref.w_c):
            s = np.sort(w)[::-1]
            assert s[k - 1] - s[k] > 1e-9 * s[0]
    mat, gprm, res = run(api, spec, dict(kw, follow_up=follow_up), "f64")
    assert res.diagnostics()["status"] == 0
    assert np.array_equal(res.pilot_r.cpu().numpy(), ref.pilot_rows)
    assert np.array_equal(res.idx_r.cpu().numpy(), ref.idx_r)
    assert np.array_equal(res.idx_c.cpu().numpy(), ref.idx_c)
    C, Rt, Umid = res.C.cpu().numpy(), res.Rt.cpu().numpy(), res.Umid.cpu().numpy()
    i, j = philox.error_sample_indices(spec.m, spec.n, 20000, seed=96)
    sc = np.sqrt(np.mean(Matrix(spec).entries(i, j) ** 2)) + 1e-300
    assert np.abs(approx_at(C, Umid, Rt, i, j) - approx_at(ref.C, ref.Umid, ref.Rt, i, j)).max() <= 1e-10 * \
        max(sc, np.sqrt((spec.sp.data ** 2).sum() / (spec.m * spec.n)))
    e_exact = float(api.error(mat, gprm, res, 0)[2].item())
    want = oc.rel_error_exact(Matrix(spec), ref.C, ref.Umid, ref.Rt)
    assert e_exact == pytest.approx(want, rel=1e-10)
    e_s = float(api.error(mat, gprm, res, 3_000_000, seed=11)[2].item())
    want_s = oc.rel_error_sampled(Matrix(spec), ref.C, ref.Umid, ref.Rt, 3_000_000, 11)[0]
    assert e_s == pytest.approx(want_s, rel=1e-10)
    print(f"{kind} {follow_up}: exact error {e_exact:.5f}, sampled {e_s:.5f}")


def test_sparse_sketch_f32_movie_full_shape(api):
    """The full 27000 x 46000 movie-like stand-in (0.56 % nonzeros) in FP32 at a 1 % sampling rate
    (k = 352), hard threshold with POW(2) weights: the sampled error within 2 % of the FP64
    oracle's on the same entries."""
    spec = workloads.movie_like()
    k = 352
    kw = dict(k1_rows=k, k1_cols=k, k2_rows=k, k2_cols=k, seed=0, weight="pow", weight_param=2.0)
    prm = oracle_params(kw)
    prm.follow_up = "hard"
    ref = oc.cabs(spec, prm)
    mat, gprm, res = run(api, spec, dict(kw, follow_up="hard"), "f32")
    g = res.idx_r.cpu().numpy()
    assert np.isin(g, ref.idx_r).mean() >= 0.98
    e = float(api.error(mat, gprm, res, 10_000_000, seed=1)[2].item())
    want = oc.rel_error_sampled(Matrix(spec), ref.C, ref.Umid, ref.Rt, 10_000_000, 1)[0]
    assert abs(e - want) <= 0.02 * want, (e, want)
    print(f"movie-like 1 %: FP32 error {e:.4f}, oracle {want:.4f}")
