"""GPU parity of the leverage-score follow-up (Section 5's leverage variant) against the FP64 oracle.

FP64: follow-up indices bit-exact with the oracle whenever the k-th and (k+1)-th largest oracle
keys differ by more than 1e-9 of the k-th (the scores and keys agree to ~1e-13 relative, so no
rounding on either side can swap them; the margin is asserted first), and the CUR product to
1e-10 of the rms entry.  Reduced precision: the keys come from the rounded embedding, so only
the draws near the boundary may differ; the indices must be a valid sample and agree with the
oracle's on most rows.
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


def _keys(ref, prm, side):
    """The oracle's keys on one side (the same definition as its leverage_sample)."""
    if side == "r":
        emb, n, stream = ref.P, ref.P.shape[0], philox.STREAM_LEVERAGE_ROWS
    else:
        emb, n, stream = ref.Q, ref.Q.shape[0], philox.STREAM_LEVERAGE_COLS
    so = ref.pilot_sigma
    p1 = min(prm.k1_rows, prm.k1_cols)
    keep = so > p1 * oc.EPS * so.max()
    sc = (emb[:, keep] ** 2 / so[keep]).sum(1)
    u = philox.unit_draws(n, prm.seed, stream)
    with np.errstate(divide="ignore"):
        return np.where(sc > 0, np.log(u) / np.where(sc > 0, sc, 1.0), -np.inf)


def _oracle(spec, kw):
    prm = oracle_params(kw)
    prm.follow_up = "leverage"
    return prm, oc.cabs(spec, prm)


@pytest.mark.parametrize("name,scale,k1,k2,ortho,seed", [
    ("rbf2000", 1.0, 50, 50, True, 0), ("rbf2000", 0.5, 30, 40, True, 1), ("rbf2000", 0.5, 30, 20, False, 2),
    ("lowrank1e5s", 0.05, 40, 40, True, 3), ("lowrank1e5s", 0.03, 64, 48, False, 4),
    ("lowrank1e5s", 1.0, 200, 200, True, 0)])
def test_sketch_f64_leverage(api, name, scale, k1, k2, ortho, seed):
    spec, _ = workloads.config(name, scale)
    kw = dict(k1_rows=k1, k1_cols=k1, k2_rows=k2, k2_cols=k2, seed=seed, orthogonalize=ortho)
    prm_o, ref = _oracle(spec, kw)
    for side, k in (("r", k2), ("c", k2)):
        key = np.sort(_keys(ref, prm_o, side))[::-1]
        assert key[k - 1] - key[k] > 1e-9 * abs(key[k - 1]), (side, key[k - 1], key[k])
    mat, prm, res = run(api, spec, dict(kw, follow_up="leverage"), "f64")
    d = res.diagnostics()
    assert d["status"] == 0
    assert np.array_equal(res.pilot_r.cpu().numpy(), ref.pilot_rows)
    assert np.array_equal(res.idx_r.cpu().numpy(), ref.idx_r)
    assert np.array_equal(res.idx_c.cpu().numpy(), ref.idx_c)
    assert d["enc_r_final"] == 0.0 and d["enc_c_final"] == 0.0
    C, Rt, Umid = res.C.cpu().numpy(), res.Rt.cpu().numpy(), res.Umid.cpu().numpy()
    i, j = philox.error_sample_indices(spec.m, spec.n, 20000, seed=97)
    sc = np.sqrt(np.mean(Matrix(spec).entries(i, j) ** 2))
    assert np.abs(approx_at(C, Umid, Rt, i, j) - approx_at(ref.C, ref.Umid, ref.Rt, i, j)).max() <= 1e-10 * sc
    assert d["rank_final"] == int(ref.final.keep.sum())


@pytest.mark.parametrize("compute,agree", [("f32", 0.95), ("bf16", 0.7)])
def test_sketch_reduced_precision_leverage(api, compute, agree):
    """FP32 / BF16 leverage follow-up on the scaled-signal low-rank workload (1e4 x 2e3, k = 40):
    distinct sorted indices in range, agreement with the FP64 oracle's sample, and an error close
    to the oracle's (sampled entries of the exact error)."""
    spec, _ = workloads.config("lowrank1e5s", 0.1)
    kw = dict(k1_rows=40, k1_cols=40, k2_rows=40, k2_cols=40, seed=6)
    _, ref = _oracle(spec, kw)
    mat, prm, res = run(api, spec, dict(kw, follow_up="leverage"), compute)
    for got, want, n in ((res.idx_r, ref.idx_r, spec.m), (res.idx_c, ref.idx_c, spec.n)):
        g = got.cpu().numpy()
        assert np.all(np.diff(g) > 0) and g[0] >= 0 and g[-1] < n
        assert np.isin(g, want).mean() >= agree, (np.isin(g, want).mean(), compute)
    e = float(api.error(mat, prm, res, 2_000_000, seed=5)[2].item())
    want = oc.rel_error_sampled(Matrix(spec), ref.C, ref.Umid, ref.Rt, 2_000_000, 5)[0]
    assert e <= 1.5 * want + 1e-3, (e, want)
    print(f"{compute}: error {e:.4g} against the oracle's {want:.4g}")
