"""Full-size GPU checks of the configurations the benchmark times (through the C ABI).

At these sizes the oracle cannot run a whole sketch inside a test, so this
file checks what it can compute one by one:
  * pilot indices, bit-exact with the oracle's sampler;
  * single entries of the follow-up C and R^T against the oracle's entry
    function;
  * the sketching routine re-run by the oracle on the GPU's own follow-up
    samples, compared through the CUR product at sampled entries;
  * the sampled error, recomputed by the oracle on the GPU's factors at the
    same Philox samples;
and properties that hold at any size (sorted distinct in-range indices, W̄ the
same block whether read from C̄ or from R̄ᵀ, finite diagnostics).
"""
import numpy as np
import pytest

import workloads
from oracle import cabs as oc
from oracle import philox
from oracle.matrices import Matrix

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    from paper_1607_07395_amd import api as a
    return a


def _sketch(api, name, seed, ns, compute="f32"):
    spec, cfg = workloads.config(name)
    k, iters = cfg["k"], cfg["iters"]
    mat = api.DeviceMatrix(spec, storage="f32")
    prm = api.make_params(k, k, k, k, kmeans_iters=iters, compute=compute, seed=seed)
    res = api.sketch(mat, prm)
    e3 = api.error(mat, prm, res, ns, seed=seed + 1000)
    torch.cuda.synchronize()
    return spec, k, prm, res, e3


def _indices(spec, k, prm, res):
    m, n = spec.m, spec.n
    assert np.array_equal(res.pilot_r.cpu().numpy(), philox.floyd_sample(m, k, prm.seed, 0))
    assert np.array_equal(res.pilot_c.cpu().numpy(), philox.floyd_sample(n, k, prm.seed, 1))
    ir, ic = res.idx_r.cpu().numpy(), res.idx_c.cpu().numpy()
    for idx, hi in ((ir, m), (ic, n)):
        assert idx.size == k and idx[0] >= 0 and idx[-1] < hi and np.all(np.diff(idx) > 0)
    return ir, ic


def _entries(spec, res, ir, ic, tol, wtol=1e-5):
    M = Matrix(spec)
    rng = np.random.default_rng(7)
    k = ir.size
    rows = rng.integers(0, spec.m, 4000)
    pos = rng.integers(0, k, 4000)
    got = res.C[torch.from_numpy(rows).cuda(), torch.from_numpy(pos).cuda()].double().cpu().numpy()
    ref = M.entries(rows, ic[pos])
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    cols = rng.integers(0, spec.n, 4000)
    got = res.Rt[torch.from_numpy(cols).cuda(), torch.from_numpy(pos).cuda()].double().cpu().numpy()
    ref = M.entries(ir[pos], cols)
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    # W̄ read from C̄ (rows idx_r) and from R̄ᵀ (rows idx_c) is the same block of A, up to
    # the FP32 rounding of two separately evaluated copies of each entry
    w_c = res.C[res.idx_r].double().cpu().numpy()
    w_r = res.Rt[res.idx_c].double().cpu().numpy().T
    assert np.abs(w_c - w_r).max() <= wtol * np.abs(w_c).max()


def _error(spec, res, e3, ns, seed):
    """The GPU's sampled error against the oracle's arithmetic at the same samples and factors."""
    M = Matrix(spec)
    i, j = philox.error_sample_indices(spec.m, spec.n, ns, seed)
    a = M.entries(i, j)
    ci = res.C[torch.from_numpy(i).cuda()].double().cpu().numpy()
    rj = res.Rt[torch.from_numpy(j).cuda()].double().cpu().numpy()
    umid = res.Umid.cpu().numpy()
    at = np.einsum("tk,tk->t", ci @ umid, rj)
    num, den = float(((a - at) ** 2).sum()), float((a * a).sum())
    g = e3.cpu().numpy()
    assert g[1] == pytest.approx(den, rel=1e-6)
    assert g[0] == pytest.approx(num, rel=1e-3)
    assert g[2] == pytest.approx(np.sqrt(num / den), rel=1e-3)


@pytest.mark.skip(reason="written for a row-wise sampled-error kernel for RBF sources and k up to 512 that was "
                         "taken out: the profiling run of the version that had it ended with the GPU box faulted, "
                         "and no cause was found in the code; kept off the GPU until one is")
@pytest.mark.parametrize("name,scale,k,compute", [
    ("rbf1e6", 0.55, 300, "f32"),      # 550000 points, d = 64: one column stripe, two 256-element segments
    ("rbf1e6", 0.02, 100, "bf16"),     # 20000 points: eight stripes, one segment, BF16 R^T
    ("rbf2000", 4.0, 270, "f32"),      # d = 10: element loads, two segments
    ("rbf2000", 4.0, 40, "f16"),       # d = 10, one segment, FP16 R^T
    ("lowrank1e5", 0.1, 300, "f32"),   # low rank, r = 200, two segments
])
def test_sampled_error_row_kernel(api, name, scale, k, compute):
    """Sampled errors with at least one sample per row (the bucketed path) on RBF and low-rank sources,
    against the oracle's arithmetic at the same samples and factors."""
    spec, _ = workloads.config(name, scale)
    ns = spec.m + 1000
    mat = api.DeviceMatrix(spec, storage="f32")
    prm = api.make_params(k, k, k, k, kmeans_iters=3, compute=compute, seed=4)
    res = api.sketch(mat, prm)
    e3 = api.error(mat, prm, res, ns, seed=77)
    torch.cuda.synchronize()
    assert res.diagnostics()["status"] == 0
    _error(spec, res, e3, ns, seed=77)


def test_lowrank_1e5_x_2e4_rank200_fullsize(api):
    ns = 100_000
    spec, k, prm, res, e3 = _sketch(api, "lowrank1e5", seed=3, ns=ns)
    ir, ic = _indices(spec, k, prm, res)
    _entries(spec, res, ir, ic, tol=1e-4)
    _error(spec, res, e3, ns, seed=prm.seed + 1000)
    # the follow-up sketching routine, re-run by the oracle on the GPU's own samples
    c = res.C.double().cpu().numpy()
    rt = res.Rt.double().cpu().numpy()
    sk = oc.sketching(c, rt, c[ir], spec.m, spec.n)
    rng = np.random.default_rng(11)
    i, j = rng.integers(0, spec.m, 20000), rng.integers(0, spec.n, 20000)
    gpu = np.einsum("tk,tk->t", c[i] @ res.Umid.cpu().numpy(), rt[j])
    ref = np.einsum("tk,tk->t", c[i] @ sk.Umid, rt[j])
    assert np.abs(gpu - ref).max() <= 1e-4 * np.sqrt(np.mean(ref * ref))
    d = res.diagnostics()
    assert d["rank_final"] == int(sk.keep.sum())


# Per compute type: entry tolerance relative to max |A| (the value's rounding plus the evaluation's,
# FP32 accumulation over d = 64), the same for two evaluated copies of W-bar, and the CUR product's
# deviation from the oracle's sketching routine on the GPU's own samples relative to the rms entry
# (the GPU forms C-bar V_w and the norms with V_w rounded to the compute type: 32 / 4 roundoffs of FP32 / BF16,
# the bounds of the reduced-precision sketch test; measured 1e-8 and 2.3e-3).
FULL_TOL = {"f32": (1e-5, 1e-5, 32 * 2.0 ** -24), "bf16": (8e-3, 8e-3, 4 * 2.0 ** -8)}


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_rbf_1e6_x_1e6_d64_k500_fullsize(api, compute):
    """The headline configuration in the precisions the benchmark serves: pilot indices bit-exact,
    sampled entries, the sampled error recomputed by the oracle, and the follow-up sketching routine
    re-run by the oracle on the GPU's own 10^6 x 500 samples."""
    ns = 50_000
    spec, k, prm, res, e3 = _sketch(api, "rbf1e6", seed=1, ns=ns, compute=compute)
    tol_e, tol_w, tol_p = FULL_TOL[compute]
    ir, ic = _indices(spec, k, prm, res)
    _entries(spec, res, ir, ic, tol=tol_e, wtol=tol_w)
    _error(spec, res, e3, ns, seed=prm.seed + 1000)
    d = res.diagnostics()
    assert 0 < d["rank_final"] <= k and np.isfinite(d["sigma1_final"])
    c = res.C.double().cpu().numpy()
    rt = res.Rt.double().cpu().numpy()
    sk = oc.sketching(c, rt, c[ir], spec.m, spec.n)
    rng = np.random.default_rng(12)
    i, j = rng.integers(0, spec.m, 20000), rng.integers(0, spec.n, 20000)
    gpu = np.einsum("tk,tk->t", c[i] @ res.Umid.cpu().numpy(), rt[j])
    ref = np.einsum("tk,tk->t", c[i] @ sk.Umid, rt[j])
    dev = np.abs(gpu - ref).max() / np.sqrt(np.mean(ref * ref))
    print(f"rbf1e6 {compute}: CUR product deviation {dev:.3g} of the rms entry, ranks {d['rank_final']} / "
          f"{int(sk.keep.sum())}")
    assert dev <= tol_p
