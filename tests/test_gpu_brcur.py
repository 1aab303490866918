"""GPU parity of the bilateral resampling CUR (Algorithm 1) and the pilot sketch alone, against the
FP64 oracle, through the C ABI.

* Samples: cabs_sample's base (streams 0 / 1) and target (streams 7 / 8) indices equal the oracle's.
* FP64: the CUR product C Umid R at 2e4 sampled entries within tol of the rms entry, where
  tol = 1e-12 + 20 eps kappa_c kappa_r: the product's first-order sensitivity to relative
  perturbations of Cbar, M and Rbar is bounded by the condition numbers of the two
  pseudo-inverses over their kept components (kappa = sigma_1 / sigma_min kept; kappa_r = 1
  when the target is the base sample, where W^+ enters once); the kept ranks equal the oracle's
  (after checking that no singular value lies within 1e-6 relative of the cut).
* Reduced precision: the sampled error close to the oracle's.
* The error of a result through cabs_error equals the oracle's on the same entries.
"""
import numpy as np
import pytest

import workloads
from oracle import brcur as ob
from oracle import cabs as oc
from oracle import philox
from oracle.matrices import Matrix
from sketch_checks import approx_at, oracle_params, run

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def api():
    from paper_1607_07395_amd import api as a
    return a


def _np(t):
    return t.detach().float().cpu().numpy() if t.dtype in (torch.bfloat16, torch.float16) else t.detach().cpu().numpy()


def _kappa_and_margin(a, rtol, cap=0):
    """Condition number over the kept components and the smallest relative distance of a singular
    value from the cut (the oracle's truncation rule)."""
    s = np.linalg.svd(a, compute_uv=False)
    tol = (rtol if rtol > 0 else max(a.shape) * EPS) * s[0]
    keep = s > tol
    if cap:
        keep &= np.arange(s.size) < cap
    kept = s[keep]
    margin = np.min(np.abs(s - tol) / s[0]) if not cap else 1.0
    return kept[0] / kept[-1], margin


def _spec(name, scale):
    if name == "scene":
        return workloads.natural_scene_like(int(6480 * scale), int(7680 * scale), seed=1)
    if name == "movie":
        return workloads.movie_like(3000, 4600, 0.08, seed=1)
    return workloads.config(name, scale)[0]


def _check_f64(api, spec, ref, res, rtol, same):
    a_full = Matrix(spec)
    br = ref.base_r
    cbar = ref.C[br, :] if same else ref.C[ref.tgt_r, :]
    kc, mc = _kappa_and_margin(cbar, rtol)
    if same:
        kr, mr = 1.0, mc
    else:
        kr, mr = _kappa_and_margin(ref.Rt[ref.tgt_c, :].T, rtol)
    assert min(mc, mr) > 1e-6, (mc, mr)
    d = res.diagnostics()
    assert d["status"] == 0
    assert d["rank_c"] == ref.rank_c and d["rank_r"] == ref.rank_r
    assert d["sigma1_c"] == pytest.approx(ref.sigma1_c, rel=1e-12)
    assert d["sigma1_r"] == pytest.approx(ref.sigma1_r, rel=1e-12)
    C, Rt, Umid = _np(res.C), _np(res.Rt), _np(res.Umid)
    amax = max(np.abs(ref.C).max(), np.abs(ref.Rt).max())
    assert np.abs(C - ref.C).max() <= 1e-12 * amax and np.abs(Rt - ref.Rt).max() <= 1e-12 * amax
    i, j = philox.error_sample_indices(spec.m, spec.n, 20000, seed=98)
    scale = np.sqrt(np.mean(a_full.entries(i, j) ** 2))
    diff = np.abs(approx_at(C, Umid, Rt, i, j) - approx_at(ref.C, ref.Umid, ref.Rt, i, j)).max() / scale
    tol = 1e-12 + 20 * EPS * kc * kr
    print(f"{spec.name}: kappa_c {kc:.3g} kappa_r {kr:.3g} product diff {diff:.3g} (tol {tol:.3g})")
    assert diff <= tol
    return tol


@pytest.mark.parametrize("name,scale,kbr,kbc,ktr,ktc,seed,rtol", [
    ("lowrank1e5", 0.05, 37, 50, 111, 150, 0, 0.0),
    ("lowrank1e5s", 0.05, 64, 40, 200, 97, 1, 0.0),
    ("rbf2000", 1.0, 40, 40, 120, 120, 2, 1e-8),
    ("scene", 0.1, 30, 33, 90, 99, 3, 1e-10),
    ("movie", 1.0, 40, 45, 120, 135, 4, 0.0),
])
def test_brcur_general_f64(api, name, scale, kbr, kbc, ktr, ktc, seed, rtol):
    spec = _spec(name, scale)
    br, bc = ob.base_sample(spec, kbr, kbc, seed)
    tr, tc = ob.target_sample(spec, ktr, ktc, seed)
    ref = ob.br_cur(spec, br, bc, tr, tc, pinv_rtol=rtol)
    mat = api.DeviceMatrix(spec, storage="f64")
    g = [api.sample(n, k, seed, s) for n, k, s in ((spec.m, kbr, 0), (spec.n, kbc, 1), (spec.m, ktr, 7),
                                                   (spec.n, ktc, 8))]
    for got, want in zip(g, (br, bc, tr, tc)):
        assert np.array_equal(got.cpu().numpy(), want)
    res = api.brcur(mat, *g, compute="f64", pinv_rtol=rtol)
    torch.cuda.synchronize()
    tol = _check_f64(api, spec, ref, res, rtol, same=False)
    # the error metric on the result: a residual perturbed by at most tol of the rms entry moves the
    # relative error by at most tol
    e = float(api.error(mat, res.params, res, 2_000_000, seed=3)[2].item())
    want = oc.rel_error_sampled(Matrix(spec), ref.C, ref.Umid, ref.Rt, 2_000_000, 3)[0]
    assert abs(e - want) <= tol + 1e-12 * want


@pytest.mark.parametrize("method,name,scale,k,seed,rtol", [
    ("pseudo_skeleton", "lowrank1e5", 0.05, 45, 0, 0.0),
    ("pseudo_skeleton", "scene", 0.1, 37, 1, 1e-10),
    ("nystrom", "rbf2000", 1.0, 60, 2, 1e-8),
    ("nystrom", "rbf2000", 0.5, 25, 3, 1e-6),
])
def test_brcur_same_sample_f64(api, method, name, scale, k, seed, rtol):
    spec = _spec(name, scale)
    if method == "nystrom":
        ref = ob.nystrom(spec, k, seed, pinv_rtol=rtol)
    else:
        ref = ob.pseudo_skeleton(spec, k, k + 3, seed, pinv_rtol=rtol)
    mat = api.DeviceMatrix(spec, storage="f64")
    if method == "nystrom":
        res = api.nystrom(mat, k, seed, compute="f64", pinv_rtol=rtol)
    else:
        res = api.pseudo_skeleton(mat, k, k + 3, seed, compute="f64", pinv_rtol=rtol)
    torch.cuda.synchronize()
    assert np.array_equal(res.base_r.cpu().numpy(), ref.base_r)
    assert np.array_equal(res.base_c.cpu().numpy(), ref.base_c)
    _check_f64(api, spec, ref, res, rtol, same=True)


def test_nystrom_rank_cap_f64(api):
    """The supplementary stability figure's knob: W^+ from the r largest singular values only.
    The error falls monotonically in r on the PSD kernel matrix (the Schur complement property
    the oracle pins), and every capped factor matches the oracle."""
    spec = _spec("rbf2000", 0.5)
    mat = api.DeviceMatrix(spec, storage="f64")
    errs = []
    for r in (1, 2, 4, 8, 16, 24):
        ref = ob.nystrom(spec, 30, 5, pinv_rtol=1e-8, rank_cap=r)
        res = api.nystrom(mat, 30, 5, compute="f64", pinv_rtol=1e-8, rank_cap=r)
        torch.cuda.synchronize()
        assert res.diagnostics()["rank_c"] == ref.rank_c
        kappa, _ = _kappa_and_margin(ref.C[ref.base_r, :], 1e-8, cap=r)
        C, Rt, Umid = _np(res.C), _np(res.Rt), _np(res.Umid)
        i, j = philox.error_sample_indices(spec.m, spec.n, 20000, seed=4)
        scale = np.sqrt(np.mean(Matrix(spec).entries(i, j) ** 2))
        diff = np.abs(approx_at(C, Umid, Rt, i, j) - approx_at(ref.C, ref.Umid, ref.Rt, i, j)).max() / scale
        assert diff <= 1e-12 + 20 * EPS * kappa, (r, diff, kappa)
        errs.append(float(api.error(mat, res.params, res, 0)[2].item()))
    assert all(b <= a * (1 + 1e-9) for a, b in zip(errs, errs[1:])), errs


@pytest.mark.parametrize("name,scale,k,seed", [("lowrank1e5", 0.05, 50, 0), ("rbf2000", 1.0, 48, 1),
                                               ("scene", 0.1, 33, 3), ("movie", 1.0, 40, 2)])
def test_pilot_follow_up_f64(api, name, scale, k, seed):
    """follow_up = pilot: the output is the pilot sketch (step 2 of Algorithm 2) on the pilot sample."""
    spec = _spec(name, scale)
    kw = dict(k1_rows=k, k1_cols=k + 2, k2_rows=k, k2_cols=k + 2, seed=seed, follow_up="pilot")
    prm_o = oracle_params(kw)
    prm_o.follow_up = "pilot"
    ref = oc.cabs(spec, prm_o)
    mat, prm, res = run(api, spec, kw, "f64")
    d = res.diagnostics()
    assert d["status"] == 0
    assert np.array_equal(res.idx_r.cpu().numpy(), ref.idx_r) and np.array_equal(res.idx_c.cpu().numpy(), ref.idx_c)
    assert np.array_equal(res.pilot_r.cpu().numpy(), ref.pilot_rows)
    assert d["rank_final"] == d["rank_pilot"] == int(ref.final.keep.sum())
    assert d["sigma1_final"] == pytest.approx(ref.final.sw[0], rel=1e-12)
    e = float(api.error(mat, prm, res, 0)[2].item())
    want = oc.rel_error_exact(Matrix(spec), ref.C, ref.Umid, ref.Rt)
    sw = ref.final.sw[ref.final.keep]
    if np.min(-np.diff(sw) / sw[1:]) < 1e-8:
        # Repeated singular values of W (the sparse integer input has them): the stabilised routine
        # scales each singular pair by its own extrapolated norms, which depend on the basis chosen
        # inside the repeated subspace, so the factor is not unique; the rest is checked above.
        print(f"{spec.name}: repeated singular values of W; error {e:.4g} (oracle {want:.4g})")
        assert np.isfinite(e)
        return
    i, j = philox.error_sample_indices(spec.m, spec.n, 20000, seed=97)
    sc = np.sqrt(np.mean(Matrix(spec).entries(i, j) ** 2))
    C, Rt, Umid = res.C.cpu().numpy(), res.Rt.cpu().numpy(), res.Umid.cpu().numpy()
    assert np.abs(approx_at(C, Umid, Rt, i, j) - approx_at(ref.C, ref.Umid, ref.Rt, i, j)).max() <= 1e-10 * sc
    assert e == pytest.approx(want, rel=1e-10)


@pytest.mark.parametrize("compute,ratio_bound", [("f32", 1.01), ("bf16", 1.1)])
def test_sketch_cur_reduced_precision(api, compute, ratio_bound):
    """FP32 / BF16 Sketch-CUR on the scaled-signal low-rank workload at 2e4 x 4e3 (base 100, target
    300; the oracle's error is 0.14 there): the sampled error within a factor of the FP64 oracle's."""
    spec = _spec("lowrank1e5s", 0.2)
    ref = ob.sketch_cur(spec, 100, 100, seed=6, pinv_rtol=1e-6)
    mat = api.DeviceMatrix(spec, storage="f32")
    res = api.sketch_cur(mat, 100, 100, 6, compute=compute, pinv_rtol=1e-6)
    e = float(api.error(mat, res.params, res, 2_000_000, seed=2)[2].item())
    want = oc.rel_error_sampled(Matrix(spec), ref.C, ref.Umid, ref.Rt, 2_000_000, 2)[0]
    print(f"Sketch-CUR {compute}: error {e:.5g}, oracle {want:.5g}")
    assert e <= ratio_bound * want + 1e-6


def test_sketch_cur_largest_sizes_f32(api):
    """The largest sizes the call takes on one side: base 1024, target 3072 (the three-times rate),
    on a 2e4 x 1.2e4 low-rank input in FP32: tall SVDs of 3072 x 1024, a 3072 x 3072 block; the
    sampled error within 1 % of the FP64 oracle's."""
    spec = workloads.lowrank_noise(20000, 12000, 200, seed=3, noise_std=1e-3, s_kind="inv")
    ref = ob.sketch_cur(spec, 1024, 1024, seed=7, pinv_rtol=1e-6)
    mat = api.DeviceMatrix(spec, storage="f32")
    res = api.sketch_cur(mat, 1024, 1024, 7, compute="f32", pinv_rtol=1e-6)
    d = res.diagnostics()
    assert d["status"] == 0
    e = float(api.error(mat, res.params, res, 2_000_000, seed=1)[2].item())
    want = oc.rel_error_sampled(Matrix(spec), ref.C, ref.Umid, ref.Rt, 2_000_000, 1)[0]
    print(f"Sketch-CUR 1024 / 3072: error {e:.5g}, oracle {want:.5g}, ranks {d['rank_c']} {d['rank_r']}")
    assert abs(e - want) <= 0.01 * want


@pytest.mark.parametrize("rows,cols", [(3000, 300), (300, 3000), (4096, 17), (2500, 1024)])
def test_svd_tall_and_wide(api, rows, cols):
    rng = np.random.default_rng(rows + cols)
    a = rng.normal(size=(rows, cols)) * np.logspace(0, -6, cols)[None, :]
    u, s, v = api.svd(torch.from_numpy(a).cuda())
    u, s, v = u.cpu().numpy(), s.cpu().numpy(), v.cpu().numpy()
    s_ref = np.linalg.svd(a, compute_uv=False)
    assert np.allclose(s, s_ref, rtol=1e-11, atol=1e-13 * s_ref[0])
    assert np.abs(u * s @ v.T - a).max() <= 1e-12 * s_ref[0]
    p = min(rows, cols)
    assert np.abs(u.T @ u - np.eye(p)).max() < 1e-10 and np.abs(v.T @ v - np.eye(p)).max() < 1e-10
