"""Shared checks of a GPU sketch against the FP64 oracle (imported by the GPU test modules)."""
import numpy as np
import pytest

from oracle import cabs as oc
from oracle import philox
from oracle.matrices import Matrix


def run(api, spec, prm_kw, compute="f64", storage=None):
    import torch
    storage = storage or ("f64" if compute == "f64" else "f32")
    mat = api.DeviceMatrix(spec, storage=storage)
    prm = api.make_params(compute=compute, **prm_kw)
    res = api.sketch(mat, prm)
    torch.cuda.synchronize()
    return mat, prm, res


def oracle_params(kw):
    kw = dict(kw)
    kw.pop("count_entries", None)
    return oc.Params(kw.pop("k1_rows"), kw.pop("k1_cols"), kw.pop("k2_rows"), kw.pop("k2_cols"),
                     kmeans_iters=kw.pop("kmeans_iters", 5), weight_kind=kw.pop("weight", "const"),
                     weight_param=kw.pop("weight_param", 0.0), sketch_kind=kw.pop("sketch", "stabilized"),
                     orthogonalize=kw.pop("orthogonalize", True), pinv_rtol=kw.pop("pinv_rtol", 0.0),
                     seed=kw.pop("seed", 0), factors=kw.pop("factors", False))


def approx_at(C, Umid, Rt, i, j):
    return np.einsum("tk,tk->t", (C[i] @ Umid), Rt[j])


def compare_f64(api, spec, kw, tol=1e-10, ref=None):
    """FP64 GPU sketch against the oracle: pilot and follow-up indices bit-exact, C and R^T to
    1e-12 of max |A|, the CUR product at 2e4 sampled entries to `tol` of the rms entry, and the
    diagnostics (kept ranks, encoding errors, cluster sizes, sigma_1, and the device count of
    entries evaluated: m k_c + n k_r per round, W's k_r k_c entries twice)."""
    kw = dict(kw, count_entries=True)
    mat, prm, res = run(api, spec, kw, "f64")
    if ref is None:
        ref = oc.cabs(spec, oracle_params(kw))
    d = res.diagnostics()
    assert d["status"] == 0
    assert np.array_equal(res.pilot_r.cpu().numpy(), ref.pilot_rows)
    assert np.array_equal(res.pilot_c.cpu().numpy(), ref.pilot_cols)
    assert np.array_equal(res.idx_r.cpu().numpy(), ref.idx_r), (d["gap_r"], ref.km_r.min_gap)
    assert np.array_equal(res.idx_c.cpu().numpy(), ref.idx_c), (d["gap_c"], ref.km_c.min_gap)
    C, Rt, Umid = res.C.cpu().numpy(), res.Rt.cpu().numpy(), res.Umid.cpu().numpy()
    amax = max(np.abs(ref.C).max(), np.abs(ref.Rt).max())
    assert np.abs(C - ref.C).max() <= 1e-13 * amax * 10
    assert np.abs(Rt - ref.Rt).max() <= 1e-13 * amax * 10
    # the CUR product at sampled entries
    i, j = philox.error_sample_indices(spec.m, spec.n, 20000, seed=99)
    a_gpu = approx_at(C, Umid, Rt, i, j)
    a_ref = approx_at(ref.C, ref.Umid, ref.Rt, i, j)
    scale = np.sqrt(np.mean(Matrix(spec).entries(i, j) ** 2))
    assert np.abs(a_gpu - a_ref).max() <= tol * scale
    # diagnostics
    assert d["rank_pilot"] == int(ref.pilot.keep.sum()) and d["rank_final"] == int(ref.final.keep.sum())
    k1r, k1c, k2r, k2c = kw["k1_rows"], kw["k1_cols"], kw["k2_rows"], kw["k2_cols"]
    assert d["entries"] == ref.entries_touched + k1r * k1c + k2r * k2c
    assert d["enc_r_pilot"] == pytest.approx(ref.km_r.e_initial, rel=1e-9)
    assert d["enc_r_final"] == pytest.approx(ref.km_r.e_final, rel=1e-9)
    assert d["enc_c_pilot"] == pytest.approx(ref.km_c.e_initial, rel=1e-9)
    assert d["enc_c_final"] == pytest.approx(ref.km_c.e_final, rel=1e-9)
    assert d["tmax_r"] == ref.km_r.max_cluster and d["tmax_c"] == ref.km_c.max_cluster
    assert d["sigma1_pilot"] == pytest.approx(ref.pilot.sw[0], rel=1e-12)
    return mat, prm, res, ref
