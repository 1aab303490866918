"""The continuous-batching server on the GPU (through the C ABI).

Each request's result is compared with the same request run alone on the
default stream: indices, factors and the sampled error must be bitwise equal
(every kernel is deterministic and touches only the request's own buffers).
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ERR_SAMPLES = 200_000


@pytest.fixture(scope="module")
def api():
    from paper_1607_07395_amd import api as a
    return a


@pytest.fixture(scope="module")
def requests(api):
    recs = workloads.request_stream(n_requests=8, qps=1e3, seed=5, m_range=(1_000, 30_000), ks=(16, 32, 64, 128))
    computes = ["f32", "bf16", "f16", "f32"]
    out = []
    for i, rec in enumerate(recs):
        spec = workloads.request_matrix(rec)
        k = min(rec["k"], spec.m, spec.n)
        prm = api.make_params(k, k, k, k, kmeans_iters=3, compute=computes[i % 4], seed=rec["seed"])
        out.append((api.DeviceMatrix(spec, storage="f32"), prm))
    return out


def _alone(api, mat, prm):
    res = api.alloc_result(mat, prm)
    api.sketch(mat, prm, out=res)
    e3 = api.error(mat, prm, res, ERR_SAMPLES, seed=prm.seed + 1)
    torch.cuda.synchronize()
    return res, e3


def _same(a, b):
    for name in ("idx_r", "idx_c", "pilot_r", "pilot_c", "C", "Rt", "Umid"):
        x, y = getattr(a, name), getattr(b, name)
        assert torch.equal(x, y), name


def test_results_alone_and_in_the_mix(api, requests):
    alone = [_alone(api, mat, prm) for mat, prm in requests]
    srv = api.Server(0, hbm_budget_bytes=4 << 30, max_slots=4)
    try:
        outs, errs, tickets = [], [], []
        for mat, prm in requests:
            res = api.alloc_result(mat, prm)
            e3 = torch.zeros(3, dtype=torch.float64, device="cuda")
            tickets.append(srv.submit(mat, prm, res, err_samples=ERR_SAMPLES, err_seed=prm.seed + 1, err_out=e3))
            outs.append(res)
            errs.append(e3)
        srv.drain()
        for t in tickets:
            assert srv.poll(t) >= 0.0
    finally:
        srv.close()
    for (ra, ea), rm, em in zip(alone, outs, errs):
        _same(ra, rm)
        assert torch.equal(ea, em)
        assert np.isfinite(em.cpu().numpy()).all()


def test_admission_by_footprint(api, requests):
    need = max(api.workspace_bytes(mat, prm) for mat, prm in requests)
    # a pool that holds one request at a time: the rest wait for memory, then run
    srv = api.Server(0, hbm_budget_bytes=need + need // 2, max_slots=4)
    try:
        outs, tickets = [], []
        for mat, prm in requests[:4]:
            res = api.alloc_result(mat, prm)
            tickets.append(srv.submit(mat, prm, res))
            outs.append(res)
        srv.drain()
        for t in tickets:
            assert srv.poll(t) >= 0.0
        for (mat, prm), res in zip(requests[:4], outs):
            ref, _ = _alone(api, mat, prm)
            _same(ref, res)
        # a request that can never fit is rejected at submission
        mat, prm = max(requests, key=lambda r: api.workspace_bytes(*r))
        small = api.Server(0, hbm_budget_bytes=api.workspace_bytes(mat, prm) // 2, max_slots=1)
        try:
            with pytest.raises(api.F.CabsError) as ei:
                small.submit(mat, prm, api.alloc_result(mat, prm))
            assert ei.value.status == api.F.ENOMEM
        finally:
            small.close()
    finally:
        srv.close()


def test_cancel_queued_request(api, requests):
    need = max(api.workspace_bytes(mat, prm) for mat, prm in requests)
    srv = api.Server(0, hbm_budget_bytes=need + need // 2, max_slots=1)
    try:
        tickets = []
        for mat, prm in requests[:5]:
            tickets.append(srv.submit(mat, prm, api.alloc_result(mat, prm)))
        assert srv.cancel(tickets[-1]) == api.F.OK  # still queued behind the others
        srv.drain()
        for t in tickets[:-1]:
            assert srv.poll(t) >= 0.0
        with pytest.raises(api.F.CabsError) as ei:
            srv.poll(tickets[-1])
        assert ei.value.status == api.F.ECANCELED
    finally:
        srv.close()


def _diag_equal(a, b):
    da, db = a.diag.cpu().numpy(), b.diag.cpu().numpy()
    assert np.array_equal(da, db, equal_nan=True)


def _shape_class(api, compute, k, follow_up="kmeans", seeds=(3, 4, 5, 6)):
    """Same-shape requests on matrices of different sizes and kinds (uneven m, n)."""
    recs = workloads.request_stream(n_requests=len(seeds), qps=1e3, seed=11, m_range=(2_000, 20_000), ks=(k,))
    out = []
    for rec, sd in zip(recs, seeds):
        spec = workloads.request_matrix(rec)
        prm = api.make_params(k, k, k, k, kmeans_iters=3, compute=compute, seed=sd, follow_up=follow_up)
        out.append((api.DeviceMatrix(spec, storage="f64" if compute == "f64" else "f32"), prm))
    return out


@pytest.mark.parametrize("compute,k,follow_up,count", [
    ("f32", 64, "kmeans", 4),      # pivoted Cholesky route: one SVD item per request
    ("bf16", 240, "kmeans", 4),    # p > 204: step-per-launch Cholesky, SVDs of 4 requests per launch
    ("f64", 20, "leverage", 3),    # the one-work-group SVD (p < 24)
    ("f32", 48, "pilot", 2),       # the pilot sketch alone: one SVD per request
    ("bf16", 400, "kmeans", 3),    # k >= 384: the QR-preconditioned SVDs, items from per-request pointers
])
def test_sketch_batch_is_bitwise_the_single_sketch(api, compute, k, follow_up, count):
    """cabs_sketch_batch: the same-shape requests share each SVD launch; every output (indices,
    C, R^T, U_mid, diagnostics) equals cabs_sketch's bit for bit."""
    reqs = _shape_class(api, compute, k, follow_up, seeds=tuple(range(7, 7 + count)))
    alone = []
    for mat, prm in reqs:
        res = api.sketch(mat, prm)
        torch.cuda.synchronize()
        alone.append(res)
    batch = api.sketch_batch([m for m, _ in reqs], [p for _, p in reqs])
    torch.cuda.synchronize()
    for a, b in zip(alone, batch):
        _same(a, b)
        _diag_equal(a, b)


def test_server_groups_same_shape_requests(api):
    """Eight same-shape requests submitted at once to a 4-slot server (groups of up to 4 form when
    several are admitted together): each result, and its sampled error, equals the request run
    alone; the same with grouping turned off."""
    reqs = _shape_class(api, "f32", 32, seeds=tuple(range(20, 28)))
    alone = [_alone(api, mat, prm) for mat, prm in reqs]
    for gmax in (4, 1):
        srv = api.Server(0, hbm_budget_bytes=4 << 30, max_slots=4)
        try:
            srv.set_group(gmax)
            outs, errs, tickets = [], [], []
            for mat, prm in reqs:
                res = api.alloc_result(mat, prm)
                e3 = torch.zeros(3, dtype=torch.float64, device="cuda")
                tickets.append(srv.submit(mat, prm, res, err_samples=ERR_SAMPLES, err_seed=prm.seed + 1, err_out=e3))
                outs.append(res)
                errs.append(e3)
            srv.drain()
            for t in tickets:
                assert srv.poll(t) >= 0.0
        finally:
            srv.close()
        for (ra, ea), rm, em in zip(alone, outs, errs):
            _same(ra, rm)
            assert torch.equal(ea, em)
