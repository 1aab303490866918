"""cabs_kmeans_noalloc, the allocation-free variant of cabs_kmeans, against cabs_kmeans itself.

The two entry points run the same kernels; the variant takes its scratch from the library's
fixed per-device array instead of a caller workspace.  Its outputs (centres, labels, objective,
snapped rows) must be bitwise those of cabs_kmeans, on consecutive calls that share the array,
the second with a smaller input (so stale contents of a larger call are present)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _inputs(rows, dim, k, seed, dtype):
    rng = np.random.default_rng(seed)
    cen = rng.normal(scale=3.0, size=(max(k // 2, 1), dim))
    p = cen[rng.integers(0, cen.shape[0], rows)] + rng.normal(size=(rows, dim))
    P = torch.from_numpy(p).to(dtype).cuda()
    w = torch.from_numpy(np.linalg.norm(p, axis=1)).cuda()
    pick = torch.from_numpy(np.sort(rng.choice(rows, k, replace=False))).cuda()
    z0 = P[pick].double().contiguous()
    return P, w, z0


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16, torch.float64])
def test_noalloc_matches_the_workspace_entry_point(dtype):
    from paper_1607_07395_amd import api
    for rows, dim, k, iters, seed in [(60_000, 200, 200, 3, 1), (7_000, 40, 33, 2, 2)]:
        P, w, z0 = _inputs(rows, dim, k, seed, dtype)
        print(f"cabs_kmeans_noalloc {dtype} rows={rows} dim={dim} k={k} iters={iters}", flush=True)
        got = api.kmeans_noalloc(P, w, z0, iters)
        want = api.kmeans(P, w, z0, iters)
        torch.cuda.synchronize()
        for name, a, b in zip(("Z", "labels", "obj2", "snap"), got, want):
            assert torch.equal(a, b), name


def test_noalloc_rejects_problems_beyond_its_scratch():
    from paper_1607_07395_amd import api
    from paper_1607_07395_amd import _ffi as F
    rows, dim, k = 1_000_000, 504, 500
    assert F.lib().cabs_kmeans_workspace_bytes(rows, dim, k, F.BF16) > F.KMEANS_NOALLOC_SCRATCH_BYTES
    P = torch.empty(rows, dim, dtype=torch.bfloat16, device="cuda")
    w = torch.ones(rows, dtype=torch.float64, device="cuda")
    z0 = torch.zeros(k, dim, dtype=torch.float64, device="cuda")
    with pytest.raises(F.CabsError) as ei:
        api.kmeans_noalloc(P, w, z0, 1)
    assert ei.value.status == F.ENOMEM
    assert b"fixed array" in F.lib().cabs_last_error()
