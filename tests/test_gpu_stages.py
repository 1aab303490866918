"""GPU parity of the individual stages against the FP64 oracle (through the C ABI)."""
import math

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


def _np(t):
    return t.detach().float().cpu().numpy() if t.dtype in (torch.bfloat16, torch.float16) else t.detach().cpu().numpy()


@pytest.mark.parametrize("n,k,seed,sid", [(1, 1, 0, 0), (10, 10, 3, 1), (1000, 50, 0, 0), (2000, 50, 7, 1),
                                         (10**6, 500, 1, 0), (10**6, 4096, 2, 3), (97, 96, 5, 2),
                                         (2**40, 33, 9, 4)])
def test_sample_bit_exact(api, n, k, seed, sid):
    got = api.sample(n, k, seed, sid).cpu().numpy()
    want = philox.floyd_sample(n, k, seed, sid)
    assert np.array_equal(got, want)


def _idx(n, k, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=k, replace=False)).astype(np.int64)


SPECS = {
    "lowrank": lambda: workloads.lowrank_noise(301, 257, 37, seed=3, noise_std=0.05),
    "rbf": lambda: workloads.rbf_mixture(301, 10, 5, 2.0, 1.0, seed=4),
    "rbf_rect": lambda: workloads.MatrixSpec(kind="rbf", m=300, n=170, x=np.random.default_rng(1).normal(size=(300, 7)),
                                              y=np.random.default_rng(2).normal(size=(170, 7)), sigma=2.5),
    "dense": lambda: workloads.dense_matrix(np.random.default_rng(5).normal(size=(290, 333))),
}


U_OUT = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}
U32 = 2.0 ** -24


def _noise_draw_bound(spec, rows, cols, compute):
    """Bound on the error of the standard normal g = r cos(2 pi u2), r = sqrt(-2 ln u1), as the
    evaluation kernel draws it.  FP64: a few ulp.  Reduced precisions: u1 rounded to FP32 and the
    FP32 logarithm change r^2 by at most 2^-23 + 8 u r^2, so r by min(2^-11.5, that / r); the
    cosine takes the top 24 bits of u2 (2 pi 2^-24) through the hardware cosine (2^-20 absolute);
    the square root and products add 4 u of |g|."""
    rr = np.asarray(rows, dtype=np.uint64)[:, None]
    cc = np.asarray(cols, dtype=np.uint64)[None, :]
    g = np.abs(philox.normal_at(spec.noise_seed, rr, cc))
    if compute == "f64":
        return 64 * U_OUT["f64"] * (g + 1.0)
    m32 = np.uint64(0xFFFFFFFF)
    sd = np.uint64(spec.noise_seed)
    w = philox.philox4x32(rr & m32, rr >> np.uint64(32), cc & m32, cc >> np.uint64(32), sd & m32,
                          sd >> np.uint64(32))
    u1 = philox.to_unit_open0((w[1] << np.uint64(32)) | w[0])
    r = np.sqrt(-2.0 * np.log(u1))
    dr2 = 2.0 ** -23 + 8 * U32 * r * r
    dr = np.minimum(2.0 ** -11.5, dr2 / np.maximum(r, 1e-300))
    return dr + r * (2 * np.pi * 2.0 ** -24 + 2.0 ** -20) + 4 * U32 * g


def _eval_bound(spec, rows, cols, compute):
    """Per-entry rounding bound of the evaluated A[rows, cols] (FP32 tables for the reduced
    precisions, FP64 tables for FP64), derived from the arithmetic of the evaluation kernel:

    * the tables are the FP64 values rounded to the storage type (relative u_s each);
    * MFMA operands are the table values rounded to the compute type (16-bit: relative u_c; the
      low-rank scale s is multiplied into the gathered factor in FP32 first), products of
      16-bit operands are exact in FP32, and the K-term sums accumulate in FP32 (FP64 for FP64):
      K u_a relative to the sum of |terms|;
    * low rank: |error| <= (2 u_c + 3 u_s + (K + 2) u_a) sum_t |pf_it s_t qf_jt| plus the noise
      draw (Box-Muller in FP32 with hardware sqrt and cos: 16 ulp of a value below 8) plus, in
      FP16, 2^-25 per term for operands below the normal range (_noise_draw_bound for the draw);
    * RBF: d2 = |x|^2 + |y|^2 - 2 x.y with the norms from the storage values in the accumulation
      type and the dot product from compute-type operands, so
      |dd2| <= (K + 4) u_a (|x|^2 + |y|^2) + 2 (2 u_c + 2 u_s + (K + 2) u_a) sum_t |x_t y_t|;
      then |dv| <= exp(-max(d2 - dd2, 0) / (2 sigma^2)) dd2 / (2 sigma^2) plus 8 ulp of the exponential
      and the rounding of its argument (3 u_a d2 / (2 sigma^2) relative);
    * the result is rounded to the compute type: u_c of the value (FP16 values below its normal
      range: 2^-25 absolute).
    Dense sources are copied, so their only error is the two roundings."""
    c = compute
    u_s = U_OUT["f64"] if c == "f64" else U32
    u_c = 0.0 if c in ("f64", "f32") else U_OUT[c]
    u_a = U_OUT["f64"] if c == "f64" else U32
    u_o = U_OUT[c]
    om = Matrix(spec)
    a = om._block(rows, cols)
    if spec.kind == "dense":  # FP16 below its normal range: absolute spacing 2^-24
        return (u_s + u_o) * np.abs(a) + (2.0 ** -25 if c == "f16" else 1e-300)
    if spec.kind == "lowrank":
        K = spec.r
        terms = np.abs(spec.pf[rows] * spec.s) @ np.abs(spec.qf[cols]).T
        noise = spec.noise_std * _noise_draw_bound(spec, rows, cols, c)
        sub = K * 2.0 ** -25 * np.abs(spec.pf).max() if c == "f16" else 0.0
        e = (2 * u_c + 3 * u_s + (K + 2) * u_a) * terms + noise + sub
        return e + u_o * (np.abs(a) + e) + (2.0 ** -25 if c == "f16" else 0.0)
    K = spec.d
    x, y = spec.x[rows], spec.y[cols]
    xn = (x * x).sum(1)[:, None]
    yn = (y * y).sum(1)[None, :]
    dots = np.abs(x) @ np.abs(y).T
    dd2 = (K + 4) * u_a * (xn + yn) + 2 * (2 * u_c + 2 * u_s + (K + 2) * u_a) * dots
    d2 = np.maximum(xn + yn - 2 * x @ y.T, 0.0)
    inv = 1.0 / (2 * spec.sigma ** 2)
    # the exponential: a few ulp, plus the rounding of its argument (relative u_a of d2 / (2 sigma^2))
    e = np.exp(-np.maximum(d2 - dd2, 0.0) * inv) * dd2 * inv + (8 + 3 * d2 * inv) * u_a * a
    return e + u_o * (a + e)


@pytest.mark.parametrize("kind", list(SPECS))
@pytest.mark.parametrize("compute", ["f64", "f32", "bf16", "f16"])
def test_eval_cols_and_rows(api, kind, compute):
    """C = A(:, J) and R^T = A(I, :)^T against the oracle's entries, every entry within its
    derived rounding bound (_eval_bound); the largest ratio error / bound is printed."""
    spec = SPECS[kind]()
    storage = "f64" if compute == "f64" else "f32"
    mat = api.DeviceMatrix(spec, storage=storage)
    om = Matrix(spec)
    worst = 0.0
    for k, seed in [(1, 0), (17, 1), (130, 2)]:
        ic = _idx(spec.n, min(k, spec.n), seed)
        ir = _idx(spec.m, min(k, spec.m), seed + 10)
        c = _np(api.eval_cols(mat, torch.from_numpy(ic).cuda(), compute))
        rt = _np(api.eval_rows_t(mat, torch.from_numpy(ir).cuda(), compute))
        cw, rw = om.cols(ic), om.rows_t(ir)
        assert c.shape == cw.shape and rt.shape == rw.shape
        bc = _eval_bound(spec, np.arange(spec.m), ic, compute)
        br = _eval_bound(spec, ir, np.arange(spec.n), compute).T
        rc = np.abs(c - cw) / bc
        rr = np.abs(rt - rw) / br
        assert rc.max() <= 1.0, (kind, compute, k, float(rc.max()))
        assert rr.max() <= 1.0, (kind, compute, k, float(rr.max()))
        worst = max(worst, float(rc.max()), float(rr.max()))
    print(f"{kind} {compute}: largest error / bound {worst:.3f}")


@pytest.mark.parametrize("compute", ["f64", "f32", "bf16"])
def test_dense_gathers_at_stand_in_size(api, compute):
    """Dense gathers (C = A(:, J) row by row, R^T = A(I, :)^T through LDS tiles) on the full
    6480 x 7680 natural-scene-like stand-in with 700 sampled rows and columns (ragged against the
    64 x 64 tiles): a gather is a copy, so every entry equals the oracle's value rounded to the
    storage type and then to the compute type."""
    spec = workloads.natural_scene_like(6480, 7680, seed=3)
    storage = "f64" if compute == "f64" else "f32"
    mat = api.DeviceMatrix(spec, storage=storage)
    om = Matrix(spec)
    ic = _idx(spec.n, 700, 5)
    ir = _idx(spec.m, 700, 6)
    c = api.eval_cols(mat, torch.from_numpy(ic).cuda(), compute).cpu()
    rt = api.eval_rows_t(mat, torch.from_numpy(ir).cuda(), compute).cpu()
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[compute]

    def rounded(a):
        t = torch.from_numpy(a if compute == "f64" else a.astype(np.float32))
        return t.to(tdt)

    assert torch.equal(c, rounded(om.cols(ic)))
    assert torch.equal(rt, rounded(om.rows_t(ir)))


def test_eval_cols_over_several_launches(api):
    """More than 2^20 blocks of 64 rows: the evaluation runs as several launches, each a
    contiguous range of row blocks.  A 2^26 + 4000-point RBF matrix (d = 2), FP32, 7 sampled
    columns; rows on both sides of the launch boundary, the first and last rows and a random
    sample are checked against the oracle's entries within the derived bound."""
    m = (1 << 26) + 4000
    rng = np.random.default_rng(31)
    spec = workloads.MatrixSpec(kind="rbf", m=m, n=500, x=rng.normal(size=(m, 2)), y=rng.normal(size=(500, 2)),
                                sigma=1.5)
    mat = api.DeviceMatrix(spec, storage="f32")
    ic = _idx(spec.n, 7, 3)
    c = api.eval_cols(mat, torch.from_numpy(ic).cuda(), "f32")
    edge = 1 << 26
    rows = np.unique(np.concatenate([np.arange(0, 50), np.arange(edge - 200, edge + 200), np.arange(m - 50, m),
                                     rng.integers(0, m, size=2000)]))
    got = c[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
    del c, mat
    want = Matrix(spec).block(rows, ic)
    bound = _eval_bound(spec, rows, ic, "f32")
    assert (np.abs(got - want) / bound).max() <= 1.0


@pytest.mark.parametrize("rows,cols,seed", [(1, 1, 0), (5, 3, 1), (3, 5, 2), (50, 50, 3), (64, 40, 4), (40, 64, 5),
                                            (200, 200, 6), (129, 200, 7), (300, 257, 8), (500, 500, 9),
                                            (64, 700, 10), (1024, 23, 11), (700, 400, 12), (400, 1000, 13),
                                            (1024, 384, 14)])
def test_svd_against_lapack(api, rows, cols, seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(rows, cols)) * np.exp(-0.2 * np.arange(cols))[None, :]
    U, S, V = (x.cpu().numpy() for x in api.svd(torch.from_numpy(a).cuda()))
    u0, s0, v0 = oc.svd_canonical(a)
    p = min(rows, cols)
    assert np.allclose(S, s0, rtol=0, atol=1e-12 * s0[0])
    assert np.abs(U * S @ V.T - a).max() <= 1e-12 * s0[0] * max(rows, cols)
    # Singular vectors of numerically zero singular values (below the truncation
    # threshold the sketch uses) are noise on both sides; only the rest is checked.
    kept = int((s0 > 10 * max(rows, cols) * 2.2e-16 * s0[0]).sum())
    assert np.abs(U[:, :kept].T @ U[:, :kept] - np.eye(kept)).max() < 1e-11
    assert np.abs(V[:, :kept].T @ V[:, :kept] - np.eye(kept)).max() < 1e-11
    gaps = np.minimum(np.abs(np.diff(np.r_[np.inf, s0])), np.abs(np.diff(np.r_[s0, -np.inf])))
    for j in range(kept):
        tol = 1e-13 * s0[0] / max(gaps[j], 1e-300) * 10
        if tol < 1e-4:
            assert np.abs(U[:, j] - u0[:, j]).max() <= tol, j
            assert np.abs(V[:, j] - v0[:, j]).max() <= tol, j


@pytest.mark.parametrize("rows,cols,seed", [(240, 240, 14), (256, 200, 16), (250, 250, 15), (512, 512, 17),
                                            (300, 480, 18), (257, 100, 19)])
def test_svd_block_path_unscaled(api, rows, cols, seed):
    """Ungraded Gaussian matrices on the block path: their Jacobi runs end at
    different sweep counts (odd and even, up to the last sweep of the
    multi-work-group phase), so the outputs come from either copy of the
    working columns.  The long side spans both LDS stash sizes of the round
    kernel (up to 256 and 257-512 rows); 512 x 512 takes the QR-preconditioned
    path (both sides at least 384, at most 1024)."""
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(rows, cols))
    U, S, V = (x.cpu().numpy() for x in api.svd(torch.from_numpy(a).cuda()))
    s0 = np.linalg.svd(a, compute_uv=False)
    assert np.allclose(S, s0, rtol=0, atol=1e-12 * s0[0])
    assert np.abs(U * S @ V.T - a).max() <= 1e-12 * s0[0] * max(rows, cols)
    p = min(rows, cols)
    assert np.abs(U.T @ U - np.eye(p)).max() < 1e-11
    assert np.abs(V.T @ V - np.eye(p)).max() < 1e-11


@pytest.mark.parametrize("fast", [1, 2, 9, 12])
def test_svd_block_path_finisher_sweeps(api, fast):
    """The same Gaussian matrix (its iteration needs about 12 sweeps) with the
    round-by-round phase cut after 1, 2, 9 or 12 sweeps: the single-work-group
    kernel runs the rest from either copy of the working columns."""
    rng = np.random.default_rng(21)
    a = rng.normal(size=(232, 232))
    U, S, V = (x.cpu().numpy() for x in api.svd(torch.from_numpy(a).cuda(), fast_sweeps=fast))
    s0 = np.linalg.svd(a, compute_uv=False)
    assert np.allclose(S, s0, rtol=0, atol=1e-12 * s0[0])
    assert np.abs(U * S @ V.T - a).max() <= 1e-12 * s0[0] * 232
    assert np.abs(U.T @ U - np.eye(232)).max() < 1e-11
    assert np.abs(V.T @ V - np.eye(232)).max() < 1e-11
    with pytest.raises(Exception):
        api.svd(torch.from_numpy(a).cuda(), fast_sweeps=25)


def test_svd_block_path_batched(api):
    rng = np.random.default_rng(12)
    a = np.stack([rng.normal(size=(210, 210)) * np.exp(-0.05 * np.arange(210))[None, :],
                  rng.normal(size=(210, 210))])
    U, S, V = (x.cpu().numpy() for x in api.svd(torch.from_numpy(a).cuda()))
    for b in range(2):
        s0 = np.linalg.svd(a[b], compute_uv=False)
        assert np.allclose(S[b], s0, atol=1e-12 * s0[0])
        assert np.abs(U[b] * S[b] @ V[b].T - a[b]).max() <= 1e-11 * s0[0]
        assert np.abs(U[b].T @ U[b] - np.eye(210)).max() < 1e-11


def test_svd_batched_and_rank_deficient(api):
    rng = np.random.default_rng(9)
    g = rng.normal(size=(30, 4))
    a = np.stack([g @ g.T, rng.normal(size=(30, 30)), np.zeros((30, 30))])
    U, S, V = (x.cpu().numpy() for x in api.svd(torch.from_numpy(a).cuda()))
    for b in range(3):
        s0 = np.linalg.svd(a[b], compute_uv=False)
        assert np.allclose(S[b], s0, atol=1e-12 * max(s0[0], 1.0))
        assert np.abs(U[b] * S[b] @ V[b].T - a[b]).max() <= 1e-11 * max(s0[0], 1.0)
    # PSD input: the eigenvectors of the kept part agree on both sides
    assert np.abs(U[0][:, :4] - V[0][:, :4]).max() < 1e-10


def _blobs(m, d, k, seed, dtype=np.float64):
    rng = np.random.default_rng(seed)
    cen = rng.normal(scale=3.0, size=(k, d))
    lab = rng.integers(0, k, size=m)
    return (cen[lab] + rng.normal(size=(m, d))).astype(dtype)


@pytest.mark.parametrize("m,d,k,weight", [(700, 5, 7, "const"), (2000, 50, 50, "pow"), (1500, 20, 130, "const"),
                                          (513, 3, 1, "const")])
def test_kmeans_and_snap_f64(api, m, d, k, weight):
    p = _blobs(m, d, max(k // 2, 1), 11)
    w = oc.upsilon(np.linalg.norm(p, axis=1), weight, 1.0)
    z0 = p[np.linspace(0, m - 1, k).astype(int)]
    for iters in (0, 1, 5):
        Z, lab, obj, sn = api.kmeans(torch.from_numpy(p).cuda(), torch.from_numpy(w).cuda(),
                                     torch.from_numpy(z0).cuda(), iters)
        ref = oc.weighted_kmeans(p, w, z0, iters)
        assert np.array_equal(lab.cpu().numpy(), ref.labels)
        assert np.abs(Z.cpu().numpy() - ref.Z).max() <= 1e-12 * (1 + np.abs(ref.Z).max())
        o = obj.cpu().numpy()
        assert o[0] == pytest.approx(ref.e_initial, rel=1e-11)
        assert o[1] == pytest.approx(ref.e_final, rel=1e-11)
        assert np.array_equal(sn.cpu().numpy(), oc.snap(p, ref.Z))


def test_kmeans_snap_conflicts_and_ties(api):
    # many identical rows and coinciding centres: every candidate list is exhausted
    p = np.zeros((600, 4))
    p[300:] = 1.0
    z0 = np.zeros((40, 4))
    w = np.ones(600)
    Z, lab, obj, sn = api.kmeans(torch.from_numpy(p).cuda(), torch.from_numpy(w).cuda(), torch.from_numpy(z0).cuda(), 2)
    ref = oc.weighted_kmeans(p, w, z0, 2)
    assert np.array_equal(lab.cpu().numpy(), ref.labels)
    assert np.array_equal(sn.cpu().numpy(), oc.snap(p, ref.Z))


@pytest.mark.parametrize("m,d,k,seed", [(20000, 6, 300, 3), (70000, 12, 640, 4)])
def test_snap_deep_exhaustion_f64(api, m, d, k, seed):
    # centres packed around the data mean: later centres find their nearest
    # rows taken in most blocks, so the per-block lists and block rescans decide
    rng = np.random.default_rng(seed)
    p = rng.normal(size=(m, d))
    z0 = p.mean(0) + 0.05 * rng.normal(size=(k, d))
    w = np.ones(m)
    Z, lab, obj, sn = api.kmeans(torch.from_numpy(p).cuda(), torch.from_numpy(w).cuda(), torch.from_numpy(z0).cuda(), 0)
    assert np.array_equal(sn.cpu().numpy(), oc.snap(p, z0))


def test_snap_duplicate_rows_across_blocks_f64(api):
    # 6 distinct points repeated over 9000 rows in random order: exact ties
    # between blocks go to the lowest row index
    rng = np.random.default_rng(8)
    pts = rng.normal(size=(6, 5))
    p = pts[rng.integers(0, 6, size=9000)]
    z0 = pts[rng.integers(0, 6, size=150)] + 1e-3 * rng.normal(size=(150, 5))
    w = np.ones(9000)
    Z, lab, obj, sn = api.kmeans(torch.from_numpy(p).cuda(), torch.from_numpy(w).cuda(), torch.from_numpy(z0).cuda(), 0)
    assert np.array_equal(sn.cpu().numpy(), oc.snap(p, z0))


@pytest.mark.parametrize("dim,dt,rows,k", [(320, "bf16", 4000, 48), (512, "bf16", 4000, 48), (512, "f16", 4000, 48),
                                           (20, "bf16", 4000, 48), (36, "f16", 4000, 48), (500, "f32", 4000, 48),
                                           (200, "f32", 4000, 48), (384, "f32", 30000, 100),
                                           (200, "bf16", 20000, 200), (504, "bf16", 60000, 500)])
def test_kmeans_fast_path_matches_generic(api, dim, dt, rows, k):
    """k-means through the fast assignment kernel against the generic tile kernel on the same
    values (a copy starting one element past a 16-byte boundary takes the generic path).
    257-512 dimensions: the fast kernel's widest k-block cases (FP32 above 256 dimensions
    streams 16-centre chunks); 20 and 36 dimensions (multiples of 4, not of 8): the tile
    kernels' 8-byte pieces.  The shapes cover one centre group and the 2-4 groups merged
    when the rows are too few to fill the chip (4000 rows; 2e4 rows x 200 centres in BF16).
    All keep the same per-element MFMA order, so labels, centres, objective and snapped rows
    are bit-identical."""
    dtype = {"bf16": torch.bfloat16, "f16": torch.float16, "f32": torch.float32}[dt]
    rng = np.random.default_rng(dim + rows)
    p = rng.normal(size=(rows, dim)).astype(np.float32)
    z0 = torch.from_numpy(p[:k].astype(np.float64)).cuda()
    w = torch.ones(rows, dtype=torch.float64, device="cuda")
    pa = torch.from_numpy(p).to(dtype).cuda()
    buf = torch.empty(rows * dim + 1, dtype=dtype, device="cuda")
    pm = buf[1:].view(rows, dim)
    pm.copy_(pa)
    assert pa.data_ptr() % 16 == 0 and pm.data_ptr() % 16 != 0
    fast = api.kmeans(pa, w, z0, 3)
    gen = api.kmeans(pm, w, z0, 3)
    for a, b in zip(fast, gen):
        assert torch.equal(a, b)
