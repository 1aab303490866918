"""Weighted k-means and snapping in FP32 / BF16 / FP16 at the shapes the benchmark runs (and in
FP64 on sparse embeddings, whose exact ties rounding decides), step by step against the FP64
oracle (Section 3.2, Eq. (wkmeans); snapping to in-sample points).

Each Lloyd iteration of the GPU path is checked against the oracle's definition of that
iteration applied to the GPU's own state, so one near-tie decided differently cannot make
the two trajectories drift apart and hide (or fake) an error later:

* assignment at Z_t: the GPU labels equal the oracle's argmin wherever the oracle's gap
  between nearest and second-nearest centre exceeds twice the rounding bound of one
  computed distance; elsewhere the GPU's centre must lie within that bound of the nearest
  (a tie).  Decisions are compared in the kernel's precision: the oracle assigns the rows as
  the kernel stores them against the centres rounded to the kernel's type (Z_t is FP64, the
  distance GEMM reads it rounded).
* the objective sum_l w_l |P_l - Z_s(l)|^2 at Z_t, within the summed rounding bounds;
* the update: Z_{t+1} equals the oracle's weighted means of P over the GPU's labels,
  within the FP64 summation bound;
* snapping after the last iteration: replaying the greedy walk over the centres in order,
  every centre finds its nearest untaken row (within the rounding bound) in the GPU's set,
  and the replay takes exactly the GPU's set.

Rounding bound of one computed distance (FP32 accumulation, K = dim terms): the kernel forms
|z|^2 - 2 p.z with the dot product accumulated in FP32 (each product exact for 16-bit inputs,
rounded once for FP32 inputs) and |z|^2 rounded to FP32, so
    |error| <= 2 (K + 2) u |p| |z| + 2 u |z|^2,   u = 2^-24,
using sum_t |p_t z_t| <= |p| |z|.  The snap pass adds |p|^2 and |z|^2 in FP64 and takes the
dot product from the same FP32 accumulation, so the same bound holds there.  FP64 compute: the
same bound with u = 2^-53, and the snap replay also admits the kernel's FP64 tie window.
"""
import math

import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import cabs as oc
from oracle import philox

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32 = 2.0 ** -24
TORCH_DT = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16, "f64": torch.float64}


def _unit(dt):
    """Unit roundoff of the distance accumulation: FP64 for FP64 compute, FP32 otherwise."""
    return 2.0 ** -53 if dt == "f64" else U32


@pytest.fixture(scope="module")
def api():
    from paper_1607_07395_amd import api as a
    return a


def _as_kernel(x, dt):
    """Values of an FP64 array after rounding to the kernel's type, back in FP64."""
    return torch.from_numpy(np.ascontiguousarray(x)).to(TORCH_DT[dt]).double().numpy()


def _dist_bound(pn, zn, K, u=U32):
    """Rounding bound of one computed squared distance (see the module docstring)."""
    return 2.0 * (K + 2) * u * pn * zn + 2.0 * u * zn * zn


def _check_assignment(P, Zk, labels, K, u=U32):
    """GPU labels at centres Zk (already in the kernel's type) against the oracle's assignment."""
    lab_ref, dmin_ref, gap_ref = oc.assign(P, Zk)
    pn = np.linalg.norm(P, axis=1)
    zmax = float(np.linalg.norm(Zk, axis=1).max())
    b = _dist_bound(pn, zmax, K, u)
    sure = gap_ref > 2.0 * b
    bad = np.flatnonzero(sure & (labels != lab_ref))
    assert bad.size == 0, (bad[:10], labels[bad[:10]], lab_ref[bad[:10]], gap_ref[bad[:10]], b[bad[:10]])
    d_chosen = ((P - Zk[labels]) ** 2).sum(1)
    excess = d_chosen - dmin_ref
    assert np.all(excess <= 2.0 * b), float((excess / b).max())
    return d_chosen, b, int((~sure).sum())


def _replay_snap(P, Zk, snap_gpu, K, u=U32):
    """The greedy snap of the GPU's centres, replayed with the GPU's set deciding the ties.  In
    FP64 the kernel also counts distances within SNAP_TIE_RTOL (|Z_j| + sqrt(d_min))^2 of the
    nearest as tied (lowest row), so the replay's window includes that."""
    D = cdist(P, Zk, "sqeuclidean")
    pn = np.linalg.norm(P, axis=1)
    zn = np.linalg.norm(Zk, axis=1)
    gset = set(int(x) for x in snap_gpu)
    taken = np.zeros(P.shape[0], dtype=bool)
    ambiguous = 0
    for j in range(Zk.shape[0]):
        dj = np.where(taken, np.inf, D[:, j])
        dmin = float(dj.min())
        b = 2.0 * _dist_bound(pn, zn[j], K, u)
        if u < U32:
            b = b + oc.SNAP_TIE_RTOL * (zn[j] + np.sqrt(max(dmin, 0.0))) ** 2
        cand = np.flatnonzero(dj <= dmin + b)
        inset = [int(l) for l in cand if int(l) in gset]
        assert inset, (j, dmin, cand[:10])
        if cand.size > 1:
            ambiguous += 1
        # FP32 and 16-bit compare exactly (the nearest computed distance wins); FP64 takes the
        # lowest row inside its tie window, as the oracle's snap does
        pick = min(inset) if u < U32 else min(inset, key=lambda l: (dj[l], l))
        taken[pick] = True
    assert np.array_equal(np.flatnonzero(taken), np.asarray(snap_gpu)), "replay does not take the GPU's rows"
    return ambiguous


def _stepwise(api, P, w, z0, iters, dt, snap=True):
    """Run cabs_kmeans for 0..iters iterations and check every step against the oracle."""
    K = P.shape[1]
    Pk = _as_kernel(P, dt)          # the rows as the kernel stores them (exact in FP64)
    Pd = torch.from_numpy(Pk).to(TORCH_DT[dt]).cuda()
    wd = torch.from_numpy(w).cuda()
    z0d = torch.from_numpy(z0).cuda()
    Zprev = labprev = None
    unsure_total = 0
    for t in range(iters + 1):
        Z, lab, obj, sn = api.kmeans(Pd, wd, z0d, t, snap=(snap and t == iters))
        torch.cuda.synchronize()
        Z, lab, obj = Z.cpu().numpy(), lab.cpu().numpy().astype(np.int64), obj.cpu().numpy()
        if t == 0:
            assert np.array_equal(Z, z0)
        else:
            # the update from the previous step's centres and labels (FP64 weighted means)
            want = oc.centroid_update(Pk, w, labprev, Zprev)
            tol = 2.0 * P.shape[0] * 1.2e-16 * np.abs(Pk).max()
            assert np.abs(Z - want).max() <= tol, (t, np.abs(Z - want).max(), tol)
        Zk = _as_kernel(Z, dt)
        d_chosen, b, unsure = _check_assignment(Pk, Zk, lab, K, _unit(dt))
        unsure_total += unsure
        # objective at Z_t (obj[1] after t iterations; obj[0] is the one at Z_0)
        want_obj = float(w @ d_chosen)
        assert abs(obj[1] - want_obj) <= float(w @ b) + 1e-12 * want_obj, (t, obj[1], want_obj)
        if t == iters and snap:
            amb = _replay_snap(Pk, Zk, sn.cpu().numpy(), K, _unit(dt))
        Zprev, labprev = Z, lab
    return unsure_total, (amb if snap else None)


def _pilot_rows(n, k, seed, stream):
    return philox.floyd_sample(n, k, seed, stream)


@pytest.fixture(scope="module")
def lowrank_embeddings():
    """The oracle's pilot embeddings P (1e5 x 200) and Q (2e4 x 200) of the 1e5 x 2e4 low-rank +
    noise workload (rank 200, s_i = 1/i, noise 1e-3, k = 200), the input the benchmark's k-means
    runs on, together with the oracle's own FP64 sketch of that workload."""
    import workloads
    spec, cfg = workloads.config("lowrank1e5")
    k = cfg["k"]
    ref = oc.cabs(spec, oc.Params.square(k, kmeans_iters=cfg["iters"], seed=0))
    return spec, ref


@pytest.mark.parametrize("side", ["rows", "cols"])
def test_kmeans_f32_lowrank_embeddings_stepwise(api, lowrank_embeddings, side):
    """FP32 fast assignment (200 dimensions: 13 k-blocks; 200 centres: 7 chunks of 32, the last
    holding 8), 5 iterations and the snap, on the 1e5-row and 2e4-row embeddings."""
    spec, ref = lowrank_embeddings
    P = ref.P if side == "rows" else ref.Q
    idx = ref.pilot_rows if side == "rows" else ref.pilot_cols
    w = ref.w_r if side == "rows" else ref.w_c
    z0 = _as_kernel(P, "f32")[idx]
    unsure, amb = _stepwise(api, P, w, z0, 5, "f32")
    print(f"{side}: rows with an undecidable nearest centre over 6 assignments: {unsure}; ambiguous snaps: {amb}")


def _blob_embedding(rows, dim, n_clusters, seed):
    """Gaussian-mixture rows with decaying per-dimension scales (like the singular-value decay of a
    pilot embedding): scale_t = (1 + t)^-1/2, cluster centres N(0, 4 scale^2), unit-scale noise."""
    rng = np.random.default_rng(seed)
    scale = 1.0 / np.sqrt(1.0 + np.arange(dim))
    cen = rng.normal(size=(n_clusters, dim)) * 2.0 * scale
    lab = rng.integers(0, n_clusters, size=rows)
    return cen[lab] + rng.normal(size=(rows, dim)) * scale


@pytest.mark.parametrize("dt,rows,dim,k,iters", [("bf16", 100_000, 504, 500, 2), ("f16", 30_000, 504, 500, 2),
                                                 ("f32", 30_000, 500, 500, 2), ("bf16", 20_000, 200, 200, 3)])
def test_kmeans_reduced_precision_stepwise(api, dt, rows, dim, k, iters):
    """16-bit fast assignment at the 1e6 x 1e6 RBF configuration's embedding width (k = 500 padded
    to 504 dimensions: the 16 k-block case) and FP32 at 500 dimensions (the generic tile kernel),
    with iterations and the snap."""
    P = _blob_embedding(rows, dim, 300, seed=dim + rows)
    w = oc.upsilon(np.linalg.norm(P, axis=1), "const", 0.0)
    z0 = _as_kernel(P, dt)[_pilot_rows(rows, k, 5, 0)]
    unsure, amb = _stepwise(api, P, w, z0, iters, dt)
    print(f"{dt} {rows}x{dim}x{k}: undecidable assignments {unsure}, ambiguous snaps {amb}")


def test_kmeans_pow_weights_f32_stepwise(api):
    """POW weights (the hard-threshold workload's weighting) through the FP32 update."""
    P = _blob_embedding(40_000, 96, 80, seed=3)
    w = oc.upsilon(np.linalg.norm(P, axis=1), "pow", 2.0)
    z0 = _as_kernel(P, "f32")[_pilot_rows(40_000, 120, 9, 1)]
    _stepwise(api, P, w, z0, 4, "f32")


def test_sketch_f64_lowrank_1e5_fullsize_matches_oracle(api, lowrank_embeddings):
    """The benchmark's 1e5 x 2e4 low-rank + noise workload in FP64 at full size (k = 200, c = 5):
    the 200 x 200 block-Jacobi SVDs, the Cholesky orthogonalisation route (p = 200 <= 204), k-means
    and snapping over 1e5 and 2e4 rows; follow-up indices bit-exact with the oracle."""
    from sketch_checks import compare_f64
    spec, ref = lowrank_embeddings
    kw = dict(k1_rows=200, k1_cols=200, k2_rows=200, k2_cols=200, kmeans_iters=5, seed=0)
    compare_f64(api, spec, kw, ref=ref)


@pytest.mark.parametrize("kind,k,seed,dt", [("movie", 40, 0, "f64"), ("news", 32, 3, "f64"), ("news", 64, 4, "f64"),
                                             ("movie", 48, 5, "f32"), ("news", 40, 6, "bf16")])
def test_kmeans_f64_sparse_embeddings_stepwise(api, kind, k, seed, dt):
    """FP64 k-means and snap on the pilot embeddings of sparse stand-ins (movie-like 3000 x 4600
    at 8 %, newsgroup-like 1877 x 6118 at 10 %).  Rows whose sampled columns are all zero embed
    to exactly 0 and several pilot rows coincide, so the oracle meets exact distance ties that the
    GPU's expansion |z|^2 - 2 p.z decides by rounding: each step is checked against the oracle's
    definition with ties inside the FP64 rounding bound (and the snap's tie window) allowed.  The
    rows of norm 0 are the snap's one shared candidate class (most centres of the column side take
    one of them); FP32 and BF16 embeddings are checked in their own precision."""
    import workloads
    spec = workloads.movie_like(3000, 4600, 0.08, seed=1) if kind == "movie" else \
        workloads.newsgroup_like(1877, 6118, 0.1, seed=2)
    ref = oc.cabs(spec, oc.Params.square(k, kmeans_iters=5, seed=seed))
    for P, idx, w in ((ref.P, ref.pilot_rows, ref.w_r), (ref.Q, ref.pilot_cols, ref.w_c)):
        unsure, amb = _stepwise(api, P, w, P[idx], 5, dt)
        print(f"{kind}: undecidable assignments {unsure}, ambiguous snaps {amb}, zero rows {int((P == 0).all(1).sum())}")
