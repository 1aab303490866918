"""Seeded generators for the matrices the sketching method is run on.

Every generator draws from ``numpy.random.default_rng(seed)`` on the host and
returns a :class:`MatrixSpec`: the description of an m x n matrix A that is
either stored (``dense``) or defined by an entry generator (``lowrank``:
A = Pg diag(s) Qg^T + noise, ``rbf``: A_ij = exp(-|x_i - y_j|^2 / (2 sigma^2))).
Random numbers that the *method* draws (pilot samples, the noise entries,
error-estimation samples) are not drawn here: they come from the counter-based
generator each side implements, keyed by the seeds stored in the spec.

The workload shapes follow the paper's experiments (dense and sparse matrices
of tens of thousands of rows and columns, sampling rates of 1-10% of sqrt(mn),
Section 5, Table 1) and the benchmark configurations listed in ``CONFIGS``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class MatrixSpec:
    """An m x n matrix known only through an entry generator or a dense array.

    kind = "dense":   ``a`` (m x n).
    kind = "lowrank": ``pf`` (m x r), ``s`` (r), ``qf`` (n x r); A_ij =
                      sum_t pf[i,t] s[t] qf[j,t] + noise_std * g(noise_seed, i, j)
                      where g is a standard normal drawn from the counter-based
                      generator at counter (i, j).
    kind = "rbf":     ``x`` (m x d), ``y`` (n x d), ``sigma``; A_ij =
                      exp(-|x_i - y_j|^2 / (2 sigma^2)).
    kind = "csr":     ``sp``, a scipy.sparse CSR matrix (canonical: sorted,
                      no duplicates) holding the nonzeros of A.
    All arrays are float64 and C-contiguous.
    """

    kind: str
    m: int
    n: int
    a: Optional[np.ndarray] = None
    pf: Optional[np.ndarray] = None
    qf: Optional[np.ndarray] = None
    s: Optional[np.ndarray] = None
    noise_std: float = 0.0
    noise_seed: int = 0
    x: Optional[np.ndarray] = None
    y: Optional[np.ndarray] = None
    sigma: float = 1.0
    sp: Optional[object] = None
    name: str = ""

    @property
    def r(self) -> int:
        return 0 if self.s is None else int(self.s.shape[0])

    @property
    def d(self) -> int:
        return 0 if self.x is None else int(self.x.shape[1])

    @property
    def nnz(self) -> int:
        return 0 if self.sp is None else int(self.sp.nnz)

    def nbytes(self) -> int:
        if self.sp is not None:
            return int(self.sp.data.nbytes + self.sp.indices.nbytes + self.sp.indptr.nbytes)
        seen, total = set(), 0
        for v in (self.a, self.pf, self.qf, self.s, self.x, self.y):
            if v is not None and id(v) not in seen:
                seen.add(id(v))
                total += int(v.nbytes)
        return total


def _median_pair_distance(x: np.ndarray, rng: np.random.Generator, pairs: int = 1000) -> float:
    """Median of |x_i - x_j| over ``pairs`` random index pairs with i != j."""
    m = x.shape[0]
    i = rng.integers(0, m, size=pairs)
    j = rng.integers(0, m - 1, size=pairs)
    j = j + (j >= i)  # uniform over j != i
    return float(np.median(np.linalg.norm(x[i] - x[j], axis=1)))


def rbf_mixture(m: int, d: int, n_clusters: int, center_std: float, cluster_sigma,
                seed: int, center_points: bool = False, name: str = "") -> MatrixSpec:
    """RBF kernel matrix over a Gaussian mixture, with Y = X (so A is PSD).

    Centres ~ N(0, center_std^2 I_d); each point picks a centre uniformly and adds
    N(0, s_c^2 I_d) noise where s_c is ``cluster_sigma`` (a number) or is drawn
    log-uniformly from the (lo, hi) pair per cluster.  The bandwidth is the
    median distance over 1000 random pairs of distinct points.
    """
    rng = np.random.default_rng(seed)
    centers = rng.normal(0.0, center_std, size=(n_clusters, d))
    if isinstance(cluster_sigma, (tuple, list)):
        lo, hi = cluster_sigma
        sig = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_clusters))
    else:
        sig = np.full(n_clusters, float(cluster_sigma))
    lab = rng.integers(0, n_clusters, size=m)
    x = centers[lab] + rng.normal(0.0, 1.0, size=(m, d)) * sig[lab][:, None]
    sigma = _median_pair_distance(x, rng)
    if center_points:
        # The kernel depends only on differences, so centring changes no entry;
        # it keeps |x|^2 small next to the distances that matter.
        x = x - x.mean(axis=0, keepdims=True)
    x = np.ascontiguousarray(x)
    return MatrixSpec(kind="rbf", m=m, n=m, x=x, y=x, sigma=sigma, name=name or f"rbf-{m}-d{d}")


def _orthonormal(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    g = rng.normal(0.0, 1.0, size=(rows, cols))
    q, _ = np.linalg.qr(g)
    return np.ascontiguousarray(q)


def lowrank_noise(m: int, n: int, r: int, seed: int, noise_std: float = 1e-3,
                  s_kind: str = "inv", noise_seed: Optional[int] = None, name: str = "") -> MatrixSpec:
    """A = Pg diag(s) Qg^T + E with Gaussian factors given orthonormal columns.

    s_kind "inv": s_i = 1/i.  s_kind "scaled": s_i = sqrt(mn)/i, so the signal
    stays well above the noise floor (E is i.i.d. N(0, noise_std^2)).
    """
    rng = np.random.default_rng(seed)
    pf = _orthonormal(rng, m, r)
    qf = _orthonormal(rng, n, r)
    i = np.arange(1, r + 1, dtype=np.float64)
    if s_kind == "inv":
        s = 1.0 / i
    elif s_kind == "scaled":
        s = math.sqrt(m * n) / i
    else:
        raise ValueError(s_kind)
    return MatrixSpec(kind="lowrank", m=m, n=n, pf=pf, qf=qf, s=s, noise_std=float(noise_std),
                      noise_seed=int(seed + 7919 if noise_seed is None else noise_seed),
                      name=name or f"lowrank-{m}x{n}-r{r}-{s_kind}")


def exact_rank(m: int, n: int, k: int, seed: int, name: str = "") -> MatrixSpec:
    """Dense A = G H^T with Gaussian G (m x k), H (n x k): rank exactly k."""
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(m, k))
    h = rng.normal(size=(n, k))
    return dense_matrix(g @ h.T, name=name or f"rank{k}-{m}x{n}")


def block_replicated(k: int, t_rows: int, t_cols: int, seed: int) -> MatrixSpec:
    """A = B kron ones(t_rows, t_cols) for a Gaussian k x k core B.

    Every row (column) of A is repeated t_rows (t_cols) times in consecutive
    blocks; the paper's stabilised sketch recovers A exactly from one row and
    one column per block.
    """
    rng = np.random.default_rng(seed)
    b = rng.normal(size=(k, k))
    return dense_matrix(np.kron(b, np.ones((t_rows, t_cols))), name=f"blockrep-{k}x{t_rows}x{t_cols}")


def dense_matrix(a: np.ndarray, name: str = "dense") -> MatrixSpec:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return MatrixSpec(kind="dense", m=a.shape[0], n=a.shape[1], a=a, name=name)


def natural_scene_like(m: int = 6480, n: int = 7680, seed: int = 0) -> MatrixSpec:
    """Dense stand-in for a natural image: a 1/f random field clipped to [0, 1]."""
    rng = np.random.default_rng(seed)
    noise = rng.normal(size=(m, n))
    fy = np.fft.fftfreq(m)[:, None]
    fx = np.fft.rfftfreq(n)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    f[0, 0] = 1.0
    spec = np.fft.rfft2(noise) / f
    spec[0, 0] = 0.0
    field = np.fft.irfft2(spec, s=(m, n))
    field = (field - field.mean()) / (4.0 * field.std()) + 0.5
    return dense_matrix(np.clip(field, 0.0, 1.0), name=f"scene-{m}x{n}")


def hubble_like(m: int = 15852, n: int = 12392, seed: int = 0, blobs: int = 4000) -> MatrixSpec:
    """Dense stand-in for a sky image: dark background plus bright Gaussian blobs."""
    rng = np.random.default_rng(seed)
    a = np.abs(rng.normal(0.0, 0.01, size=(m, n)))
    cy = rng.integers(0, m, size=blobs)
    cx = rng.integers(0, n, size=blobs)
    amp = rng.pareto(1.5, size=blobs) * 0.1
    rad = rng.uniform(1.0, 6.0, size=blobs)
    for y0, x0, h, w in zip(cy, cx, amp, rad):
        h0 = int(3 * w) + 1
        ys = slice(max(0, y0 - h0), min(m, y0 + h0 + 1))
        xs = slice(max(0, x0 - h0), min(n, x0 + h0 + 1))
        yy = np.arange(ys.start, ys.stop)[:, None] - y0
        xx = np.arange(xs.start, xs.stop)[None, :] - x0
        a[ys, xs] += h * np.exp(-(yy * yy + xx * xx) / (2.0 * w * w))
    return dense_matrix(np.minimum(a, 1.0), name=f"hubble-{m}x{n}")


def _zipf_weights(n: int, a: float, rng: np.random.Generator) -> np.ndarray:
    """Probabilities proportional to rank^-a over a random permutation of n items."""
    w = np.arange(1, n + 1, dtype=np.float64) ** -a
    w = w[rng.permutation(n)]
    return w / w.sum()


def _distinct_pairs(nnz: int, pr: np.ndarray, pc: np.ndarray, rng: np.random.Generator):
    """nnz distinct (row, column) positions, rows and columns drawn independently with
    probabilities pr and pc (repeated draws are discarded and drawn again)."""
    m, n = pr.size, pc.size
    key = np.empty(0, dtype=np.int64)
    while key.size < nnz:
        draw = int((nnz - key.size) * 1.3) + 1024
        new = rng.choice(m, size=draw, p=pr).astype(np.int64) * n + rng.choice(n, size=draw, p=pc)
        key = np.unique(np.concatenate([key, new]))
    key = key[np.sort(rng.permutation(key.size)[:nnz])]
    return key // n, key % n


def sparse_matrix(rows: np.ndarray, cols: np.ndarray, vals: np.ndarray, m: int, n: int, name: str) -> MatrixSpec:
    """A CSR source from (row, column, value) triplets (duplicates summed, explicit zeros dropped)."""
    import scipy.sparse as sps
    a = sps.csr_matrix((np.asarray(vals, dtype=np.float64), (np.asarray(rows), np.asarray(cols))), shape=(m, n))
    a.sum_duplicates()
    a.eliminate_zeros()
    a.sort_indices()
    a.indices = a.indices.astype(np.int32)
    a.indptr = a.indptr.astype(np.int64)
    return MatrixSpec(kind="csr", m=m, n=n, sp=a, name=name)


def movie_like(m: int = 27000, n: int = 46000, density: float = 0.0056, seed: int = 0, rank: int = 12) -> MatrixSpec:
    """Sparse stand-in for a movie-rating matrix (users x movies): density * m * n ratings at
    distinct positions, user and movie degrees Zipf-distributed (exponent 0.7), integer ratings
    1..5 from a rank-`rank` preference model plus user and movie offsets and noise."""
    rng = np.random.default_rng(seed)
    nnz = int(round(density * m * n))
    i, j = _distinct_pairs(nnz, _zipf_weights(m, 0.7, rng), _zipf_weights(n, 0.7, rng), rng)
    u = rng.normal(size=(m, rank)) / np.sqrt(rank)
    v = rng.normal(size=(n, rank))
    bu, bv = rng.normal(0.0, 0.4, m), rng.normal(0.0, 0.5, n)
    r = 3.5 + bu[i] + bv[j] + np.einsum("tk,tk->t", u[i], v[j]) + rng.normal(0.0, 0.5, i.size)
    return sparse_matrix(i, j, np.clip(np.rint(r), 1.0, 5.0), m, n, f"movie-like-{m}x{n}")


def newsgroup_like(m: int = 18774, n: int = 61188, density: float = 0.0022, seed: int = 0) -> MatrixSpec:
    """Sparse stand-in for a document-term count matrix: density * m * n nonzeros at distinct
    positions, term frequencies Zipf-distributed (exponent 1.1), document lengths log-normal,
    counts 1 + Poisson growing with the term's frequency."""
    rng = np.random.default_rng(seed)
    nnz = int(round(density * m * n))
    pt = _zipf_weights(n, 1.1, rng)
    dl = np.exp(rng.normal(0.0, 0.8, m))
    pd = dl / dl.sum()
    i, j = _distinct_pairs(nnz, pd, pt, rng)
    lam = 0.3 + 2.0 * np.sqrt(pt[j] / pt.max())
    return sparse_matrix(i, j, 1.0 + rng.poisson(lam), m, n, f"newsgroup-like-{m}x{n}")


# Benchmark and parity configurations.  Each entry: matrix recipe + sketch sizes.
CONFIGS = {
    # RBF kernel over 2000 points in d=10 from 20 Gaussians (centres N(0,4I),
    # unit cluster spread), k1 = k2 = 50, c = 5, FP64, exact error.
    "rbf2000": dict(kind="rbf", m=2000, d=10, n_clusters=20, center_std=2.0, cluster_sigma=1.0,
                    seed=0, k=50, iters=5, precision="f64", err_samples=0),
    # Low-rank (r = 200, s_i = 1/i) plus N(0, 1e-3^2) noise, 1e5 x 2e4, k = 200,
    # FP32, error from 1e7 sampled entries.
    "lowrank1e5": dict(kind="lowrank", m=100_000, n=20_000, r=200, s_kind="inv", noise_std=1e-3,
                       seed=0, k=200, iters=5, precision="f32", err_samples=10_000_000),
    # Same shape with s_i = sqrt(mn)/i so that the signal dominates the noise.
    "lowrank1e5s": dict(kind="lowrank", m=100_000, n=20_000, r=200, s_kind="scaled", noise_std=1e-3,
                        seed=0, k=200, iters=5, precision="f32", err_samples=10_000_000),
    # RBF kernel over 1e6 points in d = 64 from 100 Gaussians (centres N(0, I),
    # per-cluster spread log-uniform in [0.05, 0.3]); k = 500, c = 20, FP32.
    "rbf1e6": dict(kind="rbf", m=1_000_000, d=64, n_clusters=100, center_std=1.0,
                   cluster_sigma=(0.05, 0.3), seed=0, k=500, iters=20, precision="f32",
                   err_samples=10_000_000),
}


def config(name: str, scale: float = 1.0) -> tuple[MatrixSpec, dict]:
    """Build the matrix of a named configuration; ``scale`` shrinks m and n."""
    c = dict(CONFIGS[name])
    m = max(8, int(round(c["m"] * scale)))
    if c["kind"] == "rbf":
        spec = rbf_mixture(m, c["d"], c["n_clusters"], c["center_std"], c["cluster_sigma"], c["seed"],
                           center_points=True, name=f"{name}@{scale:g}")
    else:
        n = max(8, int(round(c["n"] * scale)))
        spec = lowrank_noise(m, n, min(c["r"], m, n), c["seed"], noise_std=c["noise_std"], s_kind=c["s_kind"],
                             name=f"{name}@{scale:g}")
    return spec, c


def request_stream(n_requests: int = 5000, qps: float = 100.0, seed: int = 0,
                   m_range=(1_000, 500_000), ks=(16, 32, 64, 128, 256)) -> list[dict]:
    """Serving workload: Poisson arrivals of sketch requests of uneven shape.

    Each request: m, n log-uniform in ``m_range``; with probability 1/2 a
    low-rank-plus-noise matrix (rank log-uniform in [16, 256], s_i = 1/i, noise
    1e-3), else an RBF kernel over d = 32 Gaussian-mixture points with 10-100
    clusters; target rank k uniform over ``ks``; pilot size k; seed 1000 + id.
    Only the recipe is returned; :func:`request_matrix` builds the matrix.
    """
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / qps, size=n_requests))
    lo, hi = math.log(m_range[0]), math.log(m_range[1])
    out = []
    for rid in range(n_requests):
        m = int(round(math.exp(rng.uniform(lo, hi))))
        n = int(round(math.exp(rng.uniform(lo, hi))))
        kind = "lowrank" if rng.uniform() < 0.5 else "rbf"
        k = int(ks[rng.integers(0, len(ks))])
        rec = dict(id=rid, arrival=float(t[rid]), m=m, n=n, kind=kind, k=k, seed=1000 + rid)
        if kind == "lowrank":
            rec["r"] = int(round(math.exp(rng.uniform(math.log(16), math.log(256)))))
        else:
            rec["n_clusters"] = int(rng.integers(10, 101))
        out.append(rec)
    return out


def request_matrix(rec: dict) -> MatrixSpec:
    """Build the matrix of one serving request (see :func:`request_stream`)."""
    if rec["kind"] == "lowrank":
        return lowrank_noise(rec["m"], rec["n"], rec["r"], rec["seed"], noise_std=1e-3, s_kind="inv",
                             name=f"req{rec['id']}")
    rng = np.random.default_rng(rec["seed"])
    m, n, d, nc = rec["m"], rec["n"], 32, rec["n_clusters"]
    centers = rng.normal(size=(nc, d))
    sig = np.exp(rng.uniform(math.log(0.05), math.log(0.3), size=nc))
    lx = rng.integers(0, nc, size=m)
    ly = rng.integers(0, nc, size=n)
    x = centers[lx] + rng.normal(size=(m, d)) * sig[lx][:, None]
    y = centers[ly] + rng.normal(size=(n, d)) * sig[ly][:, None]
    sigma = _median_pair_distance(x, rng)
    mu = x.mean(axis=0, keepdims=True)
    return MatrixSpec(kind="rbf", m=m, n=n, x=np.ascontiguousarray(x - mu), y=np.ascontiguousarray(y - mu),
                      sigma=sigma, name=f"req{rec['id']}")
