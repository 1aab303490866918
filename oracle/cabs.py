"""Cascaded bilateral sampling, step by step, in float64 (test infrastructure only).

The steps follow Algorithm 2 of the paper (pilot sampling, pilot sketching,
follow-up sampling by weighted k-means, follow-up sketching), the sketching
routine of Section 4.1, the weighted k-means objective of Section 3.2, the
encoding errors and cluster sizes of Section 3.1, and the orthogonalisation of
supplementary Section 3.  Readings of points the paper leaves open are stated
where they are taken.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
from scipy.spatial.distance import cdist

from . import philox
from .matrices import Matrix

EPS = float(np.finfo(np.float64).eps)

WEIGHT_KINDS = ("const", "pow", "sigmoid", "step")
SKETCH_KINDS = ("stabilized", "pseudo_skeleton")
FOLLOW_UPS = ("kmeans", "hard", "leverage", "pilot")


class RankError(RuntimeError):
    """The intersection W has no singular value above the truncation threshold."""


@dataclasses.dataclass
class Params:
    """Sample sizes and options of one sketch (paper defaults where it gives them)."""

    k1_rows: int
    k1_cols: int
    k2_rows: int
    k2_cols: int
    kmeans_iters: int = 5            # c = 5 in all of the paper's experiments (Section 4)
    weight_kind: str = "const"       # slowly growing / constant weights for dense input (Section 3.2)
    weight_param: float = 0.0
    sketch_kind: str = "stabilized"  # the stabilised routine of Section 4.1
    orthogonalize: bool = True       # supplementary Section 3 (optional in the paper)
    pinv_rtol: float = 0.0           # <= 0: max(kr, kc) * eps * sigma_1
    seed: int = 0
    factors: bool = False            # also return the orthogonalised factor form of the result
    follow_up: str = "kmeans"        # "hard" / "leverage": the hard-threshold / leverage variants of Section 5;
                                     # "pilot": no follow-up round, the output is the pilot sketch (step 2)

    @classmethod
    def square(cls, k: int, **kw) -> "Params":
        return cls(k, k, k, k, **kw)


# ---------------------------------------------------------------------------
# The sketching routine (Section 4.1)
# ---------------------------------------------------------------------------

def svd_canonical(w: np.ndarray):
    """Thin SVD W = U diag(s) V^T, s descending, with a fixed sign per pair.

    Reading: the sign of each singular pair is fixed so that the entry of
    largest magnitude of u_i is positive (the first such entry on ties).  No
    quantity of the method depends on this choice; it only makes factor
    outputs comparable.
    """
    u, s, vt = np.linalg.svd(w, full_matrices=False)
    v = vt.T
    piv = np.argmax(np.abs(u), axis=0)
    sgn = np.where(u[piv, np.arange(u.shape[1])] < 0.0, -1.0, 1.0)
    return u * sgn, s, v * sgn


@dataclasses.dataclass
class Sketch:
    U: np.ndarray        # m x p, unit-norm columns  (C V_w N_c^-1)
    S: np.ndarray        # p                          (scaled singular values)
    V: np.ndarray        # n x p, unit-norm columns  (R^T U_w N_r^-1)
    Umid: np.ndarray     # kc x kr, so that A ~ C Umid R
    sw: np.ndarray       # singular values of W (all)
    nc: np.ndarray       # column norms of C V_w (all)
    nr: np.ndarray       # column norms of R^T U_w (all)
    keep: np.ndarray     # bool mask of kept components
    tol: float


def sketching(c: np.ndarray, rt: np.ndarray, w: np.ndarray, m: int, n: int,
              kind: str = "stabilized", pinv_rtol: float = 0.0) -> Sketch:
    """The ``sketching`` routine: A ~ U diag(S) V^T from C, R and W = A(I^r, I^c).

    With W = U_w Sigma_w V_w^T, the singular vectors are extrapolated to all
    rows and columns as C V_w and R^T U_w (R is stored transposed, n x kr, as in
    the proofs of supplementary Section 1).  The stabilised form of Section 4.1
    normalises each extrapolated vector by its own norm instead of by the
    singular value, and rescales the singular values:
        U = C V_w N_c^-1,  V = R^T U_w N_r^-1,  S = Sigma_w sqrt(mn / (kr kc)),
    N_c, N_r the column norms.  Readings: (1) the paper writes V as N_r^-1 U_w^T R,
    which is its transpose; V here is n x p.  (2) The scale is printed both as
    sqrt(mn/k^2) and sqrt(mn)/k with k rows and k columns; for kr != kc it is
    taken as sqrt(mn/(kr kc)).  (3) Components whose singular value does not
    exceed tol = max(kr, kc) eps sigma_1 (or pinv_rtol sigma_1), or whose
    extrapolated norm is zero, are dropped; if none remains, RankError.

    kind = "pseudo_skeleton" is Eq. (W) of Section 2.2, A ~ C W^+ R with the same
    truncation; its factor form is U diag(nc nr / sigma) V^T.

    Umid (kc x kr) is the CUR middle factor: A ~ C Umid R, i.e.
    Umid = V_w diag(d) U_w^T with d = S / (nc nr) (stabilised) or 1 / sigma.
    """
    kr, kc = w.shape
    uw, sw, vw = svd_canonical(w)
    if sw.size == 0 or not sw[0] > 0.0:
        raise RankError("W is zero")
    tol = (pinv_rtol if pinv_rtol > 0.0 else max(kr, kc) * EPS) * float(sw[0])
    ch = c @ vw
    rh = rt @ uw
    nc = np.linalg.norm(ch, axis=0)
    nr = np.linalg.norm(rh, axis=0)
    keep = (sw > tol) & (nc > 0.0) & (nr > 0.0)
    if not keep.any():
        raise RankError("no singular value of W above the threshold")
    nck, nrk, swk = nc[keep], nr[keep], sw[keep]
    if kind == "stabilized":
        s = swk * math.sqrt(m * n / (kr * kc))
        d = s / (nck * nrk)
    elif kind == "pseudo_skeleton":
        s = nck * nrk / swk
        d = 1.0 / swk
    else:
        raise ValueError(kind)
    umid = (vw[:, keep] * d) @ uw[:, keep].T
    return Sketch(U=ch[:, keep] / nck, S=s, V=rh[:, keep] / nrk, Umid=umid, sw=sw, nc=nc, nr=nr,
                  keep=keep, tol=tol)


def orthogonalize(u: np.ndarray, s: np.ndarray, v: np.ndarray):
    """Supplementary Section 3: turn A ~ U diag(S) V^T into an exact SVD of that product.

    U = U_0 Sigma_0 V_0^T (thin SVD); then Sigma_0 V_0^T diag(S) V^T = U_1 Sigma_1 V_1^T;
    the result is (U_0 U_1, Sigma_1, V_1).  Signs canonicalised as in svd_canonical.
    """
    u0, s0, v0t = np.linalg.svd(u, full_matrices=False)
    x = ((s0[:, None] * v0t) * s[None, :]) @ v.T
    u1, s1, v1t = np.linalg.svd(x, full_matrices=False)
    uo = u0 @ u1
    vo = v1t.T
    piv = np.argmax(np.abs(uo), axis=0)
    sgn = np.where(uo[piv, np.arange(uo.shape[1])] < 0.0, -1.0, 1.0)
    return uo * sgn, s1, vo * sgn


# ---------------------------------------------------------------------------
# Follow-up sampling: weighted k-means on the embeddings (Section 3.2)
# ---------------------------------------------------------------------------

def upsilon(norms: np.ndarray, kind: str, param: float) -> np.ndarray:
    """The monotone weight function of the weighted k-means objective.

    The paper names power, sigmoid and step functions.  Readings: "const" 1,
    "pow" |p|^param, "sigmoid" 1 / (1 + exp(-param |p|)), "step" [|p| >= param].
    """
    if kind == "const":
        return np.ones_like(norms)
    if kind == "pow":
        return norms ** param
    if kind == "sigmoid":
        return 1.0 / (1.0 + np.exp(-param * norms))
    if kind == "step":
        return (norms >= param).astype(np.float64)
    raise ValueError(kind)


def assign(p: np.ndarray, z: np.ndarray):
    """Nearest centre of every row (lowest centre index on ties), its squared
    distance, and the gap to the second-nearest centre."""
    d = cdist(p, z, "sqeuclidean")
    lab = np.argmin(d, axis=1)
    dmin = d[np.arange(d.shape[0]), lab]
    if d.shape[1] > 1:
        part = np.partition(d, 1, axis=1)
        gap = part[:, 1] - part[:, 0]
    else:
        gap = np.full(d.shape[0], np.inf)
    return lab, dmin, gap


def centroid_update(p: np.ndarray, w: np.ndarray, lab: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Weighted means of the clusters; a centre whose cluster has zero total
    weight (empty cluster) keeps its position (reading: the paper is silent)."""
    z = z.copy()
    for j in range(z.shape[0]):
        sel = lab == j
        wsum = float(w[sel].sum())
        if wsum > 0.0:
            z[j] = (w[sel] @ p[sel]) / wsum
    return z


@dataclasses.dataclass
class KMeansResult:
    Z: np.ndarray
    labels: np.ndarray          # assignment to the final centres
    objective: list             # weighted encoding error at every assignment step
    e_initial: float            # objective with the initial centres (the pilot sample)
    e_final: float              # objective with the final centres
    max_cluster: int            # T, the largest cluster (Section 3.1)
    min_gap: float              # smallest nearest/second-nearest gap of the final assignment


def weighted_kmeans(p: np.ndarray, w: np.ndarray, z0: np.ndarray, iters: int) -> KMeansResult:
    """Lloyd iterations on sum_l w_l |P_l - Z_s(l)|^2 (Section 3.2, weighted objective).

    Reading: a fixed number c of iterations (c = 5 in the paper, Section 4),
    each an assignment followed by a weighted mean update.  The loop leaves
    early only when the assignment repeats, after which every further
    iteration would be a no-op, so the result equals the full c iterations.
    """
    z = np.array(z0, dtype=np.float64, copy=True)
    objective = []
    prev = None
    for _ in range(iters):
        lab, dmin, _ = assign(p, z)
        objective.append(float(w @ dmin))
        if prev is not None and np.array_equal(lab, prev):
            break
        z = centroid_update(p, w, lab, z)
        prev = lab
    lab, dmin, gap = assign(p, z)
    objective.append(float(w @ dmin))
    counts = np.bincount(lab, minlength=z.shape[0])
    return KMeansResult(Z=z, labels=lab, objective=objective, e_initial=objective[0],
                        e_final=objective[-1], max_cluster=int(counts.max()),
                        min_gap=float(gap.min()) if gap.size else math.inf)


SNAP_TIE_RTOL = 1e-11


def hard_threshold(w: np.ndarray, k: int) -> np.ndarray:
    """The hard-threshold follow-up of Section 5: the k rows with the largest
    weighting coefficients (the weights of the weighted k-means objective,
    Section 3.2), instead of the k-means centres.  Reading (the paper gives no
    tie rule): equal weights go to the lower row index; NaN weights are never
    chosen before a number.  Returned ascending."""
    w = np.asarray(w, dtype=np.float64)
    key = np.where(np.isnan(w), -np.inf, w)
    order = np.lexsort((np.arange(w.size), -key))  # primary: weight descending; then index ascending
    return np.sort(order[:k]).astype(np.int64)


def leverage_scores(u: np.ndarray, s: np.ndarray, p: int) -> np.ndarray:
    """Approximate leverage scores of the rows of A (Section 5's leverage variant, made possible
    by the orthogonalisation of the supplementary material): the squared row norms of the pilot
    sketch's left factor U (orthonormal after orthogonalisation).  Reading: only components whose
    singular value exceeds p * eps * max(s), p = min(k1_rows, k1_cols), count, since a component
    below that cut carries no information about A."""
    s = np.asarray(s, dtype=np.float64)
    keep = s > p * EPS * s.max() if s.size and s.max() > 0.0 else np.zeros(s.size, dtype=bool)
    return (u[:, keep] ** 2).sum(axis=1)


def leverage_sample(scores: np.ndarray, k: int, seed: int, stream: int) -> np.ndarray:
    """k distinct rows drawn with probabilities proportional to `scores`, without replacement
    (Section 5's leverage variant; the paper does not say how).  Reading: weighted sampling
    without replacement by exponential races (Efraimidis and Spirakis, Inf. Proc. Letters 97(5),
    2006): row i gets key ln(u_i) / score_i with u_i in (0, 1] from the counter-based generator
    (unit_draws on `stream`), rows of score 0 get -inf, and the k largest keys are taken, equal
    keys to the lower row.  This is the law of drawing k rows one after another, each with
    probability proportional to its score among the rows not yet drawn.  Returned ascending."""
    u = philox.unit_draws(scores.size, seed, stream)
    with np.errstate(divide="ignore", invalid="ignore"):
        key = np.where(scores > 0.0, np.log(u) / np.where(scores > 0.0, scores, 1.0), -np.inf)
    return hard_threshold(key, k)


def snap(p: np.ndarray, z: np.ndarray, tie_rtol: float = SNAP_TIE_RTOL) -> np.ndarray:
    """Replace every centre by its nearest in-sample point (Section 3.2).

    Reading: centres are visited in index order; each takes the nearest row of
    P not taken by an earlier centre, so the follow-up sample holds distinct
    rows.  Exact ties are common (the centre of a two-row cluster is the
    midpoint of its rows), so distances within tie_rtol * (|Z_j| + sqrt(d_min))^2
    of the nearest one count as equal and the lowest row index wins.  Returned
    sorted ascending.
    """
    if z.shape[0] > p.shape[0]:
        raise ValueError("more centres than rows")
    d = cdist(p, z, "sqeuclidean")
    zn = np.linalg.norm(z, axis=1)
    taken = np.zeros(p.shape[0], dtype=bool)
    out = np.empty(z.shape[0], dtype=np.int64)
    for j in range(z.shape[0]):
        dj = np.where(taken, np.inf, d[:, j])
        dmin = float(dj.min())
        tol = tie_rtol * (zn[j] + math.sqrt(dmin)) ** 2
        l = int(np.flatnonzero(dj <= dmin + tol)[0])
        taken[l] = True
        out[j] = l
    return np.sort(out)


def initial_centres(emb: np.ndarray, pilot_idx: np.ndarray, k2: int, n_rows: int, seed: int,
                    stream: int) -> np.ndarray:
    """Reading: k-means starts from the pilot sample itself, Z^0 = P[I] (the
    pilot sampling acts on the rank-k embedding, supplementary Section 4), so
    the follow-up encoding error can only go down.  If k2 < k1 the first k2
    pilot indices are used; if k2 > k1 a fresh Floyd sample of k2 rows is
    drawn on stream 2 (rows) or 3 (columns)."""
    if k2 <= pilot_idx.size:
        return emb[pilot_idx[:k2]].copy()
    return emb[philox.floyd_sample(n_rows, k2, seed, stream)].copy()


# ---------------------------------------------------------------------------
# Error metric (Section 5)
# ---------------------------------------------------------------------------

def rel_error_exact(mat: Matrix, c: np.ndarray, umid: np.ndarray, rt: np.ndarray, rows_per_block: int = 256) -> float:
    """|A - C Umid R|_F / |A|_F over every entry."""
    num = 0.0
    den = 0.0
    cu = c @ umid
    for r0 in range(0, mat.m, rows_per_block):
        r1 = min(mat.m, r0 + rows_per_block)
        a = mat.full_rows(r0, r1)
        at = cu[r0:r1] @ rt.T
        num += float(((a - at) ** 2).sum())
        den += float((a * a).sum())
    return math.sqrt(num / den)


def rel_error_sampled(mat: Matrix, c: np.ndarray, umid: np.ndarray, rt: np.ndarray, n_samples: int,
                      seed: int, chunk: int = 1 << 18):
    """The same ratio over n_samples i.i.d. uniform entries (with replacement).

    Returns (ratio, sum of squared residuals, sum of squared entries)."""
    num = 0.0
    den = 0.0
    cu = c @ umid
    for t0 in range(0, n_samples, chunk):
        cnt = min(chunk, n_samples - t0)
        i, j = philox.error_sample_indices(mat.m, mat.n, cnt, seed, start=t0)
        a = mat.entries(i, j)
        at = np.einsum("tk,tk->t", cu[i], rt[j])
        num += float(((a - at) ** 2).sum())
        den += float((a * a).sum())
    return math.sqrt(num / den), num, den


# ---------------------------------------------------------------------------
# The driver (Algorithm 2)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Result:
    pilot_rows: np.ndarray
    pilot_cols: np.ndarray
    idx_r: np.ndarray
    idx_c: np.ndarray
    C: np.ndarray            # m x k2c
    Rt: np.ndarray           # n x k2r
    Umid: np.ndarray         # k2c x k2r
    pilot: Sketch
    final: Sketch
    P: np.ndarray
    Q: np.ndarray
    w_r: np.ndarray
    w_c: np.ndarray
    km_r: Optional[KMeansResult]
    km_c: Optional[KMeansResult]
    entries_touched: int
    factors: Optional[tuple] = None
    pilot_C: Optional[np.ndarray] = None
    pilot_Rt: Optional[np.ndarray] = None
    pilot_sigma: Optional[np.ndarray] = None


def validate(m: int, n: int, prm: Params) -> None:
    for name in ("k1_rows", "k1_cols", "k2_rows", "k2_cols"):
        if getattr(prm, name) < 1:
            raise ValueError(f"{name} must be positive")
    if prm.k1_rows > m or prm.k2_rows > m or prm.k1_cols > n or prm.k2_cols > n:
        raise ValueError("sample size exceeds the matrix dimension")
    if prm.kmeans_iters < 0:
        raise ValueError("kmeans_iters must be >= 0")
    if prm.weight_kind not in WEIGHT_KINDS or prm.sketch_kind not in SKETCH_KINDS:
        raise ValueError("unknown weight or sketch kind")
    if prm.follow_up not in FOLLOW_UPS:
        raise ValueError("unknown follow-up kind")
    if prm.follow_up == "pilot" and (prm.k2_rows != prm.k1_rows or prm.k2_cols != prm.k1_cols):
        raise ValueError("the pilot sketch alone needs k2 = k1 on both sides")


def cabs(spec, prm: Params, track: bool = False) -> Result:
    """Algorithm 2: pilot sampling and sketching, follow-up sampling by weighted
    k-means on the pilot embeddings, follow-up sketching.

    Pilot embeddings (step 2): P = U S^(1/2), Q = V S^(1/2), using the
    orthogonalised triple when ``orthogonalize`` is set.  W is read out of the
    sampled columns C rather than evaluated again, so one round touches
    m kc + n kr - kr kc distinct entries.
    """
    m, n = spec.m, spec.n
    validate(m, n, prm)
    mat = Matrix(spec, track=track)
    touched = 0

    # Step 1: pilot sampling.
    ir = philox.floyd_sample(m, prm.k1_rows, prm.seed, philox.STREAM_PILOT_ROWS)
    ic = philox.floyd_sample(n, prm.k1_cols, prm.seed, philox.STREAM_PILOT_COLS)
    c = mat.cols(ic)
    rt = mat.rows_t(ir)
    w = c[ir, :]
    if track:
        touched += int(mat.mask.sum())
        mat.mask[:] = False
    else:
        touched += m * prm.k1_cols + n * prm.k1_rows - prm.k1_rows * prm.k1_cols

    # Step 2: pilot sketching and embeddings.
    pilot = sketching(c, rt, w, m, n, prm.sketch_kind, prm.pinv_rtol)
    if prm.follow_up == "pilot":
        # the one-shot pilot sketch of Section 5's comparison: steps 3 and 4 are skipped
        factors = orthogonalize(pilot.U, pilot.S, pilot.V) if prm.factors else None
        return Result(pilot_rows=ir, pilot_cols=ic, idx_r=ir, idx_c=ic, C=c, Rt=rt, Umid=pilot.Umid,
                      pilot=pilot, final=pilot, P=None, Q=None, w_r=None, w_c=None, km_r=None, km_c=None,
                      entries_touched=touched, factors=factors, pilot_C=c, pilot_Rt=rt, pilot_sigma=None)
    if prm.orthogonalize:
        uo, so, vo = orthogonalize(pilot.U, pilot.S, pilot.V)
    else:
        uo, so, vo = pilot.U, pilot.S, pilot.V
    root = np.sqrt(so)
    p = uo * root
    q = vo * root

    # Step 3: follow-up sampling by weighted k-means, then snapping (or, in the
    # variants of Section 5, the rows with the largest weights, or rows drawn
    # with probabilities proportional to approximate leverage scores).
    w_r = upsilon(np.linalg.norm(p, axis=1), prm.weight_kind, prm.weight_param)
    w_c = upsilon(np.linalg.norm(q, axis=1), prm.weight_kind, prm.weight_param)
    if prm.follow_up == "hard":
        km_r = km_c = None
        jr = hard_threshold(w_r, prm.k2_rows)
        jc = hard_threshold(w_c, prm.k2_cols)
    elif prm.follow_up == "leverage":
        km_r = km_c = None
        p1 = min(prm.k1_rows, prm.k1_cols)
        jr = leverage_sample(leverage_scores(uo, so, p1), prm.k2_rows, prm.seed, philox.STREAM_LEVERAGE_ROWS)
        jc = leverage_sample(leverage_scores(vo, so, p1), prm.k2_cols, prm.seed, philox.STREAM_LEVERAGE_COLS)
    else:
        z0r = initial_centres(p, ir, prm.k2_rows, m, prm.seed, philox.STREAM_INIT_ROWS)
        z0c = initial_centres(q, ic, prm.k2_cols, n, prm.seed, philox.STREAM_INIT_COLS)
        km_r = weighted_kmeans(p, w_r, z0r, prm.kmeans_iters)
        km_c = weighted_kmeans(q, w_c, z0c, prm.kmeans_iters)
        jr = snap(p, km_r.Z)
        jc = snap(q, km_c.Z)

    cb = mat.cols(jc)
    rtb = mat.rows_t(jr)
    wb = cb[jr, :]
    if track:
        touched += int(mat.mask.sum())
    else:
        touched += m * prm.k2_cols + n * prm.k2_rows - prm.k2_rows * prm.k2_cols

    # Step 4: follow-up sketching.
    final = sketching(cb, rtb, wb, m, n, prm.sketch_kind, prm.pinv_rtol)
    factors = orthogonalize(final.U, final.S, final.V) if prm.factors else None
    return Result(pilot_rows=ir, pilot_cols=ic, idx_r=jr, idx_c=jc, C=cb, Rt=rtb, Umid=final.Umid,
                  pilot=pilot, final=final, P=p, Q=q, w_r=w_r, w_c=w_c, km_r=km_r, km_c=km_c,
                  entries_touched=touched, factors=factors, pilot_C=c, pilot_Rt=rt, pilot_sigma=so)


def reconstruct(res: Result) -> np.ndarray:
    """The dense m x n approximation C Umid R (small inputs only)."""
    return res.C @ res.Umid @ res.Rt.T
