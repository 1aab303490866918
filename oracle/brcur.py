"""Bilateral resampling CUR and the linear-cost methods it contains, in float64
(test infrastructure only).

Section 2.2 frames the linear-cost sketches as one procedure (Algorithm 1,
BR-CUR): a base sample of rows I_r^b and columns I_c^b gives the factors
C = A(:, I_c^b) and R = A(I_r^b, :); a target sample I_r^t, I_c^t picks the
rows of C and the columns of R that are compared with the target block
M = A(I_r^t, I_c^t); the middle factor minimises the misfit on that block,
    U* = argmin_U |M - C(I_r^t, :) U R(:, I_c^t)|_F,
and A ~ C U* R.  Its special cases:
  * pseudo-skeleton, Eq. (W): the target sample is the base sample, so the
    compared rows and columns meet in W = A(I_r^b, I_c^b) and U* = W^+;
  * Nystrom: a symmetric positive semi-definite A with one sample used for the
    rows and the columns of both rounds, A ~ C W^+ C^T;
  * Sketch-CUR: base and target drawn independently, at different rates (the
    experiments of Section 5 use a target rate three times the base rate).
The pilot sketch of Algorithm 2 (the stabilised routine of Section 4.1 on one
uniform sample) is the sixth method of Section 5's comparison and is given here
in the same one-shot form.

Readings (where the paper leaves the choice open):
  * U* is the minimum-norm minimiser, U* = Cbar^+ M Rbar^+ (for full-rank Cbar
    and Rbar it is the only one); each pseudo-inverse drops the singular values
    that do not exceed tol = max(rows, cols) eps sigma_1 (or rtol sigma_1), the
    same truncation as the sketching routine's, and optionally keeps at most
    ``rank_cap`` of them (the supplementary stability figure varies the number
    of singular vectors used).
  * Draws: the base rows and columns come from the pilot streams (0 and 1), so
    that every one-shot method sees the same base sample for one seed; the
    target rows and columns from streams 7 and 8; Nystrom uses the column
    stream for its one sample.  All are Floyd's algorithm on Philox-4x64-10.
  * Sketch-CUR's target size is min(dim, ratio * base size), ratio 3 by default.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import philox
from .cabs import EPS, Params, cabs
from .matrices import Matrix


def pinv(a: np.ndarray, rtol: float = 0.0, rank_cap: int = 0):
    """Truncated pseudo-inverse from the thin SVD a = U diag(s) V^T:
    a^+ = V diag(1/s_i) U^T over the kept components i (s_i > tol, and i < rank_cap
    when rank_cap > 0).  Returns (a^+, kept count, s_1)."""
    u, s, vt = np.linalg.svd(a, full_matrices=False)
    s1 = float(s[0]) if s.size else 0.0
    tol = (rtol if rtol > 0.0 else max(a.shape) * EPS) * s1
    keep = s > tol
    if rank_cap > 0:
        keep &= np.arange(s.size) < rank_cap
    inv = np.where(keep, 1.0 / np.where(keep, s, 1.0), 0.0)
    return (vt.T * inv) @ u.T, int(keep.sum()), s1


@dataclasses.dataclass
class BrCurResult:
    base_r: np.ndarray
    base_c: np.ndarray
    tgt_r: Optional[np.ndarray]   # None: the target sample is the base sample
    tgt_c: Optional[np.ndarray]
    C: np.ndarray                 # m x kb_c
    Rt: np.ndarray                # n x kb_r (R stored transposed)
    Umid: np.ndarray              # kb_c x kb_r: A ~ C Umid Rt^T
    rank_c: int                   # kept components of Cbar^+ (of W^+ when the samples coincide)
    rank_r: int                   # kept components of Rbar^+ (the same as rank_c then)
    sigma1_c: float
    sigma1_r: float
    entries: int                  # entries of A read: m kb_c + n kb_r (+ kt_r kt_c for a separate target)


def br_cur(spec, base_r, base_c, tgt_r=None, tgt_c=None, pinv_rtol: float = 0.0, rank_cap: int = 0,
           track: bool = False) -> BrCurResult:
    """Algorithm 1 on the given samples (tgt_r = tgt_c = None: the target sample is the base sample)."""
    if (tgt_r is None) != (tgt_c is None):
        raise ValueError("give both target samples or neither")
    base_r = np.asarray(base_r, dtype=np.int64)
    base_c = np.asarray(base_c, dtype=np.int64)
    mat = Matrix(spec, track=track)
    c = mat.cols(base_c)            # step 1: the bases C and R
    rt = mat.rows_t(base_r)
    if tgt_r is None:
        # Eq. (W): the compared block is the intersection W = C(I_r^b, :) = A(I_r^b, I_c^b), U* = W^+
        x, rank, s1 = pinv(c[base_r, :], pinv_rtol, rank_cap)
        return BrCurResult(base_r, base_c, None, None, c, rt, x, rank, rank, s1, s1, mat.entries_read)
    tgt_r = np.asarray(tgt_r, dtype=np.int64)
    tgt_c = np.asarray(tgt_c, dtype=np.int64)
    cbar = c[tgt_r, :]              # step 2: the bases on the target sample
    rbar = rt[tgt_c, :].T
    m_blk = mat.block(tgt_r, tgt_c)  # step 3: the target block
    xc, rank_c, s1c = pinv(cbar, pinv_rtol, rank_cap)   # step 4: the minimum-norm minimiser
    xr, rank_r, s1r = pinv(rbar, pinv_rtol, rank_cap)
    umid = xc @ m_blk @ xr
    return BrCurResult(base_r, base_c, tgt_r, tgt_c, c, rt, umid, rank_c, rank_r, s1c, s1r, mat.entries_read)


def base_sample(spec, k_rows: int, k_cols: int, seed: int):
    """The uniform base sample (the pilot streams of Algorithm 2)."""
    return (philox.floyd_sample(spec.m, k_rows, seed, philox.STREAM_PILOT_ROWS),
            philox.floyd_sample(spec.n, k_cols, seed, philox.STREAM_PILOT_COLS))


def target_sample(spec, k_rows: int, k_cols: int, seed: int):
    """The independent uniform target sample of Sketch-CUR."""
    return (philox.floyd_sample(spec.m, k_rows, seed, philox.STREAM_TARGET_ROWS),
            philox.floyd_sample(spec.n, k_cols, seed, philox.STREAM_TARGET_COLS))


def sketch_cur(spec, k_rows: int, k_cols: int, seed: int, ratio: int = 3, pinv_rtol: float = 0.0,
               rank_cap: int = 0) -> BrCurResult:
    """Sketch-CUR: independent base (k_rows x k_cols) and target (ratio times as many) samples."""
    br, bc = base_sample(spec, k_rows, k_cols, seed)
    tr, tc = target_sample(spec, min(spec.m, ratio * k_rows), min(spec.n, ratio * k_cols), seed)
    return br_cur(spec, br, bc, tr, tc, pinv_rtol, rank_cap)


def pseudo_skeleton(spec, k_rows: int, k_cols: int, seed: int, pinv_rtol: float = 0.0,
                    rank_cap: int = 0) -> BrCurResult:
    """Eq. (W) on the uniform base sample: A ~ C W^+ R."""
    br, bc = base_sample(spec, k_rows, k_cols, seed)
    return br_cur(spec, br, bc, None, None, pinv_rtol, rank_cap)


def nystrom(spec, k: int, seed: int, pinv_rtol: float = 0.0, rank_cap: int = 0) -> BrCurResult:
    """Nystrom: one uniform sample I for rows and columns of a square matrix, A ~ A(:, I) W^+ A(I, :)."""
    if spec.m != spec.n:
        raise ValueError("the Nystrom method needs a square matrix")
    i = philox.floyd_sample(spec.n, k, seed, philox.STREAM_PILOT_COLS)
    return br_cur(spec, i, i, None, None, pinv_rtol, rank_cap)


def pilot_sketch(spec, k_rows: int, k_cols: int, seed: int, pinv_rtol: float = 0.0) -> BrCurResult:
    """Step 2 of Algorithm 2 alone: the stabilised sketching routine on the uniform base sample
    (the pilot sample of Algorithm 2 for the same seed)."""
    res = cabs(spec, Params(k_rows, k_cols, k_rows, k_cols, follow_up="pilot", pinv_rtol=pinv_rtol, seed=seed))
    r = int(res.final.keep.sum())
    s1 = float(res.final.sw[0])
    return BrCurResult(res.idx_r, res.idx_c, None, None, res.C, res.Rt, res.Umid, r, r, s1, s1,
                       res.entries_touched + k_rows * k_cols)
