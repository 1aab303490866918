"""Entry access to the input matrix A for the oracle (test infrastructure only).

The method may read A only through the rows and columns it samples (Section 1:
the goal is an O(m+n) sketch that never looks at the remaining entries).  The
accessor therefore exposes whole sampled columns, whole sampled rows and
single entries, and counts what the sketch reads so that tests can check the
linear entry count.  Full rows for the error metric go through a separate,
uncounted path.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial.distance import cdist

from . import philox


class Matrix:
    """Wraps a ``workloads.MatrixSpec`` and evaluates its entries in float64."""

    def __init__(self, spec, track: bool = False):
        self.spec = spec
        self.m = spec.m
        self.n = spec.n
        self.kind = spec.kind
        self.entries_read = 0
        # Optional brute-force record of every distinct entry read (small A only).
        self.mask = np.zeros((self.m, self.n), dtype=bool) if track else None

    # -- plain evaluation -------------------------------------------------
    def _block(self, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
        sp = self.spec
        if sp.kind == "dense":
            return sp.a[np.ix_(rows, cols)].astype(np.float64)
        if sp.kind == "lowrank":
            out = (sp.pf[rows] * sp.s) @ sp.qf[cols].T
            if sp.noise_std != 0.0:
                ii = np.asarray(rows, dtype=np.uint64)[:, None]
                jj = np.asarray(cols, dtype=np.uint64)[None, :]
                out = out + sp.noise_std * philox.normal_at(sp.noise_seed, ii, jj)
            return out
        if sp.kind == "rbf":
            d2 = cdist(sp.x[rows], sp.y[cols], "sqeuclidean")
            return np.exp(-np.maximum(d2, 0.0) / (2.0 * sp.sigma * sp.sigma))
        if sp.kind == "csr":
            return sp.sp[np.asarray(rows)][:, np.asarray(cols)].toarray().astype(np.float64)
        raise ValueError(sp.kind)

    def entries(self, i: np.ndarray, j: np.ndarray) -> np.ndarray:
        """A[i_t, j_t] for paired index vectors (uncounted; used by the error metric)."""
        sp = self.spec
        i = np.asarray(i, dtype=np.int64)
        j = np.asarray(j, dtype=np.int64)
        if sp.kind == "dense":
            return sp.a[i, j].astype(np.float64)
        if sp.kind == "lowrank":
            v = np.einsum("tk,tk->t", sp.pf[i] * sp.s, sp.qf[j])
            if sp.noise_std != 0.0:
                v = v + sp.noise_std * philox.normal_at(sp.noise_seed, i.astype(np.uint64), j.astype(np.uint64))
            return v
        if sp.kind == "rbf":
            diff = sp.x[i] - sp.y[j]
            d2 = np.einsum("tk,tk->t", diff, diff)
            return np.exp(-d2 / (2.0 * sp.sigma * sp.sigma))
        if sp.kind == "csr":
            # the nonzeros in row-major order have sorted keys i * n + j; an entry is listed or 0
            a = sp.sp
            if a.nnz == 0:
                return np.zeros(i.shape)
            keys = np.repeat(np.arange(self.m, dtype=np.int64), np.diff(a.indptr)) * self.n + a.indices
            q = i * self.n + j
            pos = np.minimum(np.searchsorted(keys, q), keys.size - 1)
            return np.where(keys[pos] == q, a.data[pos], 0.0).astype(np.float64)
        raise ValueError(sp.kind)

    def full_rows(self, r0: int, r1: int) -> np.ndarray:
        """Rows r0..r1-1 in full (uncounted; used only by the exact error metric)."""
        return self._block(np.arange(r0, r1), np.arange(self.n))

    # -- counted access used by the sketch --------------------------------
    def cols(self, idx: np.ndarray) -> np.ndarray:
        """C = A(:, idx), m x len(idx)."""
        idx = np.asarray(idx, dtype=np.int64)
        self.entries_read += self.m * idx.size
        if self.mask is not None:
            self.mask[:, idx] = True
        return self._block(np.arange(self.m), idx)

    def rows_t(self, idx: np.ndarray) -> np.ndarray:
        """R^T = A(idx, :)^T, n x len(idx) (rows are stored transposed)."""
        idx = np.asarray(idx, dtype=np.int64)
        self.entries_read += self.n * idx.size
        if self.mask is not None:
            self.mask[idx, :] = True
        return np.ascontiguousarray(self._block(idx, np.arange(self.n)).T)

    def block(self, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
        """A(rows, cols), len(rows) x len(cols): the target block of the resampling CUR."""
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        self.entries_read += rows.size * cols.size
        if self.mask is not None:
            self.mask[np.ix_(rows, cols)] = True
        return self._block(rows, cols)
