"""Python binding of libcabs: argument marshalling over the C ABI.

Device memory and streams come from PyTorch (ROCm); every computation runs in
the library's HIP kernels.  Names follow the C ABI (``cabs_sketch`` ->
:func:`sketch`, ``cabs_error`` -> :func:`error`, ...).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _ffi as F

PREC = {"f64": F.F64, "f32": F.F32, "bf16": F.BF16, "f16": F.F16}
TORCH_DTYPE = {F.F64: torch.float64, F.F32: torch.float32, F.BF16: torch.bfloat16, F.F16: torch.float16}
WEIGHT = {"const": F.W_CONST, "pow": F.W_POW, "sigmoid": F.W_SIGMOID, "step": F.W_STEP}
SKETCH = {"stabilized": F.SK_STABILIZED, "pseudo_skeleton": F.SK_PSEUDO_SKELETON}
FOLLOW = {"kmeans": F.FOLLOW_KMEANS, "hard": F.FOLLOW_HARD, "leverage": F.FOLLOW_LEVERAGE, "pilot": F.FOLLOW_PILOT}
SOURCE = {"dense": F.SRC_DENSE, "lowrank": F.SRC_LOWRANK, "rbf": F.SRC_RBF, "csr": F.SRC_CSR}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_alloc(nbytes: int, device) -> torch.Tensor:
    # 256-byte aligned by the caching allocator
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class DeviceMatrix:
    """Device copies of a matrix description (``workloads.MatrixSpec``) and its descriptor."""

    def __init__(self, spec, storage: str = "f32", device="cuda"):
        self.spec = spec
        self.storage = PREC[storage]
        if self.storage not in (F.F64, F.F32):
            raise ValueError("table storage must be f64 or f32")
        dt = TORCH_DTYPE[self.storage]
        self.device = torch.device(device)
        self._keep = []

        def put(arr):
            if arr is None:
                return None
            t = torch.from_numpy(np.ascontiguousarray(arr)).to(device=self.device, dtype=dt).contiguous()
            self._keep.append(t)
            return t

        d = F.CabsMatrix()
        d.kind = SOURCE[spec.kind]
        d.storage = self.storage
        d.m, d.n = spec.m, spec.n
        if spec.kind == "dense":
            self.a = put(spec.a)
            d.a, d.lda = self.a.data_ptr(), spec.n
        elif spec.kind == "lowrank":
            self.pf, self.qf, self.s = put(spec.pf), put(spec.qf), put(spec.s)
            d.pf, d.qf, d.s, d.r = self.pf.data_ptr(), self.qf.data_ptr(), self.s.data_ptr(), spec.r
            d.noise_std, d.noise_seed = spec.noise_std, spec.noise_seed
        elif spec.kind == "rbf":
            self.x = put(spec.x)
            self.y = self.x if spec.y is spec.x else put(spec.y)
            d.x, d.y, d.d, d.sigma = self.x.data_ptr(), self.y.data_ptr(), spec.d, spec.sigma
        elif spec.kind == "csr":
            a = spec.sp
            t = a.tocsc()
            t.sort_indices()

            def put_i(arr, dtype):
                x = torch.from_numpy(np.ascontiguousarray(arr.astype(dtype))).to(self.device)
                self._keep.append(x)
                return x
            self.row_ptr, self.col_idx, self.vals = put_i(a.indptr, np.int64), put_i(a.indices, np.int32), put(a.data)
            self.col_ptr, self.row_idx, self.vals_t = put_i(t.indptr, np.int64), put_i(t.indices, np.int32), put(t.data)
            d.row_ptr, d.col_idx, d.vals = self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.vals.data_ptr()
            d.col_ptr, d.row_idx, d.vals_t = self.col_ptr.data_ptr(), self.row_idx.data_ptr(), self.vals_t.data_ptr()
            d.nnz = int(a.nnz)
        else:
            raise ValueError(spec.kind)
        self.desc = d

    @property
    def m(self):
        return self.spec.m

    @property
    def n(self):
        return self.spec.n


def make_params(k1_rows, k1_cols, k2_rows, k2_cols, kmeans_iters=5, weight="const", weight_param=0.0,
                sketch="stabilized", orthogonalize=True, pinv_rtol=0.0, compute="f32", factors=False,
                seed=0, follow_up="kmeans", count_entries=False) -> F.CabsParams:
    p = F.CabsParams()
    p.k1_rows, p.k1_cols, p.k2_rows, p.k2_cols = k1_rows, k1_cols, k2_rows, k2_cols
    p.kmeans_iters = kmeans_iters
    p.weight_kind = WEIGHT[weight]
    p.weight_param = weight_param
    p.sketch_kind = SKETCH[sketch]
    p.orthogonalize = 1 if orthogonalize else 0
    p.pinv_rtol = pinv_rtol
    p.compute = PREC[compute]
    p.want_factors = 1 if factors else 0
    p.follow_up = FOLLOW[follow_up]
    p.flags = F.FLAG_COUNT_ENTRIES if count_entries else 0
    p.seed = seed
    return p


@dataclasses.dataclass
class SketchResult:
    idx_r: torch.Tensor
    idx_c: torch.Tensor
    pilot_r: torch.Tensor
    pilot_c: torch.Tensor
    C: torch.Tensor
    Rt: torch.Tensor
    Umid: torch.Tensor
    diag: torch.Tensor
    Uf: Optional[torch.Tensor] = None
    S: Optional[torch.Tensor] = None
    Vf: Optional[torch.Tensor] = None
    struct: Optional[F.CabsResult] = None

    def diagnostics(self) -> dict:
        d = self.diag.cpu().numpy()
        return {"status": int(d[F.DIAG_STATUS]), "enc_r_pilot": d[F.DIAG_ENC_R_PILOT], "enc_c_pilot": d[F.DIAG_ENC_C_PILOT],
                "enc_r_final": d[F.DIAG_ENC_R_FINAL], "enc_c_final": d[F.DIAG_ENC_C_FINAL],
                "tmax_r": int(d[F.DIAG_TMAX_R]), "tmax_c": int(d[F.DIAG_TMAX_C]),
                "rank_pilot": int(d[F.DIAG_RANK_PILOT]), "rank_final": int(d[F.DIAG_RANK_FINAL]),
                "entries": int(d[F.DIAG_ENTRIES]), "gap_r": d[F.DIAG_GAP_R], "gap_c": d[F.DIAG_GAP_C],
                "sigma1_pilot": d[F.DIAG_SIGMA1_PILOT], "sigma1_final": d[F.DIAG_SIGMA1_FINAL],
                "snap_scans_r": int(d[F.DIAG_SNAP_SCANS_R]), "snap_scans_c": int(d[F.DIAG_SNAP_SCANS_C])}


def alloc_result(mat: DeviceMatrix, prm: F.CabsParams) -> SketchResult:
    dev = mat.device
    dt = TORCH_DTYPE[prm.compute]
    kf = min(prm.k2_rows, prm.k2_cols)
    r = SketchResult(
        idx_r=torch.empty(prm.k2_rows, dtype=torch.int64, device=dev),
        idx_c=torch.empty(prm.k2_cols, dtype=torch.int64, device=dev),
        pilot_r=torch.empty(prm.k1_rows, dtype=torch.int64, device=dev),
        pilot_c=torch.empty(prm.k1_cols, dtype=torch.int64, device=dev),
        C=torch.empty(mat.m, prm.k2_cols, dtype=dt, device=dev),
        Rt=torch.empty(mat.n, prm.k2_rows, dtype=dt, device=dev),
        Umid=torch.empty(prm.k2_cols, prm.k2_rows, dtype=torch.float64, device=dev),
        diag=torch.empty(F.DIAG_LEN, dtype=torch.float64, device=dev),
    )
    if prm.want_factors:
        r.Uf = torch.empty(mat.m, kf, dtype=dt, device=dev)
        r.S = torch.empty(kf, dtype=torch.float64, device=dev)
        r.Vf = torch.empty(mat.n, kf, dtype=dt, device=dev)
    s = F.CabsResult()
    s.idx_r, s.idx_c = r.idx_r.data_ptr(), r.idx_c.data_ptr()
    s.pilot_r, s.pilot_c = r.pilot_r.data_ptr(), r.pilot_c.data_ptr()
    s.C, s.Rt, s.Umid, s.diag = r.C.data_ptr(), r.Rt.data_ptr(), r.Umid.data_ptr(), r.diag.data_ptr()
    if prm.want_factors:
        s.Uf, s.S, s.Vf = r.Uf.data_ptr(), r.S.data_ptr(), r.Vf.data_ptr()
    r.struct = s
    return r


def workspace_bytes(mat: DeviceMatrix, prm: F.CabsParams) -> int:
    n = F.lib().cabs_workspace_bytes(C.byref(mat.desc), C.byref(prm))
    if n == 0:
        raise F.CabsError(F.EINVAL, "cabs_workspace_bytes")
    return int(n)


def error_workspace_bytes(mat: DeviceMatrix, prm: F.CabsParams, n_samples: int) -> int:
    n = F.lib().cabs_error_workspace_bytes(C.byref(mat.desc), C.byref(prm), n_samples)
    if n == 0:
        raise F.CabsError(F.EINVAL, "cabs_error_workspace_bytes")
    return int(n)


def sketch(mat: DeviceMatrix, prm: F.CabsParams, ws: Optional[torch.Tensor] = None,
           out: Optional[SketchResult] = None, stream=None) -> SketchResult:
    """cabs_sketch: enqueue one CABS sketch on the current (or given) stream."""
    need = workspace_bytes(mat, prm)
    if ws is None or ws.numel() < need:
        ws = _dev_alloc(need, mat.device)
    if out is None:
        out = alloc_result(mat, prm)
    st = F.lib().cabs_sketch(C.byref(mat.desc), C.byref(prm), _ptr(ws), ws.numel(), C.byref(out.struct),
                             _stream(stream))
    F.check(st, "cabs_sketch")
    out._ws = ws
    return out


def sketch_batch(mats, prms, stream=None):
    """cabs_sketch_batch: 1-4 same-shape sketches with their SVDs batched; returns their results."""
    n = len(mats)
    M = (F.CabsMatrix * n)(*[m.desc for m in mats])
    P = (F.CabsParams * n)(*prms)
    outs = [alloc_result(m, p) for m, p in zip(mats, prms)]
    R = (F.CabsResult * n)(*[o.struct for o in outs])
    wss = [_dev_alloc(workspace_bytes(m, p), m.device) for m, p in zip(mats, prms)]
    W = (C.c_void_p * n)(*[w.data_ptr() for w in wss])
    B = (C.c_size_t * n)(*[w.numel() for w in wss])
    F.check(F.lib().cabs_sketch_batch(n, M, P, W, B, R, _stream(stream)), "cabs_sketch_batch")
    for o, w in zip(outs, wss):
        o._ws = w
    return outs


def error(mat: DeviceMatrix, prm: F.CabsParams, res: SketchResult, n_samples: int = 0, seed: int = 0,
          ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """cabs_error: returns a device tensor [sum sq residual, sum sq entries, ratio]."""
    need = int(F.lib().cabs_error_workspace_bytes(C.byref(mat.desc), C.byref(prm), n_samples))
    if need == 0:
        raise F.CabsError(F.EINVAL, "cabs_error_workspace_bytes")
    if ws is None or ws.numel() < need:
        ws = _dev_alloc(need, mat.device)
    out3 = torch.empty(3, dtype=torch.float64, device=mat.device)
    st = F.lib().cabs_error(C.byref(mat.desc), C.byref(prm), C.byref(res.struct), n_samples, seed, _ptr(ws),
                            ws.numel(), _ptr(out3), _stream(stream))
    F.check(st, "cabs_error")
    out3._ws = ws
    return out3


# ---------------------------------------------------------------------------
# Bilateral resampling CUR (cabs_brcur) and its special cases
# ---------------------------------------------------------------------------
STREAM_PILOT_ROWS, STREAM_PILOT_COLS, STREAM_TARGET_ROWS, STREAM_TARGET_COLS = 0, 1, 7, 8


@dataclasses.dataclass
class BrCurResult:
    base_r: torch.Tensor
    base_c: torch.Tensor
    tgt_r: Optional[torch.Tensor]
    tgt_c: Optional[torch.Tensor]
    C: torch.Tensor
    Rt: torch.Tensor
    Umid: torch.Tensor
    diag: torch.Tensor
    params: F.CabsParams          # sizes and precision for cabs_error (k2 = the base sizes)
    struct: F.CabsResult          # C, Rt, Umid for cabs_error

    def diagnostics(self) -> dict:
        d = self.diag.cpu().numpy()
        return {"status": int(d[F.BRCUR_DIAG_STATUS]), "rank_c": int(d[F.BRCUR_DIAG_RANK_C]),
                "rank_r": int(d[F.BRCUR_DIAG_RANK_R]), "sigma1_c": d[F.BRCUR_DIAG_SIGMA1_C],
                "sigma1_r": d[F.BRCUR_DIAG_SIGMA1_R]}


def brcur(mat: DeviceMatrix, base_r: torch.Tensor, base_c: torch.Tensor, tgt_r: Optional[torch.Tensor] = None,
          tgt_c: Optional[torch.Tensor] = None, compute: str = "f32", pinv_rtol: float = 0.0, rank_cap: int = 0,
          ws: Optional[torch.Tensor] = None, stream=None) -> BrCurResult:
    """cabs_brcur: Algorithm 1 on device index tensors (no target: the target sample is the base sample)."""
    prm = F.CabsBrCurParams()
    prm.kb_rows, prm.kb_cols = base_r.numel(), base_c.numel()
    same = tgt_r is None
    prm.kt_rows = prm.kb_rows if same else tgt_r.numel()
    prm.kt_cols = prm.kb_cols if same else tgt_c.numel()
    prm.compute = PREC[compute]
    prm.rank_cap = rank_cap
    prm.pinv_rtol = pinv_rtol
    need = int(F.lib().cabs_brcur_workspace_bytes(C.byref(mat.desc), C.byref(prm), 1 if same else 0))
    if need == 0:
        raise F.CabsError(F.EINVAL, "cabs_brcur_workspace_bytes: " + F.lib().cabs_last_error().decode())
    if ws is None or ws.numel() < need:
        ws = _dev_alloc(need, mat.device)
    dt = TORCH_DTYPE[prm.compute]
    dev = mat.device
    c = torch.empty(mat.m, prm.kb_cols, dtype=dt, device=dev)
    rt = torch.empty(mat.n, prm.kb_rows, dtype=dt, device=dev)
    umid = torch.empty(prm.kb_cols, prm.kb_rows, dtype=torch.float64, device=dev)
    diag = torch.empty(F.BRCUR_DIAG_LEN, dtype=torch.float64, device=dev)
    st = F.lib().cabs_brcur(C.byref(mat.desc), C.byref(prm), _ptr(base_r), _ptr(base_c), _ptr(tgt_r), _ptr(tgt_c),
                            _ptr(ws), ws.numel(), _ptr(c), _ptr(rt), _ptr(umid), _ptr(diag), _stream(stream))
    F.check(st, "cabs_brcur")
    eprm = make_params(prm.kb_rows, prm.kb_cols, prm.kb_rows, prm.kb_cols, compute=compute)
    s = F.CabsResult()
    s.C, s.Rt, s.Umid = c.data_ptr(), rt.data_ptr(), umid.data_ptr()
    res = BrCurResult(base_r, base_c, tgt_r, tgt_c, c, rt, umid, diag, eprm, s)
    res._ws = ws
    return res


def sketch_cur(mat: DeviceMatrix, k_rows: int, k_cols: int, seed: int, ratio: int = 3, compute: str = "f32",
               pinv_rtol: float = 0.0, rank_cap: int = 0, stream=None) -> BrCurResult:
    """Sketch-CUR: uniform base sample (streams 0 / 1) and an independent target sample ratio times as
    large (streams 7 / 8), both by cabs_sample."""
    br = sample(mat.m, k_rows, seed, STREAM_PILOT_ROWS, mat.device, stream)
    bc = sample(mat.n, k_cols, seed, STREAM_PILOT_COLS, mat.device, stream)
    tr = sample(mat.m, min(mat.m, ratio * k_rows), seed, STREAM_TARGET_ROWS, mat.device, stream)
    tc = sample(mat.n, min(mat.n, ratio * k_cols), seed, STREAM_TARGET_COLS, mat.device, stream)
    return brcur(mat, br, bc, tr, tc, compute, pinv_rtol, rank_cap, stream=stream)


def pseudo_skeleton(mat: DeviceMatrix, k_rows: int, k_cols: int, seed: int, compute: str = "f32",
                    pinv_rtol: float = 0.0, rank_cap: int = 0, stream=None) -> BrCurResult:
    """Eq. (W) on the uniform base sample: A ~ C W^+ R."""
    br = sample(mat.m, k_rows, seed, STREAM_PILOT_ROWS, mat.device, stream)
    bc = sample(mat.n, k_cols, seed, STREAM_PILOT_COLS, mat.device, stream)
    return brcur(mat, br, bc, None, None, compute, pinv_rtol, rank_cap, stream=stream)


def nystrom(mat: DeviceMatrix, k: int, seed: int, compute: str = "f32", pinv_rtol: float = 0.0, rank_cap: int = 0,
            stream=None) -> BrCurResult:
    """Nystrom: one uniform sample (stream 1) for the rows and columns of a square matrix."""
    if mat.m != mat.n:
        raise ValueError("the Nystrom method needs a square matrix")
    i = sample(mat.n, k, seed, STREAM_PILOT_COLS, mat.device, stream)
    return brcur(mat, i, i, None, None, compute, pinv_rtol, rank_cap, stream=stream)


def sample(n: int, k: int, seed: int, stream_id: int, device="cuda", stream=None) -> torch.Tensor:
    """cabs_sample: k distinct sorted indices of [0, n) (Floyd on Philox)."""
    out = torch.empty(k, dtype=torch.int64, device=device)
    F.check(F.lib().cabs_sample(n, k, seed, stream_id, _ptr(out), _stream(stream)), "cabs_sample")
    return out


def eval_cols(mat: DeviceMatrix, idx: torch.Tensor, compute: str = "f32", stream=None) -> torch.Tensor:
    """cabs_eval_cols: A(:, idx) as an m x k tensor."""
    p = PREC[compute]
    out = torch.empty(mat.m, idx.numel(), dtype=TORCH_DTYPE[p], device=mat.device)
    F.check(F.lib().cabs_eval_cols(C.byref(mat.desc), _ptr(idx), idx.numel(), p, _ptr(out), _stream(stream)),
            "cabs_eval_cols")
    return out


def eval_rows_t(mat: DeviceMatrix, idx: torch.Tensor, compute: str = "f32", stream=None) -> torch.Tensor:
    """cabs_eval_rows_t: A(idx, :)^T as an n x k tensor."""
    p = PREC[compute]
    out = torch.empty(mat.n, idx.numel(), dtype=TORCH_DTYPE[p], device=mat.device)
    F.check(F.lib().cabs_eval_rows_t(C.byref(mat.desc), _ptr(idx), idx.numel(), p, _ptr(out), _stream(stream)),
            "cabs_eval_rows_t")
    return out


def svd(a: torch.Tensor, stream=None, fast_sweeps=None):
    """cabs_svd (cabs_svd_ex when fast_sweeps is given) on a (batch, rows, cols) or (rows, cols)
    float64 device tensor -> U, S, V."""
    squeeze = a.dim() == 2
    a3 = (a[None] if squeeze else a).contiguous()
    if a3.dtype != torch.float64:
        raise TypeError("cabs_svd works in float64")
    b, rows, cols = a3.shape
    p = min(rows, cols)
    U = torch.empty(b, rows, p, dtype=torch.float64, device=a.device)
    S = torch.empty(b, p, dtype=torch.float64, device=a.device)
    V = torch.empty(b, cols, p, dtype=torch.float64, device=a.device)
    need = int(F.lib().cabs_svd_workspace_bytes(b, rows, cols))
    if need == 0:
        raise F.CabsError(F.EINVAL, "cabs_svd_workspace_bytes")
    ws = _dev_alloc(need, a.device)
    if fast_sweeps is None:
        F.check(F.lib().cabs_svd(b, rows, cols, _ptr(a3), _ptr(U), _ptr(S), _ptr(V), _ptr(ws), ws.numel(),
                                 _stream(stream)), "cabs_svd")
    else:
        F.check(F.lib().cabs_svd_ex(b, rows, cols, _ptr(a3), _ptr(U), _ptr(S), _ptr(V), _ptr(ws), ws.numel(),
                                    int(fast_sweeps), _stream(stream)), "cabs_svd_ex")
    if squeeze:
        return U[0], S[0], V[0]
    return U, S, V


def kmeans(P: torch.Tensor, w: torch.Tensor, Z0: torch.Tensor, iters: int, snap: bool = True, stream=None):
    """cabs_kmeans -> (Z, labels, obj2, snapped indices or None)."""
    rows, dim = P.shape
    k = Z0.shape[0]
    prec = {torch.float64: F.F64, torch.float32: F.F32, torch.bfloat16: F.BF16, torch.float16: F.F16}[P.dtype]
    dev = P.device
    Z = torch.empty(k, dim, dtype=torch.float64, device=dev)
    labels = torch.empty(rows, dtype=torch.int32, device=dev)
    obj2 = torch.empty(2, dtype=torch.float64, device=dev)
    sn = torch.empty(k, dtype=torch.int64, device=dev) if snap else None
    need = int(F.lib().cabs_kmeans_workspace_bytes(rows, dim, k, prec))
    if need == 0:
        raise F.CabsError(F.EINVAL, "cabs_kmeans_workspace_bytes")
    ws = _dev_alloc(need, dev)
    F.check(F.lib().cabs_kmeans(rows, dim, k, prec, _ptr(P.contiguous()), _ptr(w.contiguous()),
                                _ptr(Z0.contiguous()), iters, _ptr(Z), _ptr(labels), _ptr(obj2), _ptr(sn), _ptr(ws),
                                ws.numel(), _stream(stream)), "cabs_kmeans")
    return Z, labels, obj2, sn


def kmeans_noalloc(P: torch.Tensor, w: torch.Tensor, Z0: torch.Tensor, iters: int, snap: bool = True,
                   out=None, stream=None):
    """cabs_kmeans_noalloc -> (Z, labels, obj2, snapped indices or None).  Outputs are allocated
    here unless `out` = (Z, labels, obj2, snap) is given; the library call itself allocates nothing."""
    rows, dim = P.shape
    k = Z0.shape[0]
    prec = {torch.float64: F.F64, torch.float32: F.F32, torch.bfloat16: F.BF16, torch.float16: F.F16}[P.dtype]
    dev = P.device
    if out is None:
        out = (torch.empty(k, dim, dtype=torch.float64, device=dev), torch.empty(rows, dtype=torch.int32, device=dev),
               torch.empty(2, dtype=torch.float64, device=dev),
               torch.empty(k, dtype=torch.int64, device=dev) if snap else None)
    Z, labels, obj2, sn = out
    F.check(F.lib().cabs_kmeans_noalloc(rows, dim, k, prec, _ptr(P), _ptr(w), _ptr(Z0), iters, _ptr(Z),
                                        _ptr(labels), _ptr(obj2), _ptr(sn), _stream(stream)), "cabs_kmeans_noalloc")
    return Z, labels, obj2, sn


def timing_enable(on: bool = True) -> None:
    """cabs_timing_enable."""
    F.check(F.lib().cabs_timing_enable(1 if on else 0), "cabs_timing_enable")


def timing_reset() -> None:
    """cabs_timing_reset."""
    F.lib().cabs_timing_reset()


def timing_read(family: str):
    """cabs_timing_read -> (total milliseconds, launches)."""
    ms = C.c_double(0.0)
    n = C.c_int64(0)
    F.check(F.lib().cabs_timing_read(family.encode(), C.byref(ms), C.byref(n)), "cabs_timing_read")
    return ms.value, n.value


class Server:
    """cabs_server_*: continuous-batching sketch server on one device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 8 << 30, max_slots: int = 8):
        self.h = F.lib().cabs_server_create(device, hbm_budget_bytes, max_slots)
        if not self.h:
            raise F.CabsError(F.EINVAL, "cabs_server_create")
        self._live = {}

    def submit(self, mat: DeviceMatrix, prm: F.CabsParams, out: SketchResult, err_samples: Optional[int] = None,
               err_seed: int = 0, err_out: Optional[torch.Tensor] = None, stream=None) -> int:
        """Queue a sketch into `out`; with err_samples set, also its relative
        Frobenius error into err_out (3 float64 on the device: num, den, ratio).
        The request runs after the work already enqueued on `stream` (default:
        torch's current stream)."""
        t = C.c_uint64(0)
        p3 = None
        if err_samples is not None:
            if err_out is None or err_out.numel() < 3 or err_out.dtype != torch.float64:
                raise ValueError("err_out must be a float64 device tensor of 3 elements")
            p3 = _ptr(err_out)
        prm_copy = F.CabsParams.from_buffer_copy(prm)
        F.check(F.lib().cabs_submit(self.h, C.byref(mat.desc), C.byref(prm_copy), C.byref(out.struct),
                                    int(err_samples or 0), int(err_seed), p3, _stream(stream), C.byref(t)),
                "cabs_submit")
        self._live[t.value] = (mat, prm_copy, out, err_out)
        return t.value

    def poll(self, ticket: int):
        lat = C.c_double(0.0)
        st = F.lib().cabs_poll(self.h, ticket, C.byref(lat))
        if st == F.EBUSY:
            return None
        self._live.pop(ticket, None)
        F.check(st, "cabs_poll")
        return lat.value

    def cancel(self, ticket: int) -> int:
        return F.lib().cabs_cancel(self.h, ticket)

    def set_group(self, group_max: int) -> None:
        """cabs_server_set_group: same-shape requests admitted together share their SVD launches
        (1..4 per group; 1 turns it off)."""
        F.check(F.lib().cabs_server_set_group(self.h, int(group_max)), "cabs_server_set_group")

    def drain(self):
        F.check(F.lib().cabs_server_drain(self.h), "cabs_server_drain")

    def close(self):
        if self.h:
            F.lib().cabs_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
