"""CPU checks of the C ABI: the library loads and exports every declared symbol;
argument validation and workspace planning work without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cabs.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(cabs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("cabs_sketch", "cabs_error", "cabs_workspace_bytes", "cabs_last_error", "cabs_server_create",
                 "cabs_submit", "cabs_poll", "cabs_cancel", "cabs_server_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1607_07395_amd import _ffi as F
    lib = F.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(F.exported_symbols()) == _declared()
    assert lib.cabs_version().startswith(b"libcabs")


def _desc(m=1000, n=800, r=20):
    from paper_1607_07395_amd import _ffi as F
    d = F.CabsMatrix()
    d.kind, d.storage, d.m, d.n = F.SRC_LOWRANK, F.F32, m, n
    d.pf = d.qf = d.s = 0x1000   # never dereferenced by the planner
    d.r = r
    d.noise_std = 1e-3
    return d


def test_workspace_planning_and_validation_on_cpu():
    from paper_1607_07395_amd import _ffi as F
    from paper_1607_07395_amd.api import make_params
    lib = F.lib()
    d = _desc()
    p = make_params(20, 20, 20, 20, compute="f32")
    ws = lib.cabs_workspace_bytes(C.byref(d), C.byref(p))
    assert ws > 0
    # linear in m + n: doubling both roughly doubles the workspace
    d2 = _desc(2000, 1600)
    ws2 = lib.cabs_workspace_bytes(C.byref(d2), C.byref(p))
    assert 1.6 * ws < ws2 < 2.4 * ws
    # invalid: k larger than m, FP64 compute on FP32 tables, unknown kind
    bad = make_params(2000, 20, 20, 20)
    assert lib.cabs_workspace_bytes(C.byref(d), C.byref(bad)) == 0
    assert lib.cabs_workspace_bytes(C.byref(d), C.byref(make_params(20, 20, 20, 20, compute="f64"))) == 0
    d.kind = 7
    assert lib.cabs_workspace_bytes(C.byref(d), C.byref(p)) == 0
    assert b"unknown source kind" in lib.cabs_last_error()
    # follow-up kind: the hard-threshold and leverage selections plan their own workspace;
    # unknown kinds and unknown flag bits are rejected
    d = _desc()
    h = make_params(20, 20, 20, 20, compute="f32", follow_up="hard")
    assert lib.cabs_workspace_bytes(C.byref(d), C.byref(h)) > 0
    lv = make_params(20, 20, 20, 20, compute="f32", follow_up="leverage")
    assert lib.cabs_workspace_bytes(C.byref(d), C.byref(lv)) > 0
    pil = make_params(20, 30, 20, 30, compute="f32", follow_up="pilot")
    assert 0 < lib.cabs_workspace_bytes(C.byref(d), C.byref(pil)) < lib.cabs_workspace_bytes(C.byref(d), C.byref(p))
    pil.k2_cols = 31   # the pilot sketch alone keeps the pilot sizes
    assert lib.cabs_workspace_bytes(C.byref(d), C.byref(pil)) == 0
    assert b"k2 = k1" in lib.cabs_last_error()
    h.follow_up = 4
    assert lib.cabs_workspace_bytes(C.byref(d), C.byref(h)) == 0
    assert b"follow-up" in lib.cabs_last_error()
    h.follow_up = 0
    h.flags = 2
    assert lib.cabs_workspace_bytes(C.byref(d), C.byref(h)) == 0


def test_entry_points_reject_bad_arguments_without_launching():
    from paper_1607_07395_amd import _ffi as F
    from paper_1607_07395_amd.api import make_params
    lib = F.lib()
    d = _desc()
    p = make_params(20, 20, 20, 20)
    res = F.CabsResult()  # all null
    assert lib.cabs_sketch(C.byref(d), C.byref(p), None, 0, C.byref(res), None) == F.EINVAL
    assert lib.cabs_sample(10, 11, 0, 0, C.c_void_p(0x1000), None) == F.EINVAL
    assert lib.cabs_sample(10, 3, 0, 0, None, None) == F.EINVAL
    assert lib.cabs_svd(1, 5000, 3, None, None, None, None, None, 0, None) == F.EINVAL
    assert lib.cabs_svd(1, 1100, 1100, None, None, None, None, None, 0, None) == F.EINVAL
    assert lib.cabs_svd_workspace_bytes(1, 4096, 1024) > 0 and lib.cabs_svd_workspace_bytes(1, 4097, 10) == 0
    assert lib.cabs_svd_ex(1, 50, 50, None, None, None, None, None, 0, -1, None) == F.EINVAL
    assert lib.cabs_svd_ex(1, 50, 50, None, None, None, None, None, 0, 25, None) == F.EINVAL
    assert lib.cabs_kmeans(10, 3, 11, F.F32, None, None, None, 1, None, None, None, None, None, 0, None) == F.EINVAL
    # the allocation-free k-means: invalid sizes, and problems beyond its fixed scratch, are rejected
    # before any device call
    fake = C.c_void_p(0x1000)
    assert lib.cabs_kmeans_noalloc(10, 3, 11, F.F32, fake, fake, fake, 1, fake, None, None, None, None) == F.EINVAL
    assert lib.cabs_kmeans_noalloc(1_000_000, 504, 500, F.BF16, fake, fake, fake, 1, fake, None, None, None,
                                   None) == F.ENOMEM
    assert b"fixed array" in lib.cabs_last_error()
    assert lib.cabs_svd_workspace_bytes(1, 50, 50) > 0
    assert lib.cabs_kmeans_workspace_bytes(10_000, 50, 50, F.F32) > 0
    # workspace too small -> ENOMEM before anything is launched
    res.idx_r = res.idx_c = res.C = res.Rt = res.Umid = 0x1000
    assert lib.cabs_sketch(C.byref(d), C.byref(p), C.c_void_p(0x100000), 1024, C.byref(res), None) == F.ENOMEM
    assert b"workspace too small" in lib.cabs_last_error()
    # unaligned workspace
    assert lib.cabs_sketch(C.byref(d), C.byref(p), C.c_void_p(0x100001), 1 << 40, C.byref(res), None) == F.EINVAL


def test_brcur_planning_and_validation_on_cpu():
    from paper_1607_07395_amd import _ffi as F
    lib = F.lib()
    d = _desc()
    p = F.CabsBrCurParams()
    p.kb_rows, p.kb_cols, p.kt_rows, p.kt_cols, p.compute = 20, 30, 60, 90, F.F32
    gen = lib.cabs_brcur_workspace_bytes(C.byref(d), C.byref(p), 0)
    same = lib.cabs_brcur_workspace_bytes(C.byref(d), C.byref(p), 1)
    assert gen > same > 0
    # the target sizes are ignored when the target is the base sample
    p.kt_rows = 5000
    assert lib.cabs_brcur_workspace_bytes(C.byref(d), C.byref(p), 1) == same
    assert lib.cabs_brcur_workspace_bytes(C.byref(d), C.byref(p), 0) == 0
    p.kt_rows = 60
    for field, value in (("kb_rows", 0), ("kb_cols", 1025), ("kt_cols", 4097), ("kt_cols", 801), ("rank_cap", -1),
                         ("flags", 1), ("compute", F.F64)):
        old = getattr(p, field)
        setattr(p, field, value)
        assert lib.cabs_brcur_workspace_bytes(C.byref(d), C.byref(p), 0) == 0, field
        setattr(p, field, old)
    fake = C.c_void_p(0x1000)
    # one target pointer without the other, missing outputs, a short workspace: rejected before any launch
    assert lib.cabs_brcur(C.byref(d), C.byref(p), fake, fake, fake, None, fake, 1 << 30, fake, fake, fake, None,
                          None) == F.EINVAL
    assert lib.cabs_brcur(C.byref(d), C.byref(p), fake, fake, None, None, C.c_void_p(0x100000), 1 << 30, fake, fake,
                          None, None, None) == F.EINVAL
    assert lib.cabs_brcur(C.byref(d), C.byref(p), fake, fake, fake, fake, C.c_void_p(0x100000), 1024, fake, fake,
                          fake, None, None) == F.ENOMEM
    assert b"workspace too small" in lib.cabs_last_error()


def test_sketch_batch_rejects_bad_arguments_without_launching():
    from paper_1607_07395_amd import _ffi as F
    from paper_1607_07395_amd.api import make_params
    lib = F.lib()
    mats = (F.CabsMatrix * 2)(_desc(), _desc(2000, 900))
    prms = (F.CabsParams * 2)(make_params(20, 20, 20, 20), make_params(20, 20, 20, 24))
    outs = (F.CabsResult * 2)()
    ws = (C.c_void_p * 2)(0x100000, 0x200000)
    wb = (C.c_size_t * 2)(1 << 30, 1 << 30)
    for n in (0, 5):
        assert lib.cabs_sketch_batch(n, mats, prms, ws, wb, outs, None) == F.EINVAL
    assert lib.cabs_sketch_batch(2, mats, prms, ws, wb, outs, None) == F.EINVAL   # different shapes
    assert b"differs in shape" in lib.cabs_last_error()
    prms[1].k2_cols = 20
    prms[0].want_factors = prms[1].want_factors = 1
    assert lib.cabs_sketch_batch(2, mats, prms, ws, wb, outs, None) == F.EINVAL   # the factor form is not batched
    prms[0].want_factors = prms[1].want_factors = 0
    assert lib.cabs_sketch_batch(2, mats, prms, ws, wb, outs, None) == F.EINVAL   # null result buffers


def test_server_rejects_invalid_creation():
    from paper_1607_07395_amd import _ffi as F
    lib = F.lib()
    assert not lib.cabs_server_create(0, 1 << 20, 0)
    assert not lib.cabs_server_create(0, 16, 4)


def test_server_rejects_bad_arguments_with_a_reason():
    """cabs_server_create checks its arguments before any device call and says why through cabs_last_error."""
    from paper_1607_07395_amd import _ffi as F
    from paper_1607_07395_amd import api
    for budget, slots in ((1024, 2), (1 << 20, 0), (1 << 20, 65)):
        with pytest.raises(F.CabsError, match="max_slots must be 1..64"):
            api.Server(0, budget, slots)
