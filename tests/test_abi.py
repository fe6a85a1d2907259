"""Host-side checks of the C ABI that need no GPU: the library loads, exports every function the
header declares, and rejects malformed input before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2102_11089_amd import ldpc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ldpcci.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ldpc_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ldpc.load()
    names = declared_functions()
    assert names, "no declarations parsed"
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(ldpc.EXPORTS)


def test_header_constants_match_binding():
    src = open(HEADER).read()
    consts = dict(re.findall(r"#define (LDPC_[A-Z_0-9]+) \(?(-?\d+)\)?", src))
    assert int(consts["LDPC_FLOODING"]) == ldpc.FLOODING
    assert int(consts["LDPC_LAYERED"]) == ldpc.LAYERED
    assert int(consts["LDPC_RBP"]) == ldpc.RBP
    assert int(consts["LDPC_CIRBP"]) == ldpc.CIRBP
    assert int(consts["LDPC_ME_CIRBP"]) == ldpc.ME_CIRBP
    assert int(consts["LDPC_REPLAY"]) == ldpc.REPLAY
    assert int(consts["LDPC_LMDRBP"]) == ldpc.LMDRBP
    assert int(consts["LDPC_SLMDRBP"]) == ldpc.SLMDRBP
    assert int(consts["LDPC_LMD_CIRBP"]) == ldpc.LMD_CIRBP
    assert int(consts["LDPC_ME_LMD_CIRBP"]) == ldpc.ME_LMD_CIRBP
    for name in ("AUTO", "LDS", "GLOBAL", "GLOBAL_ALL", "GLOBAL_LT", "GLOBAL_FRAME", "GLOBAL_REC", "GLOBAL_STATE"):
        assert int(consts["LDPC_STORE_" + name]) == getattr(ldpc, "STORE_" + name)
    for name in ("AUTO", "GLOBAL", "LDS", "QC"):
        assert int(consts["LDPC_TOPO_" + name]) == getattr(ldpc, "TOPO_" + name)
    assert int(consts["LDPC_FILL_LOWEST"]) == ldpc.FILL_LOWEST and int(consts["LDPC_FILL_HASH"]) == ldpc.FILL_HASH
    assert int(consts["LDPC_SPA_F32"]) == ldpc.SPA_F32
    assert int(consts["LDPC_MS_FIX"]) == ldpc.MS_FIX
    for k, v in ldpc.ERRORS.items():
        assert int(consts[v]) == k


def test_struct_sizes():
    assert C.sizeof(ldpc.ldpc_schedule) == 48
    assert C.sizeof(ldpc.ldpc_outputs) == 11 * 8
    assert C.sizeof(ldpc.ldpc_code_stats) == 64


def test_strerror():
    for rc in ldpc.ERRORS:
        assert isinstance(ldpc.ldpc_strerror(rc), str) and ldpc.ldpc_strerror(rc)


@pytest.mark.parametrize("case", ["unsorted", "dup", "range", "short_row", "empty_col", "layer_overlap"])
def test_code_validation_rejects_malformed(case):
    rp = np.array([0, 3, 6], dtype=np.int32)
    col = np.array([0, 1, 2, 1, 2, 3], dtype=np.int32)
    lp = None
    M, N = 2, 4
    if case == "unsorted":
        col = np.array([1, 0, 2, 1, 2, 3], dtype=np.int32)
    elif case == "dup":
        col = np.array([0, 1, 1, 1, 2, 3], dtype=np.int32)
    elif case == "range":
        col = np.array([0, 1, 2, 1, 2, 4], dtype=np.int32)
    elif case == "short_row":
        rp = np.array([0, 1, 6], dtype=np.int32)
    elif case == "empty_col":
        N = 5
    elif case == "layer_overlap":
        lp = np.array([0, 2], dtype=np.int32)
    with pytest.raises(RuntimeError, match="LDPC_EINVAL"):
        ldpc.ldpc_code_from_csr(M, N, rp, col, lp)


def test_code_rank_rejects_null_arguments():
    lib = ldpc.load()
    r = C.c_int32(0)
    assert lib.ldpc_code_rank(None, C.byref(r)) == -1


def test_decode_rejects_null_arguments():
    lib = ldpc.load()
    s = ldpc.schedule(ldpc.CIRBP)
    out = ldpc.ldpc_outputs()
    assert lib.ldpc_decode(None, C.byref(s), None, 1, 10, None, 0, C.byref(out), None) == -1
    assert lib.ldpc_decode_noalloc(None, C.byref(s), None, 1, 10, None, 0, C.byref(out), None) == -1
    assert lib.ldpc_decode_noalloc(None, None, None, -1, 10, None, 0, None, None) == -1


def test_noalloc_scratch_limit_is_declared():
    m = re.search(r"#define LDPC_NOALLOC_SCRATCH_BYTES \((\d+)ll << (\d+)\)", open(HEADER).read())
    assert m and int(m.group(1)) << int(m.group(2)) == 128 << 20


def test_unrolled_entry_points_reject_bad_arguments():
    lib = ldpc.load()
    assert lib.ldpc_unrolled_ckpt_floats(None, 300, 32) == -1
    assert lib.ldpc_unrolled_forward(None, None, None, None, 1, 10, 32, None, None, None, None) == -1
    assert lib.ldpc_unrolled_backward(None, None, None, 1, 10, 32, None, None, None, None, None) == -1
    assert ldpc.UNROLL_MAX_CKPT_EVERY == 128
    hdr = open(HEADER).read()
    assert "#define LDPC_UNROLL_MAX_CKPT_EVERY 128" in hdr


def test_describe_plan_rejects_bad_arguments():
    lib = ldpc.load()
    s = ldpc.schedule(ldpc.CIRBP)
    info = ldpc.ldpc_plan_info()
    assert C.sizeof(ldpc.ldpc_plan_info) == 48
    assert lib.ldpc_describe_plan(None, C.byref(s), 8, C.byref(info)) == -1


def test_batch_tuning_validation_and_round_trip():
    """The batched launch's tuning is validated and kept on the host (no device call)."""
    lib = ldpc.load()
    T = ldpc.ldpc_tuning
    assert lib.ldpc_set_batch_tuning(C.byref(T(64, 0, 0, 0))) == -1    # block: one frame per workgroup
    assert lib.ldpc_set_batch_tuning(C.byref(T(0, 0, 0, 1))) == -1     # topology is not a batch knob
    assert lib.ldpc_set_batch_tuning(C.byref(T(0, 33, 0, 0))) == -1    # at most 32 frames per CU
    assert lib.ldpc_set_batch_tuning(C.byref(T(0, 0, 9, 0))) == -1     # unknown storage
    assert lib.ldpc_set_batch_tuning(C.byref(T(0, 0, ldpc.STORE_GLOBAL_STATE, 0))) == -5  # no batched form
    out = T()
    assert lib.ldpc_get_batch_tuning(None) == -1
    try:
        assert lib.ldpc_set_batch_tuning(C.byref(T(0, 12, ldpc.STORE_GLOBAL_REC, 0))) == 0
        assert lib.ldpc_get_batch_tuning(C.byref(out)) == 1
        assert (out.block, out.frames_per_cu, out.storage, out.topology) == (0, 12, ldpc.STORE_GLOBAL_REC, 0)
    finally:
        assert lib.ldpc_set_batch_tuning(None) == 0
    assert lib.ldpc_get_batch_tuning(C.byref(out)) == 0
    s = ldpc.schedule(ldpc.CIRBP)
    assert lib.ldpc_autotune_batch(None, 1, C.byref(s), None, 0, None, 0, 0, 2, None, None, None) == -1


def test_lds_probe_rejects_bad_arguments():
    lib = ldpc.load()
    b, t = C.c_double(0.0), C.c_float(0.0)
    sink = (C.c_uint32 * 4)()
    for width, blocks, iters in ((3, 4, 16), (32, 4, 16), (16, 0, 16), (16, 4, 0), (16, 4, (1 << 24) + 1)):
        assert lib.ldpc_probe_lds(width, blocks, iters, sink, None, C.byref(b), C.byref(t)) == -1
    assert lib.ldpc_probe_lds(16, 4, 16, None, None, C.byref(b), C.byref(t)) == -1
    assert lib.ldpc_probe_lds(16, 4, 16, sink, None, None, C.byref(t)) == -1
