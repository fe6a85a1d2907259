"""Host-code cases run in a child process against the library built with host-side AddressSanitizer
and UndefinedBehaviorSanitizer (``paper_2102_11089_amd.build.build_sanitized``); started by
``test_host_sanitized.py`` with the sanitizer runtime preloaded.  Any sanitizer report ends the
process with a non-zero status.  No GPU is needed: a code that passes validation reaches the first
device call and returns LDPC_EHIP there (or LDPC_OK where a device exists).

Usage: python tests/sanitized_host_cases.py <library>
"""
import ctypes as C
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2102_11089_amd import ldpc  # noqa: E402
from paper_2102_11089_amd import synth as S  # noqa: E402

OK, EINVAL, EHIP = 0, -1, -3


def csr(M, N, rows, layers=None):
    rp = np.zeros(M + 1, dtype=np.int32)
    for m, r in enumerate(rows):
        rp[m + 1] = rp[m] + len(r)
    col = np.array([c for r in rows for c in r], dtype=np.int32)
    out = C.c_void_p()
    lp = None if layers is None else np.asarray(layers, dtype=np.int32)
    rc = lib.ldpc_code_from_csr(M, N, rp.ctypes.data, col.ctypes.data, None if lp is None else lp.ctypes.data,
                                0 if lp is None else len(lp) - 1, C.byref(out))
    if rc == OK:
        lib.ldpc_code_free(out)
    return rc


def qc(shift, Z):
    sh = np.ascontiguousarray(shift, dtype=np.int32)
    out = C.c_void_p()
    rc = lib.ldpc_code_from_qc(sh.shape[0], sh.shape[1], Z, sh.ctypes.data, C.byref(out))
    if rc == OK:
        lib.ldpc_code_free(out)
    return rc


def expect(name, rc, allowed):
    print(f"{name}: {rc}", flush=True)
    if rc not in allowed:
        raise SystemExit(f"{name}: return code {rc}, expected one of {allowed}")


def main():
    global lib
    lib = ldpc.load(sys.argv[1])
    valid = (OK, EHIP)
    # ---- well-formed codes, including extreme shapes ----
    c0 = S.workload_code("c0")
    expect("c0 PEG (3,6) n=96", csr(c0.M, c0.N, [list(c0.col[c0.row_ptr[m]:c0.row_ptr[m + 1]]) for m in range(c0.M)]),
           valid)
    expect("row of degree 32", csr(2, 33, [list(range(32)), [0, 32]]), valid)
    expect("rows of degree 64", csr(2, 64, [list(range(64)), list(range(64))]), (-5,))
    rows = [[0, 1 + m] for m in range(63)]
    expect("VN of degree 63", csr(63, 64, rows), valid)
    rows = [[0, 1 + m] for m in range(64)]
    expect("VN of degree 64", csr(64, 65, rows), valid)
    expect("layer partition", csr(4, 6, [[0, 1], [2, 3], [0, 4], [1, 5]], layers=[0, 2, 4]), valid)
    base = S.bg1_shaped_base(11089)
    shift = np.where(base > 0, np.random.default_rng(5).integers(0, 52, size=base.shape), -1)
    expect("BG1-shaped Z=52", qc(shift, 52), valid)
    expect("68 blocks in a base row", qc(np.zeros(base.shape, dtype=np.int32), 52), (-5,))
    expect("all shifts 0 (4-cycles everywhere)", qc(np.zeros((4, 8), dtype=np.int32), 16), valid)
    expect("Z = 1", qc(np.array([[0, 0, -1], [-1, 0, 0]]), 1), valid)
    big = np.array([[0, 5, 9, -1], [-1, 2, 0, 7]], dtype=np.int32)
    expect("Z = 2^20 (n = 4194304)", qc(big, 1 << 20), valid)
    # ---- malformed: rejected before any device call ----
    expect("unsorted row", csr(2, 4, [[1, 0], [2, 3]]), (EINVAL,))
    expect("duplicate column", csr(2, 4, [[1, 1, 2], [0, 3]]), (EINVAL,))
    expect("column out of range", csr(2, 4, [[0, 4], [1, 2, 3]]), (EINVAL,))
    expect("negative column", csr(2, 4, [[-1, 0], [1, 2, 3]]), (EINVAL,))
    expect("row of degree 1", csr(2, 3, [[0], [0, 1, 2]]), (EINVAL,))
    expect("empty column", csr(2, 5, [[0, 1], [2, 3]]), (EINVAL,))
    expect("empty layer", csr(4, 6, [[0, 1], [2, 3], [0, 4], [1, 5]], layers=[0, 2, 2, 4]), (EINVAL,))
    expect("layer sharing a VN", csr(4, 6, [[0, 1], [1, 3], [0, 4], [2, 5]], layers=[0, 2, 4]), (EINVAL,))
    expect("layers not ending at M", csr(4, 6, [[0, 1], [2, 3], [0, 4], [1, 5]], layers=[0, 2, 3]), (EINVAL,))
    rp = np.array([1, 3, 5], dtype=np.int32)
    col = np.array([0, 1, 2, 3, 0, 1], dtype=np.int32)
    out = C.c_void_p()
    expect("row_ptr[0] != 0", lib.ldpc_code_from_csr(2, 4, rp.ctypes.data, col.ctypes.data, None, 0, C.byref(out)),
           (EINVAL,))
    rp = np.array([0, 3, 1 << 29], dtype=np.int32)
    expect("more than 2^28 edges", lib.ldpc_code_from_csr(2, 4, rp.ctypes.data, col.ctypes.data, None, 0, C.byref(out)),
           (EINVAL,))
    expect("M = 0", lib.ldpc_code_from_csr(0, 4, rp.ctypes.data, col.ctypes.data, None, 0, C.byref(out)), (EINVAL,))
    expect("null arrays", lib.ldpc_code_from_csr(2, 4, None, None, None, 0, C.byref(out)), (EINVAL,))
    expect("shift below -1", qc(np.array([[0, -2], [0, 1]]), 4), (EINVAL,))
    expect("shift >= Z", qc(np.array([[0, 4], [0, 1]]), 4), (EINVAL,))
    expect("base row with one block", qc(np.array([[0, -1, -1], [0, 1, 2]]), 4), (EINVAL,))
    expect("empty base column", qc(np.array([[0, 1, -1], [0, 1, -1]]), 4), (EINVAL,))
    expect("Z = 0", qc(np.array([[0, 1], [1, 0]]), 0), (EINVAL,))
    expect("n = 2^24", qc(np.array([[0, 1], [1, 0]]), 1 << 23), (-5,))
    expect("n beyond 2^26", qc(np.array([[0, 1], [1, 0]]), 1 << 26), (EINVAL,))
    # ---- entry points with bad arguments ----
    s = ldpc.schedule(ldpc.CIRBP)
    o = ldpc.ldpc_outputs()
    info = ldpc.ldpc_plan_info()
    expect("decode null code", lib.ldpc_decode(None, C.byref(s), None, 1, 10, None, 0, C.byref(o), None), (EINVAL,))
    expect("decode_noalloc null code", lib.ldpc_decode_noalloc(None, C.byref(s), None, 1, 10, None, 0, C.byref(o), None),
           (EINVAL,))
    expect("describe_plan null code", lib.ldpc_describe_plan(None, C.byref(s), 8, C.byref(info)), (EINVAL,))
    expect("describe_batch_plan no codes", lib.ldpc_describe_batch_plan(None, 0, C.byref(s), 8, C.byref(info)),
           (EINVAL,))
    expect("unrolled_forward null code", lib.ldpc_unrolled_forward(None, None, None, None, 1, 10, 32, None, None, None,
                                                                    None), (EINVAL,))
    T = ldpc.ldpc_tuning
    expect("batch tuning: bad storage", lib.ldpc_set_batch_tuning(C.byref(T(0, 0, 9, 0))), (EINVAL,))
    expect("batch tuning: clear", lib.ldpc_set_batch_tuning(None), (OK,))
    for rc in (0, -1, -2, -3, -4, -5, -99):
        assert lib.ldpc_strerror(rc)
    print("sanitized host cases done", flush=True)


if __name__ == "__main__":
    main()
