"""Python binding of the C ABI in ``include/ldpcci.h`` (ctypes; argument marshalling only).

The functions ``ldpc_code_from_csr``, ``ldpc_code_info``, ``ldpc_code_free``, ``ldpc_decode`` and
``ldpc_strerror`` mirror the C entry points one to one.  PyTorch supplies device memory and the
stream; every decoding step runs in the HIP kernels of ``libldpcci.so``.  There is no fallback:
if the library is missing or no GPU is present, loading raises.

``decode`` is a convenience wrapper that allocates the output tensors and returns them.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libldpcci.so")

# schedules / arithmetic / fill (values of include/ldpcci.h)
FLOODING, LAYERED, RBP, CIRBP, ME_CIRBP, REPLAY, LMDRBP, SLMDRBP, LMD_CIRBP, ME_LMD_CIRBP = range(10)
SPA_F32, MS_FIX = 0, 1
FILL_LOWEST, FILL_HASH = 0, 1
ERRORS = {0: "LDPC_OK", -1: "LDPC_EINVAL", -2: "LDPC_ENOMEM", -3: "LDPC_EHIP", -4: "LDPC_ECAPACITY",
          -5: "LDPC_EUNSUPPORTED"}

EXPORTS = ("ldpc_code_from_csr", "ldpc_code_from_qc", "ldpc_code_info", "ldpc_code_rank", "ldpc_code_free",
           "ldpc_decode", "ldpc_decode_noalloc",
           "ldpc_decode_batch", "ldpc_describe_plan", "ldpc_describe_batch_plan", "ldpc_set_tuning", "ldpc_get_tuning", "ldpc_autotune",
           "ldpc_set_batch_tuning", "ldpc_get_batch_tuning", "ldpc_autotune_batch", "ldpc_tuning_save",
           "ldpc_tuning_load", "ldpc_awgn_frames", "ldpc_sweep_create", "ldpc_sweep_run", "ldpc_sweep_free",
           "ldpc_unrolled_ckpt_floats", "ldpc_unrolled_forward", "ldpc_unrolled_backward",
           "ldpc_request_abort", "ldpc_probe_lds", "ldpc_strerror", "ldpc_last_hip_error")
UNROLL_MAX_CKPT_EVERY = 128
STORE_AUTO, STORE_LDS, STORE_GLOBAL, STORE_GLOBAL_ALL, STORE_GLOBAL_LT, STORE_GLOBAL_FRAME, STORE_GLOBAL_REC, \
    STORE_GLOBAL_STATE = 0, 1, 2, 3, 4, 5, 6, 7
TOPO_AUTO, TOPO_GLOBAL, TOPO_LDS, TOPO_QC = 0, 1, 2, 3

# layout of ldpc_frame_desc (40 bytes)
FRAME_DESC = np.dtype([("code", "<i4"), ("kind", "<i4"), ("gamma", "<f4"), ("reserved", "<i4"),
                       ("max_updates", "<i8"), ("llr_off", "<i8"), ("out_off", "<i8")])


class ldpc_schedule(C.Structure):
    _fields_ = [("kind", C.c_int32), ("arith", C.c_int32), ("q_bits", C.c_int32), ("frac_bits", C.c_int32),
                ("gamma", C.c_float), ("n_p", C.c_int32), ("n_g", C.c_int32), ("fill", C.c_int32),
                ("seed", C.c_uint64), ("check_every", C.c_int64)]


class ldpc_outputs(C.Structure):
    _fields_ = [(name, C.c_void_p) for name in
                ("bits", "llr_out", "updates_used", "steps_used", "fallbacks", "trace", "dump_c2v",
                 "dump_pre", "dump_L", "dump_Lt", "dump_D")]


class ldpc_tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("frames_per_cu", C.c_int32), ("storage", C.c_int32),
                ("topology", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class ldpc_plan_info(C.Structure):
    _fields_ = [(k, C.c_int32) for k in ("kernel", "storage", "topology", "block", "grid", "frames_per_workgroup",
                                          "workgroups_per_cu", "persistent", "lds_bytes", "reserved")] + \
               [("scratch_bytes", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_ if k != "reserved"}


class ldpc_code_stats(C.Structure):
    _fields_ = [("M", C.c_int32), ("N", C.c_int32), ("E", C.c_int32), ("max_dv", C.c_int32),
                ("max_dc", C.c_int32), ("n_layers", C.c_int32), ("max_touch", C.c_int32),
                ("lds_bytes_f32", C.c_int64), ("lds_bytes_fix", C.c_int64), ("mean_dv", C.c_float),
                ("mean_dc", C.c_float), ("gf2_rank", C.c_int32), ("reserved", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libldpcci.so (built by ``paper_2102_11089_amd.build``); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: run `python -m paper_2102_11089_amd.build`")
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.ldpc_code_from_csr.argtypes = [C.c_int32, C.c_int32, P, P, P, C.c_int32, C.POINTER(C.c_void_p)]
    lib.ldpc_code_from_csr.restype = C.c_int
    lib.ldpc_code_from_qc.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, C.POINTER(C.c_void_p)]
    lib.ldpc_code_from_qc.restype = C.c_int
    lib.ldpc_code_info.argtypes = [P, C.POINTER(ldpc_code_stats)]
    lib.ldpc_code_info.restype = C.c_int
    lib.ldpc_code_rank.argtypes = [P, C.POINTER(C.c_int32)]
    lib.ldpc_code_rank.restype = C.c_int
    lib.ldpc_code_free.argtypes = [P]
    lib.ldpc_code_free.restype = None
    lib.ldpc_decode.argtypes = [P, C.POINTER(ldpc_schedule), P, C.c_int32, C.c_int64, P, C.c_int64,
                                C.POINTER(ldpc_outputs), P]
    lib.ldpc_decode.restype = C.c_int
    lib.ldpc_decode_noalloc.argtypes = lib.ldpc_decode.argtypes
    lib.ldpc_decode_noalloc.restype = C.c_int
    lib.ldpc_decode_batch.argtypes = [P, C.c_int32, C.POINTER(ldpc_schedule), P, C.c_int32, P, C.c_int64, P, P,
                                      C.c_int64, P, P, P, P]
    lib.ldpc_decode_batch.restype = C.c_int
    lib.ldpc_describe_plan.argtypes = [P, C.POINTER(ldpc_schedule), C.c_int32, C.POINTER(ldpc_plan_info)]
    lib.ldpc_describe_plan.restype = C.c_int
    lib.ldpc_describe_batch_plan.argtypes = [P, C.c_int32, C.POINTER(ldpc_schedule), C.c_int32,
                                             C.POINTER(ldpc_plan_info)]
    lib.ldpc_describe_batch_plan.restype = C.c_int
    lib.ldpc_set_tuning.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(ldpc_tuning)]
    lib.ldpc_set_tuning.restype = C.c_int
    lib.ldpc_get_tuning.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(ldpc_tuning)]
    lib.ldpc_get_tuning.restype = C.c_int
    lib.ldpc_autotune.argtypes = [P, C.POINTER(ldpc_schedule), P, C.c_int32, C.c_int64, C.c_int32,
                                  C.POINTER(ldpc_tuning), C.POINTER(C.c_float), P]
    lib.ldpc_autotune.restype = C.c_int
    lib.ldpc_set_batch_tuning.argtypes = [C.POINTER(ldpc_tuning)]
    lib.ldpc_set_batch_tuning.restype = C.c_int
    lib.ldpc_get_batch_tuning.argtypes = [C.POINTER(ldpc_tuning)]
    lib.ldpc_get_batch_tuning.restype = C.c_int
    lib.ldpc_autotune_batch.argtypes = [P, C.c_int32, C.POINTER(ldpc_schedule), P, C.c_int32, P, C.c_int64, C.c_int64,
                                        C.c_int32, C.POINTER(ldpc_tuning), C.POINTER(C.c_float), P]
    lib.ldpc_autotune_batch.restype = C.c_int
    lib.ldpc_tuning_save.argtypes = [C.c_char_p]
    lib.ldpc_tuning_save.restype = C.c_int
    lib.ldpc_tuning_load.argtypes = [C.c_char_p]
    lib.ldpc_tuning_load.restype = C.c_int
    lib.ldpc_awgn_frames.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_float, C.c_uint64, C.c_int32, P, P]
    lib.ldpc_awgn_frames.restype = C.c_int
    lib.ldpc_probe_lds.argtypes = [C.c_int32, C.c_int32, C.c_int64, P, P, C.POINTER(C.c_double),
                                   C.POINTER(C.c_float)]
    lib.ldpc_probe_lds.restype = C.c_int
    lib.ldpc_request_abort.argtypes = [C.c_int32]
    lib.ldpc_request_abort.restype = C.c_int
    lib.ldpc_sweep_create.argtypes = [P, C.POINTER(ldpc_schedule), C.c_int64, P, C.c_int32, P, C.c_int32, C.c_float,
                                      C.c_int32, C.POINTER(C.c_void_p)]
    lib.ldpc_sweep_create.restype = C.c_int
    lib.ldpc_sweep_run.argtypes = [P, C.c_uint64, P, P]
    lib.ldpc_sweep_run.restype = C.c_int
    lib.ldpc_sweep_free.argtypes = [P]
    lib.ldpc_sweep_free.restype = None
    lib.ldpc_unrolled_ckpt_floats.argtypes = [P, C.c_int32, C.c_int32]
    lib.ldpc_unrolled_ckpt_floats.restype = C.c_int64
    lib.ldpc_unrolled_forward.argtypes = [P, P, P, P, C.c_int32, C.c_int32, C.c_int32, P, P, P, P]
    lib.ldpc_unrolled_forward.restype = C.c_int
    lib.ldpc_unrolled_backward.argtypes = [P, P, P, C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P]
    lib.ldpc_unrolled_backward.restype = C.c_int
    lib.ldpc_strerror.argtypes = [C.c_int]
    lib.ldpc_strerror.restype = C.c_char_p
    lib.ldpc_last_hip_error.argtypes = []
    lib.ldpc_last_hip_error.restype = C.c_int
    _lib = lib
    return lib


def ldpc_strerror(rc: int) -> str:
    return load().ldpc_strerror(rc).decode()


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what}: {ERRORS.get(rc, rc)} ({ldpc_strerror(rc)}), hip={load().ldpc_last_hip_error()}")


def _need(cond: bool, msg: str):
    if not cond:
        raise ValueError(msg)


def _cuda(t, name: str, dtype, cols: Optional[int] = None, rows: Optional[int] = None, device=None):
    """``t`` as a contiguous CUDA tensor of ``dtype``; with ``cols`` (and ``rows``) given it must be
    2-D of that width (and height).  The kernels index these buffers by the sizes passed beside
    them, so a tensor that is smaller, strided or of another type is refused here (ValueError)."""
    import torch
    _need(isinstance(t, torch.Tensor) and t.is_cuda, f"{name}: a CUDA tensor is required")
    _need(t.dtype == dtype, f"{name}: dtype {dtype} is required, got {t.dtype}")
    if device is not None:
        _need(t.device == device, f"{name}: must be on {device}, got {t.device}")
    if cols is not None:
        _need(t.dim() == 2 and t.shape[1] == cols and (rows is None or t.shape[0] == rows),
              f"{name}: shape ({'B' if rows is None else rows}, {cols}) is required, got {tuple(t.shape)}")
    return t.contiguous()


def ldpc_code_from_csr(M: int, N: int, row_ptr: np.ndarray, col_idx: np.ndarray,
                       layer_ptr: Optional[np.ndarray] = None) -> int:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    lp = None if layer_ptr is None else np.ascontiguousarray(layer_ptr, dtype=np.int32)
    h = C.c_void_p()
    rc = load().ldpc_code_from_csr(M, N, rp.ctypes.data, ci.ctypes.data, None if lp is None else lp.ctypes.data,
                                   0 if lp is None else len(lp) - 1, C.byref(h))
    _check(rc, "ldpc_code_from_csr")
    return h.value


def ldpc_code_from_qc(mb: int, nb: int, Z: int, shift: np.ndarray) -> int:
    sh = np.ascontiguousarray(shift, dtype=np.int32)
    assert sh.shape == (mb, nb)
    h = C.c_void_p()
    _check(load().ldpc_code_from_qc(mb, nb, Z, sh.ctypes.data, C.byref(h)), "ldpc_code_from_qc")
    return h.value


def ldpc_code_info(handle: int) -> ldpc_code_stats:
    st = ldpc_code_stats()
    _check(load().ldpc_code_info(handle, C.byref(st)), "ldpc_code_info")
    return st


def ldpc_code_rank(handle: int) -> int:
    r = C.c_int32(-1)
    _check(load().ldpc_code_rank(handle, C.byref(r)), "ldpc_code_rank")
    return int(r.value)


def ldpc_code_free(handle: int) -> None:
    load().ldpc_code_free(handle)


def ldpc_decode(handle: int, schedule: ldpc_schedule, llr_ptr: int, B: int, max_updates: int,
                replay_ptr: Optional[int], replay_len: int, outputs: ldpc_outputs, stream: int) -> None:
    rc = load().ldpc_decode(handle, C.byref(schedule), llr_ptr, B, max_updates, replay_ptr, replay_len,
                            C.byref(outputs), stream)
    _check(rc, "ldpc_decode")


def ldpc_decode_noalloc(handle: int, schedule: ldpc_schedule, llr_ptr: int, B: int, max_updates: int,
                        replay_ptr: Optional[int], replay_len: int, outputs: ldpc_outputs, stream: int) -> None:
    rc = load().ldpc_decode_noalloc(handle, C.byref(schedule), llr_ptr, B, max_updates, replay_ptr, replay_len,
                                    C.byref(outputs), stream)
    _check(rc, "ldpc_decode_noalloc")


def ldpc_decode_batch(handles, schedule: ldpc_schedule, frames_ptr: int, F: int, llr_ptr: int, llr_len: int,
                      bits_ptr: int, llr_out_ptr: Optional[int], out_len: int, upd_ptr: int, steps_ptr: Optional[int],
                      fall_ptr: Optional[int], stream: int) -> None:
    arr = (C.c_void_p * len(handles))(*handles)
    rc = load().ldpc_decode_batch(arr, len(handles), C.byref(schedule), frames_ptr, F, llr_ptr, llr_len, bits_ptr,
                                  llr_out_ptr, out_len, upd_ptr, steps_ptr, fall_ptr, stream)
    _check(rc, "ldpc_decode_batch")


def ldpc_describe_plan(handle, s: ldpc_schedule, B: int) -> ldpc_plan_info:
    info = ldpc_plan_info()
    _check(load().ldpc_describe_plan(handle, C.byref(s), B, C.byref(info)), "ldpc_describe_plan")
    return info


def ldpc_describe_batch_plan(handles, s: ldpc_schedule, F: int) -> ldpc_plan_info:
    info = ldpc_plan_info()
    arr = (C.c_void_p * len(handles))(*handles)
    _check(load().ldpc_describe_batch_plan(arr, len(handles), C.byref(s), F, C.byref(info)),
           "ldpc_describe_batch_plan")
    return info


def ldpc_set_tuning(handle, kind: int, arith: int, t: Optional[ldpc_tuning]) -> None:
    _check(load().ldpc_set_tuning(handle, kind, arith, None if t is None else C.byref(t)), "ldpc_set_tuning")


def ldpc_get_tuning(handle, kind: int, arith: int) -> Optional[ldpc_tuning]:
    t = ldpc_tuning()
    rc = load().ldpc_get_tuning(handle, kind, arith, C.byref(t))
    if rc < 0:
        _check(rc, "ldpc_get_tuning")
    return t if rc == 1 else None


def ldpc_autotune(handle, s: ldpc_schedule, llr_ptr: int, B: int, max_updates: int, reps: int, stream: int):
    t = ldpc_tuning()
    ms = C.c_float(0.0)
    _check(load().ldpc_autotune(handle, C.byref(s), llr_ptr, B, max_updates, reps, C.byref(t), C.byref(ms), stream),
           "ldpc_autotune")
    return t, float(ms.value)


def ldpc_set_batch_tuning(t: Optional[ldpc_tuning]) -> None:
    _check(load().ldpc_set_batch_tuning(None if t is None else C.byref(t)), "ldpc_set_batch_tuning")


def ldpc_get_batch_tuning() -> Optional[ldpc_tuning]:
    t = ldpc_tuning()
    rc = load().ldpc_get_batch_tuning(C.byref(t))
    if rc < 0:
        _check(rc, "ldpc_get_batch_tuning")
    return t if rc == 1 else None


def ldpc_autotune_batch(handles, s: ldpc_schedule, frames_ptr: int, F: int, llr_ptr: int, llr_len: int,
                        out_len: int, reps: int, stream: int):
    arr = (C.c_void_p * len(handles))(*handles)
    t = ldpc_tuning()
    ms = C.c_float(0.0)
    _check(load().ldpc_autotune_batch(arr, len(handles), C.byref(s), frames_ptr, F, llr_ptr, llr_len, out_len, reps,
                                      C.byref(t), C.byref(ms), stream), "ldpc_autotune_batch")
    return t, float(ms.value)


def ldpc_tuning_save(path: str) -> None:
    _check(load().ldpc_tuning_save(path.encode()), "ldpc_tuning_save")


def ldpc_tuning_load(path: str) -> int:
    n = load().ldpc_tuning_load(path.encode())
    if n < 0:
        _check(n, "ldpc_tuning_load")
    return int(n)


def ldpc_awgn_frames(cw_ptr: int, P: int, N: int, B: int, sigma2: float, seed: int, point: int, llr_ptr: int,
                     stream: int) -> None:
    _check(load().ldpc_awgn_frames(cw_ptr, P, N, B, sigma2, seed & (2**64 - 1), point, llr_ptr, stream),
           "ldpc_awgn_frames")


def ldpc_request_abort(on: bool) -> None:
    """Set (True) or clear (False) the process-wide abort flag: decodes start no further frame
    while it is set, and report updates_used = -1 for the frames they did not start."""
    _check(load().ldpc_request_abort(1 if on else 0), "ldpc_request_abort")


def ldpc_probe_lds(width: int, blocks: int, iters: int, sink_ptr: int, stream: int):
    b, t = C.c_double(0.0), C.c_float(0.0)
    _check(load().ldpc_probe_lds(width, blocks, iters, sink_ptr, stream, C.byref(b), C.byref(t)), "ldpc_probe_lds")
    return b.value, t.value


def ldpc_sweep_create(handle, s: ldpc_schedule, max_updates: int, cw_ptr: int, P: int, ebn0_db, rate: float,
                      B: int) -> int:
    arr = (C.c_float * len(ebn0_db))(*[float(x) for x in ebn0_db])
    out = C.c_void_p()
    _check(load().ldpc_sweep_create(handle, C.byref(s), max_updates, cw_ptr, P, arr, len(ebn0_db), rate, B,
                                    C.byref(out)), "ldpc_sweep_create")
    return out.value


def ldpc_sweep_run(sweep: int, seed: int, counters_ptr: int, stream: int) -> None:
    _check(load().ldpc_sweep_run(sweep, seed & (2**64 - 1), counters_ptr, stream), "ldpc_sweep_run")


def ldpc_sweep_free(sweep: int) -> None:
    load().ldpc_sweep_free(sweep)


def ldpc_unrolled_ckpt_floats(handle, T: int, ckpt_every: int) -> int:
    n = load().ldpc_unrolled_ckpt_floats(handle, T, ckpt_every)
    _check(int(n) if n < 0 else 0, "ldpc_unrolled_ckpt_floats")
    return int(n)


def ldpc_unrolled_forward(handle, llr_ptr, w_ptr, trace_ptr, B, T, ckpt_every, ckpt_ptr, soft_ptr, c2v_ptr,
                          stream) -> None:
    rc = load().ldpc_unrolled_forward(handle, llr_ptr, w_ptr, trace_ptr, B, T, ckpt_every, ckpt_ptr, soft_ptr,
                                      c2v_ptr, stream)
    _check(rc, "ldpc_unrolled_forward")


def ldpc_unrolled_backward(handle, w_ptr, trace_ptr, B, T, ckpt_every, ckpt_ptr, grad_soft_ptr, grad_llr_ptr,
                           grad_w_ptr, stream) -> None:
    rc = load().ldpc_unrolled_backward(handle, w_ptr, trace_ptr, B, T, ckpt_every, ckpt_ptr, grad_soft_ptr,
                                       grad_llr_ptr, grad_w_ptr, stream)
    _check(rc, "ldpc_unrolled_backward")


# ----------------------------------------------------------------------------------------------
# convenience layer over torch tensors
# ----------------------------------------------------------------------------------------------
class Code:
    """Owns a library code handle built from a ``synth.Code`` (or any object with M, N, row_ptr,
    col and optional layer_ptr).  Quasi-cyclic codes (``qc_shift`` set) go through
    ``ldpc_code_from_qc`` unless ``csr=True``."""

    def __init__(self, code, csr: bool = False):
        self.M, self.N, self.E = int(code.M), int(code.N), int(code.row_ptr[-1])
        sh = getattr(code, "qc_shift", None)
        if sh is not None and not csr:
            mb, nb = sh.shape
            self.handle = ldpc_code_from_qc(mb, nb, int(code.qc_Z), sh)
        else:
            self.handle = ldpc_code_from_csr(self.M, self.N, code.row_ptr, code.col,
                                             getattr(code, "layer_ptr", None))
        self.stats = ldpc_code_info(self.handle)

    def gf2_rank(self) -> int:
        """Rank of H over GF(2) (computed once by the library and kept in the handle)."""
        return ldpc_code_rank(self.handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            ldpc_code_free(h)
            self.handle = None


@dataclass
class Decoded:
    bits: "object"
    llr_out: "object"
    updates_used: "object"
    steps_used: "object"
    fallbacks: "object"
    trace: Optional[object] = None
    c2v: Optional[object] = None
    pre: Optional[object] = None
    L: Optional[object] = None
    Lt: Optional[object] = None
    D: Optional[object] = None


def schedule(kind: int, arith: int = SPA_F32, gamma: float = 0.1, q_bits: int = 6, frac_bits: int = 1,
             n_p: int = 1, n_g: int = 16, fill: int = FILL_LOWEST, seed: int = 0, check_every: int = 1):
    return ldpc_schedule(kind, arith, q_bits, frac_bits, gamma, n_p, n_g, fill, seed & (2**64 - 1), check_every)


def decode(code: Code, llr, kind: int, arith: int = SPA_F32, max_updates: int = 0, gamma: float = 0.1,
           q_bits: int = 6, frac_bits: int = 1, n_p: int = 1, n_g: int = 16, fill: int = FILL_LOWEST,
           seed: int = 0, check_every: int = 1, replay=None, trace: bool = False, dump: bool = False,
           stream=None, noalloc: bool = False) -> Decoded:
    """Decode a (B, N) float32 CUDA tensor of channel LLRs; returns device tensors.  noalloc: call
    ldpc_decode_noalloc (scratch from the library's fixed device array) instead of ldpc_decode."""
    import torch
    llr = _cuda(llr, "llr", torch.float32, cols=code.N)
    B = llr.shape[0]
    dev = llr.device
    bits = torch.empty((B, code.N), dtype=torch.uint8, device=dev)
    llr_out = torch.empty((B, code.N), dtype=torch.float32, device=dev)
    upd = torch.empty(B, dtype=torch.int64, device=dev)
    steps = torch.empty(B, dtype=torch.int64, device=dev)
    fall = torch.empty(B, dtype=torch.int64, device=dev)
    tr = torch.full((B, max(max_updates, 1)), -1, dtype=torch.int32, device=dev) if trace else None
    d = {}
    if dump:
        d = dict(c2v=torch.zeros((B, code.E), device=dev), pre=torch.zeros((B, code.E), device=dev),
                 L=torch.zeros((B, code.N), device=dev), Lt=torch.zeros((B, code.N), device=dev),
                 D=torch.zeros((B, code.N), device=dev))
    rep = None
    rep_len = 0
    if replay is not None:
        rep = torch.as_tensor(replay).to(device=dev, dtype=torch.int32).contiguous()
        _need(rep.dim() == 2 and rep.shape[0] == B, f"replay: shape ({B}, T) is required, got {tuple(rep.shape)}")
        rep_len = rep.shape[1]
    ptr = lambda t: None if t is None else t.data_ptr()
    outs = ldpc_outputs(ptr(bits), ptr(llr_out), ptr(upd), ptr(steps), ptr(fall), ptr(tr), ptr(d.get("c2v")),
                        ptr(d.get("pre")), ptr(d.get("L")), ptr(d.get("Lt")), ptr(d.get("D")))
    s = schedule(kind, arith, gamma, q_bits, frac_bits, n_p, n_g, fill, seed, check_every)
    st = (stream if stream is not None else torch.cuda.current_stream(dev)).cuda_stream
    (ldpc_decode_noalloc if noalloc else ldpc_decode)(code.handle, s, llr.data_ptr(), B, max_updates, ptr(rep),
                                                      rep_len, outs, st)
    return Decoded(bits, llr_out, upd, steps, fall, tr, d.get("c2v"), d.get("pre"), d.get("L"), d.get("Lt"),
                   d.get("D"))


def decode_batch(codes, frames: np.ndarray, llr_pool, out_len: int, arith: int = SPA_F32, q_bits: int = 6,
                 frac_bits: int = 1, check_every: int = 1, stream=None):
    """Batched decode: ``codes`` is a list of ``Code``; ``frames`` a numpy array of FRAME_DESC;
    ``llr_pool`` a float32 CUDA tensor.  Returns (bits_pool, llr_out_pool, updates_used,
    steps_used, fallbacks) as device tensors."""
    import torch
    _need(isinstance(frames, np.ndarray) and frames.dtype == FRAME_DESC and frames.ndim == 1,
          "frames: a 1-D numpy array of FRAME_DESC is required")
    _need(out_len >= 0, "out_len must be >= 0")
    llr_pool = _cuda(llr_pool, "llr_pool", torch.float32).reshape(-1)
    dev = llr_pool.device
    F = len(frames)
    fr = torch.from_numpy(np.ascontiguousarray(frames).view(np.uint8).copy()).to(dev)
    bits = torch.zeros(out_len, dtype=torch.uint8, device=dev)
    llr_out = torch.zeros(out_len, dtype=torch.float32, device=dev)
    upd = torch.zeros(F, dtype=torch.int64, device=dev)
    steps = torch.zeros(F, dtype=torch.int64, device=dev)
    fall = torch.zeros(F, dtype=torch.int64, device=dev)
    s = schedule(0, arith, 0.0, q_bits, frac_bits, 1, 16, 0, 0, check_every)
    st = (stream if stream is not None else torch.cuda.current_stream(dev)).cuda_stream
    ldpc_decode_batch([c.handle for c in codes], s, fr.data_ptr(), F, llr_pool.data_ptr(), llr_pool.numel(),
                      bits.data_ptr(), llr_out.data_ptr(), out_len, upd.data_ptr(), steps.data_ptr(), fall.data_ptr(), st)
    return bits, llr_out, upd, steps, fall


def set_batch_tuning(frames_per_cu: int = 0, storage: int = STORE_AUTO, clear: bool = False) -> None:
    """Launch shape of later ``decode_batch`` calls (process-wide); ``clear`` restores the default."""
    ldpc_set_batch_tuning(None if clear else ldpc_tuning(0, frames_per_cu, storage, TOPO_AUTO))


def get_batch_tuning() -> Optional[dict]:
    t = ldpc_get_batch_tuning()
    return None if t is None else t.as_dict()


def autotune_batch(codes, frames: np.ndarray, llr_pool, out_len: int, arith: int = SPA_F32, q_bits: int = 6,
                   frac_bits: int = 1, check_every: int = 1, reps: int = 2, stream=None):
    """Tune the batched launch on a sample batch (arguments as for ``decode_batch``); returns
    (knobs as a dict, best milliseconds).  The result applies to later ``decode_batch`` calls."""
    import torch
    _need(isinstance(frames, np.ndarray) and frames.dtype == FRAME_DESC and frames.ndim == 1,
          "frames: a 1-D numpy array of FRAME_DESC is required")
    llr_pool = _cuda(llr_pool, "llr_pool", torch.float32).reshape(-1)
    dev = llr_pool.device
    fr = torch.from_numpy(np.ascontiguousarray(frames).view(np.uint8).copy()).to(dev)
    s = schedule(0, arith, 0.0, q_bits, frac_bits, 1, 16, 0, 0, check_every)
    st = (stream if stream is not None else torch.cuda.current_stream(dev)).cuda_stream
    t, ms = ldpc_autotune_batch([c.handle for c in codes], s, fr.data_ptr(), len(frames), llr_pool.data_ptr(),
                                llr_pool.numel(), out_len, reps, st)
    return t.as_dict(), ms


# ----------------------------------------------------------------------------------------------
# differentiable unrolled decoder
# ----------------------------------------------------------------------------------------------
def record_schedule(code: Code, llr, T: int, kind: int = CIRBP, gamma: float = 0.1, stream=None):
    """Record T single-edge updates per frame (no early stop): an int32 (B, T) CUDA tensor."""
    assert kind in (RBP, CIRBP, LMDRBP, SLMDRBP, LMD_CIRBP)
    return decode(code, llr, kind, SPA_F32, max_updates=T, gamma=gamma, check_every=0, trace=True,
                  stream=stream).trace


def unrolled_forward(code: Code, llr, w, trace, ckpt_every: int = 32, checkpoints: bool = True,
                     c2v: bool = False, stream=None):
    """Damped replay of ``trace`` (B, T): returns (soft L (B, N), checkpoints or None, c2v or None)."""
    import torch
    llr = _cuda(llr, "llr", torch.float32, cols=code.N)
    w = torch.as_tensor(w).to(device=llr.device, dtype=torch.float32).contiguous()
    tr = torch.as_tensor(trace).to(device=llr.device, dtype=torch.int32).contiguous()
    _need(tr.dim() == 2 and tr.shape[0] == llr.shape[0],
          f"trace: shape ({llr.shape[0]}, T) is required, got {tuple(tr.shape)}")
    _need(w.numel() == code.E, f"w: {code.E} weights are required, got {w.numel()}")
    B, T = int(tr.shape[0]), int(tr.shape[1])
    soft = torch.empty((B, code.N), dtype=torch.float32, device=llr.device)
    ck = None
    if checkpoints:
        ck = torch.empty(max(1, B * ldpc_unrolled_ckpt_floats(code.handle, T, ckpt_every)), dtype=torch.float32,
                         device=llr.device)
    c2v_out = torch.empty((B, code.E), dtype=torch.float32, device=llr.device) if c2v else None
    st = (stream if stream is not None else torch.cuda.current_stream(llr.device)).cuda_stream
    ptr = lambda t: None if t is None else t.data_ptr()
    ldpc_unrolled_forward(code.handle, llr.data_ptr(), w.data_ptr(), tr.data_ptr(), B, T, ckpt_every, ptr(ck),
                          soft.data_ptr(), ptr(c2v_out), st)
    return soft, ck, c2v_out


def unrolled_backward(code: Code, w, trace, ckpt, grad_soft, ckpt_every: int = 32, stream=None):
    """Adjoint of ``unrolled_forward``: returns (d/d llr (B, N), d/d w (E,))."""
    import torch
    _need(isinstance(grad_soft, torch.Tensor) and grad_soft.is_cuda, "grad_soft: a CUDA tensor is required")
    dev = grad_soft.device
    w = torch.as_tensor(w).to(device=dev, dtype=torch.float32).contiguous()
    tr = torch.as_tensor(trace).to(device=dev, dtype=torch.int32).contiguous()
    _need(tr.dim() == 2, f"trace: shape (B, T) is required, got {tuple(tr.shape)}")
    B, T = int(tr.shape[0]), int(tr.shape[1])
    gs = _cuda(grad_soft.to(dtype=torch.float32), "grad_soft", torch.float32, cols=code.N, rows=B)
    _need(w.numel() == code.E, f"w: {code.E} weights are required, got {w.numel()}")
    if B > 0 and T > 0:
        need = B * ldpc_unrolled_ckpt_floats(code.handle, T, ckpt_every)
        ckpt = _cuda(ckpt, "ckpt", torch.float32, device=dev)
        _need(ckpt.numel() >= need, f"ckpt: {need} floats are required, got {ckpt.numel()}")
    g_llr = torch.empty((B, code.N), dtype=torch.float32, device=dev)
    g_w = torch.empty(code.E, dtype=torch.float32, device=dev)
    st = (stream if stream is not None else torch.cuda.current_stream(dev)).cuda_stream
    ldpc_unrolled_backward(code.handle, w.data_ptr(), tr.data_ptr(), B, T, ckpt_every, ckpt.data_ptr(),
                           gs.data_ptr(), g_llr.data_ptr(), g_w.data_ptr(), st)
    return g_llr, g_w


_unrolled_fn = None


def _unrolled_function():
    global _unrolled_fn
    if _unrolled_fn is None:
        import torch

        class UnrolledDecode(torch.autograd.Function):
            """soft = replay(llr, w; fixed trace); gradients by the hand-written adjoint kernel."""

            @staticmethod
            def forward(ctx, llr, w, code, trace, ckpt_every):
                soft, ck, _ = unrolled_forward(code, llr.detach(), w.detach(), trace, ckpt_every)
                ctx.code = code
                ctx.ckpt_every = ckpt_every
                ctx.save_for_backward(w.detach(), trace, ck)
                return soft

            @staticmethod
            def backward(ctx, grad_soft):
                w, trace, ck = ctx.saved_tensors
                g_llr, g_w = unrolled_backward(ctx.code, w, trace, ck, grad_soft, ctx.ckpt_every)
                return (g_llr if ctx.needs_input_grad[0] else None, g_w if ctx.needs_input_grad[1] else None,
                        None, None, None)

        _unrolled_fn = UnrolledDecode
    return _unrolled_fn


def unrolled_decode(code: Code, llr, w, trace, ckpt_every: int = 32):
    """Differentiable soft output of the damped replay (torch.autograd.Function)."""
    return _unrolled_function().apply(llr, w, code, trace, ckpt_every)


# ----------------------------------------------------------------------------------------------
# launch tuning
# ----------------------------------------------------------------------------------------------
def set_tuning(code: Code, kind: int, arith: int, block: int = 0, frames_per_cu: int = 0, storage: int = 0,
               topology: int = 0, clear: bool = False) -> None:
    ldpc_set_tuning(code.handle, kind, arith, None if clear else ldpc_tuning(block, frames_per_cu, storage, topology))


STORE_NAMES = {STORE_LDS: "lds", STORE_GLOBAL: "global", STORE_GLOBAL_ALL: "global_all",
               STORE_GLOBAL_LT: "global_lt", STORE_GLOBAL_FRAME: "global_frame", STORE_GLOBAL_REC: "global_rec",
               STORE_GLOBAL_STATE: "global_state"}
TOPO_NAMES = {TOPO_GLOBAL: "global", TOPO_LDS: "lds", TOPO_QC: "qc"}


def describe_plan(code: Code, B: int, kind: int, arith: int = SPA_F32, gamma: float = 0.1, q_bits: int = 6,
                  frac_bits: int = 1, n_p: int = 1, n_g: int = 16, fill: int = FILL_LOWEST,
                  check_every: int = 1) -> dict:
    """The launch a decode of B frames would use (on the current device), as a dict; storage and
    topology are also given by name."""
    s = schedule(kind, arith, gamma, q_bits, frac_bits, n_p, n_g, fill, 0, check_every)
    d = ldpc_describe_plan(code.handle, s, B).as_dict()
    d["storage_name"] = STORE_NAMES.get(d["storage"], "?")
    d["topology_name"] = TOPO_NAMES.get(d["topology"], "?")
    return d


def describe_batch_plan(codes, F: int, arith: int = SPA_F32, q_bits: int = 6, frac_bits: int = 1,
                        check_every: int = 1) -> dict:
    """The launch ``decode_batch`` would use for F frames over these codes (on the current device)."""
    s = schedule(0, arith, 0.0, q_bits, frac_bits, 1, 16, 0, 0, check_every)
    d = ldpc_describe_batch_plan([c.handle for c in codes], s, F).as_dict()
    d["storage_name"] = STORE_NAMES.get(d["storage"], "?")
    d["topology_name"] = TOPO_NAMES.get(d["topology"], "?")
    return d


def autotune(code: Code, llr, kind: int, arith: int = SPA_F32, max_updates: int = 0, gamma: float = 0.1,
             q_bits: int = 6, frac_bits: int = 1, n_p: int = 1, n_g: int = 16, fill: int = FILL_LOWEST,
             check_every: int = 1, reps: int = 2, stream=None):
    """Tune the launch of one schedule on sample frames (a (B, N) float32 CUDA tensor); returns
    (knobs as a dict, best milliseconds).  The result is kept for later decodes of this code."""
    import torch
    llr = _cuda(llr, "llr", torch.float32, cols=code.N)
    s = schedule(kind, arith, gamma, q_bits, frac_bits, n_p, n_g, fill, 0, check_every)
    st = (stream if stream is not None else torch.cuda.current_stream(llr.device)).cuda_stream
    t, ms = ldpc_autotune(code.handle, s, llr.data_ptr(), llr.shape[0], max_updates, reps, st)
    return t.as_dict(), ms


# ----------------------------------------------------------------------------------------------
# SNR sweeps (one captured hipGraph per sweep)
# ----------------------------------------------------------------------------------------------
def awgn_frames(codewords, B: int, sigma2: float, seed: int, point: int = 0, stream=None):
    """(B, N) float32 channel LLRs on the device from a (P, N) uint8 CUDA codeword pool."""
    import torch
    cw = _cuda(codewords, "codewords", torch.uint8)
    _need(cw.dim() == 2, f"codewords: shape (P, N) is required, got {tuple(cw.shape)}")
    P, N = cw.shape
    llr = torch.empty((B, N), dtype=torch.float32, device=cw.device)
    st = (stream if stream is not None else torch.cuda.current_stream(cw.device)).cuda_stream
    ldpc_awgn_frames(cw.data_ptr(), P, N, B, sigma2, seed, point, llr.data_ptr(), st)
    return llr


def probe_lds(width: int = 16, blocks: int = 0, iters: int = 2048, stream=None) -> float:
    """Measured LDS read bandwidth in GB/s (``ldpc_probe_lds``): `blocks` workgroups of 256 lanes
    (default 8 per CU of device 0), `iters` x 16 reads of `width` bytes per lane."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    if blocks <= 0:
        blocks = 8 * torch.cuda.get_device_properties(dev).multi_processor_count
    sink = torch.zeros(blocks, dtype=torch.int32, device=dev)
    st = (stream if stream is not None else torch.cuda.current_stream(dev)).cuda_stream
    nbytes, ms = ldpc_probe_lds(width, blocks, iters, sink.data_ptr(), st)
    return nbytes / (ms * 1e-3) / 1e9


class Sweep:
    """A captured sweep: ``run(seed)`` returns an int64 (S, 4) CUDA tensor of per-point
    (frames, frame errors, bit errors, sum of updates)."""

    def __init__(self, code: Code, codewords, ebn0_db, rate: float, B: int, kind: int, arith: int = SPA_F32,
                 max_updates: int = 0, gamma: float = 0.1, q_bits: int = 6, frac_bits: int = 1, n_p: int = 1,
                 n_g: int = 16, fill: int = FILL_LOWEST, check_every: int = 1):
        import torch
        self.code = code
        self.codewords = _cuda(codewords, "codewords", torch.uint8, cols=code.N)  # referenced by the graph
        self.S = len(ebn0_db)
        s = schedule(kind, arith, gamma, q_bits, frac_bits, n_p, n_g, fill, 0, check_every)
        self.handle = ldpc_sweep_create(code.handle, s, max_updates, self.codewords.data_ptr(),
                                        self.codewords.shape[0], ebn0_db, rate, B)

    def run(self, seed: int, stream=None):
        import torch
        dev = self.codewords.device
        out = torch.empty((self.S, 4), dtype=torch.int64, device=dev)
        st = (stream if stream is not None else torch.cuda.current_stream(dev)).cuda_stream
        ldpc_sweep_run(self.handle, seed, out.data_ptr(), st)
        return out

    def close(self):
        if getattr(self, "handle", None):
            ldpc_sweep_free(self.handle)
            self.handle = None

    def __del__(self):
        if _lib is not None:
            self.close()
