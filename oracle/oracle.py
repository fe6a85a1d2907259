"""Python access to the plain C oracle (``ldpc_oracle.c``, ``unrolled_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg of the
benchmark use it; the GPU library never does.  The oracle shares no code with the GPU path.

``decode`` mirrors the GPU library's ``decode`` in its arguments and outputs, with the channel
LLRs taken as float64 (they are the same float32 values the GPU receives, widened exactly).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "ldpc_oracle.c"), os.path.join(_HERE, "unrolled_oracle.c")]
_LIB = os.path.join(_HERE, "libldpc_oracle.so")

FLOODING, LAYERED, RBP, CIRBP, MECIRBP, REPLAY, LMDRBP, SLMDRBP, LMDCIRBP, MELMDCIRBP = range(10)
FILL_LOWEST, FILL_HASH = 0, 1
SPA, MSFIX = 0, 1
COUNTERS = ("prop", "v2c", "pre", "ci", "ci_self", "fallback", "cmp", "steps")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, -O2)."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(s) for s in _SRCS)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, *_SRCS,
                               "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


class _Code(C.Structure):
    _fields_ = [("M", C.c_int32), ("N", C.c_int32), ("E", C.c_int32),
                ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("col_ptr", C.c_void_p), ("col_row", C.c_void_p), ("col_eid", C.c_void_p),
                ("n_layers", C.c_int32), ("layer_ptr", C.c_void_p)]


class _Sched(C.Structure):
    _fields_ = [("kind", C.c_int32), ("arith", C.c_int32), ("q_bits", C.c_int32),
                ("frac_bits", C.c_int32), ("gamma", C.c_double), ("n_p", C.c_int32),
                ("n_g", C.c_int32), ("check_every", C.c_int64), ("selfcheck", C.c_int32),
                ("fill", C.c_int32), ("seed", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.oc_decode.restype = C.c_int
        P = C.c_void_p
        _lib.oc_decode.argtypes = [P, P, C.c_int32, P, C.c_int64, P, C.c_int64, P, P, P, P, P, P,
                                   P, P, P, P, P, C.c_int32]
        _lib.oc_boxplus.restype = C.c_double
        _lib.oc_boxplus.argtypes = [C.c_double, C.c_double]
        _lib.oc_c2v_tanh.restype = C.c_double
        _lib.oc_c2v_tanh.argtypes = [C.c_void_p, C.c_int]
        _lib.oc_ci_spa.restype = C.c_double
        _lib.oc_ci_spa.argtypes = [C.c_double, C.c_double]
        _lib.oc_splitmix64.restype = C.c_uint64
        _lib.oc_splitmix64.argtypes = [C.c_uint64]
        _lib.oc_fill_key.restype = C.c_uint64
        _lib.oc_fill_key.argtypes = [C.c_uint64] * 4
        _lib.oc_alg4_select_keyed.restype = C.c_int32
        _lib.oc_alg4_select_keyed.argtypes = [C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                              C.c_void_p]
        _lib.ou_forward.restype = C.c_int
        _lib.ou_forward.argtypes = [P, C.c_int32, P, P, P, C.c_int32, P, P, C.c_int32]
        _lib.ou_backward.restype = C.c_int
        _lib.ou_backward.argtypes = [P, C.c_int32, P, P, P, C.c_int32, P, P, P, C.c_int32]
        _lib.ou_boxplus_grad.restype = C.c_double
        _lib.ou_boxplus_grad.argtypes = [C.c_double, C.c_double]
        _lib.oc_alg4_select_excl.restype = C.c_int32
        _lib.oc_alg4_select_excl.argtypes = [C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                             C.c_void_p, C.c_void_p]
        _lib.oc_alg4_select.restype = C.c_int32
        _lib.oc_alg4_select.argtypes = [C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


@dataclass
class Result:
    bits: np.ndarray
    llr_out: np.ndarray
    updates_used: np.ndarray
    steps_used: np.ndarray
    trace: Optional[np.ndarray] = None
    counters: Optional[np.ndarray] = None
    c2v: Optional[np.ndarray] = None
    pre: Optional[np.ndarray] = None
    L: Optional[np.ndarray] = None
    Lt: Optional[np.ndarray] = None
    D: Optional[np.ndarray] = None

    def counter(self, name: str) -> np.ndarray:
        return self.counters[:, COUNTERS.index(name)]


def _code_struct(code):
    """ctypes view of a ``synth.Code`` (the arrays in ``keep`` must outlive the call)."""
    col_ptr, col_row, col_eid = code.csc()
    keep = [np.ascontiguousarray(a, dtype=np.int32) for a in
            (code.row_ptr, code.col, col_ptr, col_row, col_eid)]
    lp = None if code.layer_ptr is None else np.ascontiguousarray(code.layer_ptr, dtype=np.int32)
    keep.append(lp)
    H = _Code(code.M, code.N, code.E, *[a.ctypes.data for a in keep[:5]],
              0 if lp is None else len(lp) - 1, _ptr(lp))
    return H, keep


def decode(code, llr, kind: int, arith: int = SPA, max_updates: int = 0, gamma: float = 0.1,
           q_bits: int = 6, frac_bits: int = 1, n_p: int = 1, n_g: int = 16, check_every: int = 1,
           replay: Optional[np.ndarray] = None, trace: bool = False, dump: bool = False,
           selfcheck: bool = False, threads: int = 1, fill: int = 0, seed: int = 0) -> Result:
    """Run the oracle on B frames.  ``code`` is a ``synth.Code``; llr is (B, N)."""
    llr = np.ascontiguousarray(np.asarray(llr, dtype=np.float64))
    if llr.ndim == 1:
        llr = llr[None]
    B, N = llr.shape
    assert N == code.N
    H, keep = _code_struct(code)
    s = _Sched(kind, arith, q_bits, frac_bits, gamma, n_p, n_g, check_every, int(selfcheck), fill,
               seed & (2**64 - 1))
    bits = np.zeros((B, N), dtype=np.uint8)
    llr_out = np.zeros((B, N), dtype=np.float64)
    upd = np.zeros(B, dtype=np.int64)
    steps = np.zeros(B, dtype=np.int64)
    tr = np.full((B, max(max_updates, 1)), -1, dtype=np.int32) if trace else None
    cnt = np.zeros((B, len(COUNTERS)), dtype=np.int64)
    d = {}
    if dump:
        d = dict(c2v=np.zeros((B, code.E)), pre=np.zeros((B, code.E)), L=np.zeros((B, N)),
                 Lt=np.zeros((B, N)), D=np.zeros((B, N)))
    rep = None
    rep_len = 0
    if kind == REPLAY:
        rep = np.ascontiguousarray(replay, dtype=np.int32)
        if rep.ndim == 1:
            rep = rep[None]
        rep_len = rep.shape[1]
    rc = lib().oc_decode(C.byref(H), C.byref(s), C.c_int32(B), _ptr(llr), C.c_int64(max_updates),
                         _ptr(rep), C.c_int64(rep_len), _ptr(bits), _ptr(llr_out), _ptr(upd),
                         _ptr(steps), _ptr(tr), _ptr(cnt), _ptr(d.get("c2v")), _ptr(d.get("pre")),
                         _ptr(d.get("L")), _ptr(d.get("Lt")), _ptr(d.get("D")), C.c_int32(threads))
    if rc != 0:
        raise RuntimeError(f"oracle error {rc}")
    return Result(bits, llr_out, upd, steps, tr, cnt, d.get("c2v"), d.get("pre"), d.get("L"),
                  d.get("Lt"), d.get("D"))


def boxplus(a: float, b: float) -> float:
    return lib().oc_boxplus(a, b)


def c2v_tanh(v) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().oc_c2v_tanh(v.ctypes.data, len(v))


def ci_spa(L: float, Lt: float) -> float:
    return lib().oc_ci_spa(L, Lt)


def alg4_select(bins, n_g: int, n_p: int) -> np.ndarray:
    bins = np.ascontiguousarray(bins, dtype=np.int32)
    out = np.zeros(len(bins), dtype=np.int32)
    k = lib().oc_alg4_select(len(bins), bins.ctypes.data, n_g, n_p, out.ctypes.data)
    return out[:k]


def splitmix64(z: int) -> int:
    return lib().oc_splitmix64(z & (2**64 - 1))


def fill_key(seed: int, frame: int, step: int, n: int) -> int:
    return lib().oc_fill_key(seed & (2**64 - 1), frame, step, n)


def alg4_select_keyed(bins, n_g: int, n_p: int, keys) -> np.ndarray:
    bins = np.ascontiguousarray(bins, dtype=np.int32)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.zeros(len(bins), dtype=np.int32)
    k = lib().oc_alg4_select_keyed(len(bins), bins.ctypes.data, n_g, n_p, keys.ctypes.data, out.ctypes.data)
    return out[:k]


def alg4_select_excl(bins, n_g: int, n_p: int, excl, keys=None) -> np.ndarray:
    """Algorithm 4 among the VNs with excl[n] == 0 (Algorithm 6's refill)."""
    bins = np.ascontiguousarray(bins, dtype=np.int32)
    excl = np.ascontiguousarray(excl, dtype=np.uint8)
    kp = None if keys is None else np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.zeros(len(bins), dtype=np.int32)
    k = lib().oc_alg4_select_excl(len(bins), bins.ctypes.data, n_g, n_p, None if kp is None else kp.ctypes.data,
                                  excl.ctypes.data, out.ctypes.data)
    return out[:k]


# ----------------------------------------------------------------------------------------------
# damped replay of a fixed schedule and its gradient (unrolled_oracle.c)
# ----------------------------------------------------------------------------------------------
def _unrolled_args(code, llr, w, trace):
    llr = np.ascontiguousarray(np.asarray(llr, dtype=np.float64))
    if llr.ndim == 1:
        llr = llr[None]
    tr = np.ascontiguousarray(trace, dtype=np.int32)
    if tr.ndim == 1:
        tr = tr[None]
    w = np.ascontiguousarray(np.broadcast_to(np.asarray(w, dtype=np.float64), (code.E,)))
    assert llr.shape[1] == code.N and tr.shape[0] == llr.shape[0]
    return llr, w, tr


def unrolled_forward(code, llr, w, trace, threads: int = 1):
    """Damped replay of ``trace`` (B, T) from c2v = 0, L = llr: returns (L (B, N), c2v (B, E))."""
    llr, w, tr = _unrolled_args(code, llr, w, trace)
    B, T = tr.shape
    H, keep = _code_struct(code)
    L = np.zeros((B, code.N))
    c2v = np.zeros((B, code.E))
    rc = lib().ou_forward(C.byref(H), B, llr.ctypes.data, w.ctypes.data, tr.ctypes.data, T, L.ctypes.data,
                          c2v.ctypes.data, threads)
    if rc != 0:
        raise RuntimeError(f"oracle error {rc}")
    return L, c2v


def unrolled_backward(code, llr, w, trace, grad_L, threads: int = 1):
    """Gradient through the damped replay: returns (d/d llr (B, N), per-frame d/d w (B, E))."""
    llr, w, tr = _unrolled_args(code, llr, w, trace)
    B, T = tr.shape
    gL = np.ascontiguousarray(np.asarray(grad_L, dtype=np.float64).reshape(B, code.N))
    H, keep = _code_struct(code)
    g_llr = np.zeros((B, code.N))
    g_w = np.zeros((B, code.E))
    rc = lib().ou_backward(C.byref(H), B, llr.ctypes.data, w.ctypes.data, tr.ctypes.data, T, gL.ctypes.data,
                           g_llr.ctypes.data, g_w.ctypes.data, threads)
    if rc != 0:
        raise RuntimeError(f"oracle error {rc}")
    return g_llr, g_w


def boxplus_grad(a: float, b: float) -> float:
    return lib().ou_boxplus_grad(a, b)
