"""Brute-force decoding of tiny codes by codeword enumeration (TEST INFRASTRUCTURE ONLY).

These are the exact references the oracle is pinned to: they use no message passing at all.

* ``codewords``: all 2^K codewords, from an own GF(2) null-space basis of H;
* ``bitwise_map_llr``: log P(u_n = 0 | y) / P(u_n = 1 | y) for equiprobable codewords, i.e. the
  a-posteriori LLR that belief propagation computes exactly on cycle-free graphs;
* ``ml_codeword``: the codeword maximising sum_n (1 - 2 c_n) llr_n (maximum likelihood on the
  BPSK/AWGN channel with LLRs 2 y / sigma^2).
"""
from __future__ import annotations

import numpy as np


def nullspace_gf2(H: np.ndarray) -> np.ndarray:
    """Basis (K x N) of {c : H c = 0 mod 2} by Gauss-Jordan elimination on uint8 rows."""
    A = (np.asarray(H, dtype=np.uint8) & 1).copy()
    M, N = A.shape
    piv_cols = []
    r = 0
    for c in range(N):
        rows = np.nonzero(A[r:, c])[0]
        if len(rows) == 0:
            continue
        p = r + rows[0]
        A[[r, p]] = A[[p, r]]
        for rr in range(M):
            if rr != r and A[rr, c]:
                A[rr] ^= A[r]
        piv_cols.append(c)
        r += 1
        if r == M:
            break
    free = [c for c in range(N) if c not in piv_cols]
    basis = np.zeros((len(free), N), dtype=np.uint8)
    for k, fcol in enumerate(free):
        basis[k, fcol] = 1
        for i, pc in enumerate(piv_cols):
            basis[k, pc] = A[i, fcol]
    return basis


def codewords(H: np.ndarray) -> np.ndarray:
    basis = nullspace_gf2(H)
    K = basis.shape[0]
    assert K <= 20, "too many codewords to enumerate"
    msgs = ((np.arange(2 ** K)[:, None] >> np.arange(K)[None, :]) & 1).astype(np.int64)
    return ((msgs @ basis.astype(np.int64)) & 1).astype(np.uint8)


def _logsumexp(x: np.ndarray) -> float:
    m = np.max(x)
    return float(m + np.log(np.sum(np.exp(x - m))))


def bitwise_map_llr(H: np.ndarray, llr: np.ndarray, cws: np.ndarray = None) -> np.ndarray:
    """Exact a-posteriori LLRs.  P(c | y) is proportional to exp(sum_n (1 - 2 c_n) llr_n / 2)."""
    if cws is None:
        cws = codewords(H)
    llr = np.asarray(llr, dtype=np.float64)
    score = 0.5 * ((1.0 - 2.0 * cws) @ llr)
    out = np.zeros(len(llr))
    for n in range(len(llr)):
        out[n] = _logsumexp(score[cws[:, n] == 0]) - _logsumexp(score[cws[:, n] == 1])
    return out


def ml_codeword(H: np.ndarray, llr: np.ndarray, cws: np.ndarray = None) -> np.ndarray:
    if cws is None:
        cws = codewords(H)
    score = (1.0 - 2.0 * cws) @ np.asarray(llr, dtype=np.float64)
    return cws[int(np.argmax(score))]
