"""Seeded synthetic inputs shared by the decoder tests, the benchmark and the oracle tests.

This module holds no decoder arithmetic.  It builds parity-check matrices, draws random codewords
and produces BPSK/AWGN channel LLRs, i.e. everything the decoders take as *input*:

* the code model: an M x N parity-check matrix H, with M(n) / N(m) adjacency (Sec. II-A);
* the channel: BPSK x_n = 1 - 2 u_n over AWGN with variance sigma^2, channel LLR 2 y_n / sigma^2
  (Sec. II-A and Sec. V), sigma^2 = 1 / (2 R 10^(Eb/N0 / 10)) for unit-energy symbols.

The paper's own codes (IEEE 802.11 and 5G NR matrices, a Gallager code from an archive) are not
reproduced; the generators below build seeded stand-ins of the same length/rate class:

* ``peg_regular``: (dv, dc)-regular code by progressive edge growth (Hu, Eleftheriou, Arnold, 2005);
* ``qc_bg1_shaped``: 46 x 68 quasi-cyclic base matrix with a degree profile shaped like a
  base-graph-1 code (22 information columns, 4 core parity columns, 42 degree-one extension
  columns; 316 nonzero blocks), random circulant shifts;
* ``qc_24col``: 24-column quasi-cyclic family with a dual-diagonal parity part (rates 1/2 .. 5/6).

Canonical edge order everywhere: edge id = position in the row-major (check-major, VN ascending)
enumeration of the nonzeros of H.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


# ----------------------------------------------------------------------------------------------
# Code container
# ----------------------------------------------------------------------------------------------
@dataclass
class Code:
    """Parity-check matrix in CSR form with canonical (row-major) edge ids.

    ``layer_ptr`` partitions the rows into consecutive layers [layer_ptr[l], layer_ptr[l+1]);
    rows inside one layer touch disjoint VN sets (checked by ``validate``).  ``None`` means
    one row per layer.
    """

    M: int
    N: int
    row_ptr: np.ndarray  # int32 [M+1]
    col: np.ndarray  # int32 [E], ascending inside each row
    layer_ptr: Optional[np.ndarray] = None  # int32 [n_layers+1]
    name: str = ""
    design_rate: float = 0.5
    # quasi-cyclic description, when the code has one: base shifts (mb x nb, -1 = zero block), Z
    qc_shift: Optional[np.ndarray] = None
    qc_Z: int = 0
    _gen: Optional[tuple] = field(default=None, repr=False)

    @property
    def E(self) -> int:
        return int(self.row_ptr[-1])

    def row_of_edge(self) -> np.ndarray:
        return np.repeat(np.arange(self.M, dtype=np.int32), np.diff(self.row_ptr)).astype(np.int32)

    def csc(self):
        """(col_ptr[N+1], col_row[E], col_eid[E]); inside a column the checks ascend."""
        rows = self.row_of_edge()
        eid = np.arange(self.E, dtype=np.int32)
        order = np.lexsort((rows, self.col))
        col_ptr = np.zeros(self.N + 1, dtype=np.int32)
        np.add.at(col_ptr, self.col.astype(np.int64) + 1, 1)
        col_ptr = np.cumsum(col_ptr).astype(np.int32)
        return col_ptr, rows[order].astype(np.int32), eid[order].astype(np.int32)

    def dense(self) -> np.ndarray:
        H = np.zeros((self.M, self.N), dtype=np.uint8)
        H[self.row_of_edge(), self.col] = 1
        return H

    def validate(self) -> None:
        rp, c = self.row_ptr, self.col
        assert rp.dtype == np.int32 and c.dtype == np.int32
        assert rp[0] == 0 and len(rp) == self.M + 1 and np.all(np.diff(rp) >= 1)
        for m in range(self.M):
            r = c[rp[m]:rp[m + 1]]
            assert np.all(np.diff(r) > 0), f"row {m} not strictly ascending"
            assert r.min() >= 0 and r.max() < self.N
        assert np.all(np.bincount(c, minlength=self.N) >= 1), "VN without edges"
        if self.layer_ptr is not None:
            lp = self.layer_ptr
            assert lp[0] == 0 and lp[-1] == self.M and np.all(np.diff(lp) >= 1)
            for l in range(len(lp) - 1):
                vs = c[rp[lp[l]]:rp[lp[l + 1]]]
                assert len(np.unique(vs)) == len(vs), f"layer {l} rows share a VN"

    # GF(2) generator (pivot/free split) cached per code
    def generator(self):
        if self._gen is None:
            self._gen = gf2_nullspace_map(self.dense())
        return self._gen

    @property
    def K(self) -> int:
        return len(self.generator()[1])


def code_from_rows(M: int, N: int, rows: list, **kw) -> Code:
    row_ptr = np.zeros(M + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum([len(r) for r in rows])
    col = np.concatenate([np.sort(np.asarray(r, dtype=np.int32)) for r in rows]).astype(np.int32)
    return Code(M=M, N=N, row_ptr=row_ptr, col=col, **kw)


# ----------------------------------------------------------------------------------------------
# PEG (3,6)-regular codes
# ----------------------------------------------------------------------------------------------
def peg_regular(N: int, dv: int = 3, dc: int = 6, seed: int = 1) -> Code:
    """Progressive edge growth, VN by VN; each new edge goes to a check as far as possible from
    the VN in the current graph (lowest current degree first, seeded random tie-break), with the
    check degree capped at dc so that the result is (dv, dc)-regular."""
    assert (N * dv) % dc == 0
    M = N * dv // dc
    rng = np.random.default_rng(seed)
    vn_adj = [[] for _ in range(N)]
    cn_adj = [[] for _ in range(M)]
    cdeg = np.zeros(M, dtype=np.int64)

    def pick(cands):
        cands = np.asarray(sorted(cands))
        d = cdeg[cands]
        best = cands[d == d.min()]
        return int(best[rng.integers(len(best))])

    for j in range(N):
        for k in range(dv):
            open_checks = {m for m in range(M) if cdeg[m] < dc} - set(vn_adj[j])
            if k == 0:
                m_sel = pick(open_checks)
            else:
                # breadth-first expansion from v_j over the current graph, one check level at
                # a time; stop when the reached set stops growing or would cover every open
                # check, and pick among the open checks not reached at that depth
                reached = set(vn_adj[j])
                frontier = set(reached)
                seen_v = {j}
                while True:
                    new_v = {v for m in frontier for v in cn_adj[m]} - seen_v
                    seen_v |= new_v
                    new_c = {m for v in new_v for m in vn_adj[v]} - reached
                    if not new_c or not (open_checks - (reached | new_c)):
                        cand = open_checks - reached
                        if not cand:
                            cand = open_checks
                        break
                    reached |= new_c
                    frontier = new_c
                m_sel = pick(cand)
            vn_adj[j].append(m_sel)
            cn_adj[m_sel].append(j)
            cdeg[m_sel] += 1
    rows = [sorted(cn_adj[m]) for m in range(M)]
    code = code_from_rows(M, N, rows, name=f"peg({dv},{dc})N{N}s{seed}", design_rate=1 - dv / dc)
    code.validate()
    return code


# ----------------------------------------------------------------------------------------------
# Quasi-cyclic codes
# ----------------------------------------------------------------------------------------------
def expand_qc(shift: np.ndarray, Z: int, name: str = "", design_rate: float = 0.5) -> Code:
    """Lift a base matrix: block (i, j) with shift s >= 0 connects check i*Z + r to VN
    j*Z + ((r + s) mod Z).  Layers are the block rows (Z VN-disjoint rows each)."""
    mb, nb = shift.shape
    rows = []
    for i in range(mb):
        js = [j for j in range(nb) if shift[i, j] >= 0]
        assert js, f"empty base row {i}"
        for r in range(Z):
            rows.append([j * Z + ((r + int(shift[i, j])) % Z) for j in js])
    code = code_from_rows(mb * Z, nb * Z, rows, name=name, design_rate=design_rate)
    code.layer_ptr = (np.arange(mb + 1, dtype=np.int32) * Z).astype(np.int32)
    code.qc_shift = shift.astype(np.int16)
    code.qc_Z = Z
    code.validate()
    return code


def qc_regular(dv: int, dc: int, Z: int, seed: int = 1) -> Code:
    """(dv, dc)-regular QC code: an all-ones dv x dc base lifted by Z with seeded shifts, redrawn
    until no 2 x 2 block submatrix closes a 4-cycle (s11 - s12 + s22 - s21 != 0 mod Z), so the
    Tanner graph has girth at least 6.  n = dc Z, design rate 1 - dv/dc."""
    rng = np.random.default_rng(seed)
    for _ in range(10000):
        shift = rng.integers(0, Z, size=(dv, dc))
        ok = True
        for i1 in range(dv):
            for i2 in range(i1 + 1, dv):
                d = (shift[i1] - shift[i2]) % Z  # 4-cycle: equal differences in two columns
                if len(np.unique(d)) < dc:
                    ok = False
                    break
            if not ok:
                break
        if ok:
            return expand_qc(shift.astype(np.int32), Z, name=f"qc{dv}{dc}_Z{Z}s{seed}", design_rate=1 - dv / dc)
    raise RuntimeError("no 4-cycle-free shifts found")


def bg1_shaped_base(seed: int = 1) -> np.ndarray:
    """46 x 68 base pattern (1 = circulant, 0 = zero block) with 316 nonzeros.

    Columns: 0..21 information, 22..25 core parity, 26..67 degree-one extension parity.
    Rows:    0..3 core, 4..45 extension.  Columns 0 and 1 are the heavy columns."""
    rng = np.random.default_rng(seed)
    B = np.zeros((46, 68), dtype=np.int8)
    # core rows: 19 of 22 information columns each (heavy columns always present)
    for i in range(4):
        drop = rng.choice(np.arange(2, 22), size=3, replace=False)
        B[i, :22] = 1
        B[i, drop] = 0
    # core parity: weight-3 column then a dual diagonal
    for i, j in [(0, 22), (1, 22), (3, 22), (0, 23), (1, 23), (1, 24), (2, 24), (2, 25), (3, 25)]:
        B[i, j] = 1
    # extension rows: own degree-one column plus entries in the information/core columns
    n_other = [7] * 6 + [5] * 3 + [4] * 33
    assert sum(n_other) == 189
    for t, r in enumerate(range(4, 46)):
        B[r, 26 + t] = 1
        heavy = 0 if t % 2 == 0 else 1
        B[r, heavy] = 1
        pool = np.arange(2, 26)
        w = np.where(pool < 22, 1.0, 0.25)
        pick = rng.choice(pool, size=n_other[t] - 1, replace=False, p=w / w.sum())
        B[r, pick] = 1
    assert int(B.sum()) == 316
    return B


def qc_bg1_shaped(Z: int, seed: int = 1) -> Code:
    """BG1-shaped 46 x 68 QC code, n = 68 Z, design rate 22/68, shifts uniform in [0, Z)."""
    B = bg1_shaped_base(seed)
    rng = np.random.default_rng(seed + 1000003)
    shift = np.where(B > 0, rng.integers(0, Z, size=B.shape), -1).astype(np.int32)
    return expand_qc(shift, Z, name=f"bg1shaped_Z{Z}s{seed}", design_rate=22 / 68)


def qc_24col_base(mb: int, seed: int = 1) -> np.ndarray:
    """24-column base pattern with mb rows: (24 - mb) information columns with seeded weights,
    then a weight-3 parity column and a dual diagonal (802.11-like parity structure)."""
    rng = np.random.default_rng(seed * 7919 + mb)
    nb = 24
    kb = nb - mb
    B = np.zeros((mb, nb), dtype=np.int8)
    # parity part
    B[0, kb] = B[mb // 2, kb] = B[mb - 1, kb] = 1
    for t in range(1, mb):
        B[t - 1, kb + t] = 1
        B[t, kb + t] = 1
    # information columns: target about 3.58 average VN degree overall for rate 1/2 (86 entries)
    target_info = {12: 86, 8: 88, 6: 88, 4: 80}.get(mb, 4 * kb) - int(B.sum())
    w = np.full(kb, max(2, target_info // kb))
    extra = target_info - int(w.sum())
    for _ in range(max(0, extra)):
        w[rng.integers(kb)] += 1
    w = np.minimum(w, mb)
    for j in range(kb):
        rows = rng.choice(mb, size=int(w[j]), replace=False)
        B[rows, j] = 1
    # every row needs at least two entries
    for i in range(mb):
        while B[i].sum() < 2:
            B[i, rng.integers(kb)] = 1
    return B


def qc_24col(Z: int, mb: int, seed: int = 1) -> Code:
    B = qc_24col_base(mb, seed)
    rng = np.random.default_rng(seed * 104729 + Z * 31 + mb)
    shift = np.where(B > 0, rng.integers(0, Z, size=B.shape), -1).astype(np.int32)
    return expand_qc(shift, Z, name=f"qc24_Z{Z}_mb{mb}s{seed}", design_rate=1 - mb / 24)


# ----------------------------------------------------------------------------------------------
# Small hand-made codes used by tests
# ----------------------------------------------------------------------------------------------
def spc_code(N: int) -> Code:
    """Single parity check of length N (one check row)."""
    c = code_from_rows(1, N, [list(range(N))], name=f"spc{N}", design_rate=(N - 1) / N)
    c.validate()
    return c


def random_tree_code(n_checks: int, seed: int = 0, max_dc: int = 4) -> Code:
    """Random cycle-free Tanner graph: checks are added one by one, each attaching to exactly
    one existing VN plus fresh VNs, so the bipartite graph stays a tree."""
    rng = np.random.default_rng(seed)
    rows = []
    N = int(rng.integers(2, max_dc + 1))
    rows.append(list(range(N)))
    for _ in range(n_checks - 1):
        anchor = int(rng.integers(N))
        fresh = int(rng.integers(1, max_dc))
        rows.append([anchor] + list(range(N, N + fresh)))
        N += fresh
    c = code_from_rows(len(rows), N, rows, name=f"tree{n_checks}s{seed}", design_rate=0.5)
    c.validate()
    return c


# ----------------------------------------------------------------------------------------------
# GF(2) encoding
# ----------------------------------------------------------------------------------------------
def gf2_nullspace_map(H: np.ndarray):
    """Reduced row echelon form of H over GF(2) with bit-packed rows.

    Returns (pivots, free, A) such that every codeword c satisfies
    c[pivots] = A @ c[free] (mod 2), with A of shape (rank, K); K = N - rank."""
    M, N = H.shape
    W = (N + 63) // 64
    padded = np.zeros((M, W * 64), dtype=np.uint8)
    padded[:, :N] = H
    rowsbits = np.packbits(padded, axis=1, bitorder="little").view(np.uint64).copy()
    pivots = []
    r = 0
    for c in range(N):
        if r == M:
            break
        w, b = divmod(c, 64)
        bit = np.uint64(1) << np.uint64(b)
        col = (rowsbits[r:, w] & bit) != 0
        nz = np.nonzero(col)[0]
        if len(nz) == 0:
            continue
        p = r + nz[0]
        if p != r:
            rowsbits[[r, p]] = rowsbits[[p, r]]
        mask = (rowsbits[:, w] & bit) != 0
        mask[r] = False
        rowsbits[mask] ^= rowsbits[r]
        pivots.append(c)
        r += 1
    rank = r
    R = np.unpackbits(rowsbits[:rank].view(np.uint8), axis=1, bitorder="little")[:, :N]
    pivots = np.asarray(pivots, dtype=np.int64)
    free = np.setdiff1d(np.arange(N), pivots)
    A = R[:, free].astype(np.uint8)
    return pivots, free, A


def encode(code: Code, info: np.ndarray) -> np.ndarray:
    """Codewords (B x N, uint8) for information bits placed on the free columns (B x K)."""
    pivots, free, A = code.generator()
    info = np.asarray(info, dtype=np.uint8)
    B = info.shape[0]
    cw = np.zeros((B, code.N), dtype=np.uint8)
    cw[:, free] = info
    cw[:, pivots] = (info.astype(np.int64) @ A.T.astype(np.int64)) & 1
    return cw


def random_codewords(code: Code, B: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    info = rng.integers(0, 2, size=(B, code.K), dtype=np.uint8)
    return encode(code, info)


# ----------------------------------------------------------------------------------------------
# BPSK / AWGN channel
# ----------------------------------------------------------------------------------------------
def sigma2_from_ebn0(ebn0_db: float, rate: float) -> float:
    """Noise variance for unit-energy BPSK at the given Eb/N0 and code rate (N0/2 = sigma^2)."""
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def awgn_llr(codewords: np.ndarray, sigma2: float, seed: int, dtype=np.float32) -> np.ndarray:
    """Channel LLRs 2 y / sigma^2 with y = (1 - 2 u) + w, w ~ N(0, sigma^2)."""
    rng = np.random.default_rng(seed)
    x = 1.0 - 2.0 * codewords.astype(np.float64)
    y = x + np.sqrt(sigma2) * rng.standard_normal(x.shape)
    return (2.0 * y / sigma2).astype(dtype)


def frames(code: Code, B: int, ebn0_db: float, seed: int, zero_codeword: bool = False,
           rate: Optional[float] = None, dtype=np.float32):
    """(codewords, llr) for B frames at Eb/N0 (dB); seeds for info and noise derive from seed."""
    if zero_codeword:
        cw = np.zeros((B, code.N), dtype=np.uint8)
    else:
        cw = random_codewords(code, B, seed * 2 + 1)
    s2 = sigma2_from_ebn0(ebn0_db, code.design_rate if rate is None else rate)
    return cw, awgn_llr(cw, s2, seed * 2 + 2, dtype=dtype)


# ----------------------------------------------------------------------------------------------
# Counter-based channel noise (the recipe of the on-device sweep generator)
# ----------------------------------------------------------------------------------------------
_PHILOX_M0, _PHILOX_M1 = 0xD2511F53, 0xCD9E8D57   # round multipliers
_PHILOX_W0, _PHILOX_W1 = 0x9E3779B9, 0xBB67AE85   # key increments (Weyl sequence)


def philox4x32_10(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
    as 1, 2, 3", SC 2011): ctr (..., 4) and key (..., 2) uint32 arrays -> (..., 4) uint32."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64) + np.zeros_like(c[0])
    k1 = np.asarray(key[..., 1], dtype=np.uint64) + np.zeros_like(c[0])
    mask = np.uint64(0xFFFFFFFF)
    for r in range(10):
        p0 = np.uint64(_PHILOX_M0) * c[0]
        p1 = np.uint64(_PHILOX_M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c = [(hi1 ^ c[1] ^ k0) & mask, lo1, (hi0 ^ c[3] ^ k1) & mask, lo0]
        k0 = (k0 + np.uint64(_PHILOX_W0)) & mask
        k1 = (k1 + np.uint64(_PHILOX_W1)) & mask
    return np.stack(c, axis=-1).astype(np.uint32)


def philox_awgn_llr(codewords: np.ndarray, B: int, sigma2: float, seed: int, point: int) -> np.ndarray:
    """B frames of channel LLRs for sweep point ``point``: frame f carries codeword f mod P of the
    (P, N) pool; the noise of bit n is one Box-Muller normal from Philox4x32-10 with counter
    (n, f, point, 0) and key (seed mod 2^32, seed >> 32):  u1 = (x0 + 1) 2^-32, u2 = x1 2^-32,
    z = sqrt(-2 ln u1) cos(2 pi u2),  llr = 2 (1 - 2c + sigma z) / sigma^2.  float64 result."""
    P, N = codewords.shape
    f = np.arange(B, dtype=np.uint64)[:, None]
    n = np.arange(N, dtype=np.uint64)[None, :]
    ctr = np.zeros((B, N, 4), dtype=np.uint64)
    ctr[..., 0] = n
    ctr[..., 1] = f
    ctr[..., 2] = point
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    x = philox4x32_10(ctr, key).astype(np.float64)
    u1 = (x[..., 0] + 1.0) * 2.0 ** -32
    u2 = x[..., 1] * 2.0 ** -32
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    c = codewords[np.arange(B) % P].astype(np.float64)
    return 2.0 * ((1.0 - 2.0 * c) + np.sqrt(sigma2) * z) / sigma2


# ----------------------------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------------------------
def workload_code(name: str) -> Code:
    """c0: PEG (3,6) N=96; c1: BG1-shaped Z=52; c3: BG1-shaped Z=128; c4: PEG (3,6) N=576."""
    if name == "c0":
        return peg_regular(96, 3, 6, seed=2102)
    if name == "c1":
        return qc_bg1_shaped(52, seed=11089)
    if name == "c3":
        return qc_bg1_shaped(128, seed=11089)
    if name == "c4":
        return peg_regular(576, 3, 6, seed=576)
    raise KeyError(name)
