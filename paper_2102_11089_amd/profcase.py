"""One decode of a named workload, for running under a profiler (rocprofv3 --pmc / --kernel-trace).

    python -m paper_2102_11089_amd.profcase <workload> <schedule> <arith> [frames] [ebn0]
    python -m paper_2102_11089_amd.profcase copy <bytes>
    python -m paper_2102_11089_amd.profcase random <bytes> <accesses> [width bytes]
    python -m paper_2102_11089_amd.profcase account [frames] [sector bytes]
    python -m paper_2102_11089_amd.profcase phase <profile library> c1|c3
    python -m paper_2102_11089_amd.profcase traffic <out.json> <kernel> <fetch.csv> <write.csv> \
        <copy_fetch.csv> <copy_write.csv> <copy_bytes> [workload text] [first|last]

workload: c0 (PEG (3,6) n=96), c1 (BG1-shaped Z=52), c4 (PEG (3,6) n=576); schedule: cirbp | rbp |
flooding | layered; arith: f32 | fix.  One untimed warm-up decode, then one decode; prints the
total number of updates so counters can be divided per update.

``copy`` runs two plain device-to-device copies of a buffer of the given size: the reference for
scaling the FETCH_SIZE / WRITE_SIZE counters to bytes.

``random`` measures scattered 8-byte gathers and scatters over a buffer of the given size: the
memory system's rate for the decoder's scattered record accesses.

``account`` counts, per single-edge update of a traced c1 decode, the memory sectors each part of
the frame state costs in the benchmark's layout (pairs, VN records, two-hop table).

``phase`` loads the phase-timing build (``python -m paper_2102_11089_amd.build profile``) and
prints the cycles per update (c1: FP32 CIRBP, 65536 frames at 1.25 dB, 256 distinct) or per step
(c3: ME-CIRBP and ME-LMD-CIRBP at N_P 8 and 64, 8192 frames at 1.5 dB, 256 distinct) that each phase takes, summed over the
wavefronts (c1) or over thread 0 of each workgroup (c3).

``traffic`` turns rocprofv3 counter files (``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE`` runs,
``*_counter_collection.csv``) into HBM bytes for the first (default) or last dispatch whose kernel
name contains <kernel>: each counter (KiB per dispatch) is scaled by the ratio of the copy's known bytes to what
the same counter read for the largest dispatch of the copy run.  Writes a JSON document tagged
with the digest of the library sources it was measured on.
"""
import csv
import json
import sys


def first_counter(path: str, kernel: str, which: str = "first") -> float:
    """The counter of the first (or last) dispatch whose kernel name contains `kernel`."""
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path)) if kernel in r["Kernel_Name"]]
    if not vals:
        raise SystemExit(f"no dispatch of {kernel!r} in {path}")
    return vals[-1] if which == "last" else vals[0]


def max_counter(path: str) -> float:
    return max(float(r["Counter_Value"]) for r in csv.DictReader(open(path)))


def traffic_case(argv):
    from .build import sources_digest
    out, kernel, fcsv, wcsv, cfcsv, cwcsv, cbytes = argv[:7]
    workload = argv[7] if len(argv) > 7 else ""
    which = argv[8] if len(argv) > 8 else "first"
    cbytes = int(cbytes)
    f_kib, w_kib = first_counter(fcsv, kernel, which), first_counter(wcsv, kernel, which)
    cf_kib, cw_kib = max_counter(cfcsv), max_counter(cwcsv)
    fs, ws = cbytes / (cf_kib * 1024.0), cbytes / (cw_kib * 1024.0)
    doc = {"kernel": kernel, "workload": workload,
           "fetch_kib_per_launch": f_kib, "write_kib_per_launch": w_kib,
           "copy_bytes": cbytes, "copy_fetch_kib": cf_kib, "copy_write_kib": cw_kib,
           "fetch_scale": round(fs, 6), "write_scale": round(ws, 6),
           "traffic_bytes_per_launch": int(round(f_kib * 1024.0 * fs + w_kib * 1024.0 * ws)),
           "kernel_sources_sha256": sources_digest()}
    with open(out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(json.dumps(doc), flush=True)


def copy_case(nbytes: int):
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copied bytes", src.numel() * 4, "twice", flush=True)


def random_case(nbytes: int, accesses: int, width: int = 8):
    """Throughput of scattered accesses of `width` bytes (aligned to their size) over a buffer of
    nbytes in device memory (width 8: the access pattern of the decoder's VN records, each in its
    own sector): a gather of `accesses` random elements, a scatter of as many, and a copy of the
    same index/value volume for comparison.  Prints accesses per second and the 64-byte sector
    rate of each."""
    import time
    import torch
    w = max(1, width // 8)
    n = nbytes // (8 * w)
    buf = torch.zeros((n, w), dtype=torch.float64, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    idx = torch.randint(0, n, (accesses,), generator=g, device="cuda")
    vals = torch.ones((accesses, w), dtype=torch.float64, device="cuda")
    out = torch.empty_like(vals)

    def timeit(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t
    tg = timeit(lambda: torch.index_select(buf, 0, idx, out=out))
    ts = timeit(lambda: buf.index_copy_(0, idx, vals))
    tc = timeit(lambda: out.copy_(vals))
    for name, t in (("gather", tg), ("scatter", ts)):
        print(f"{name} of {8 * w} B: {accesses / t / 1e9:.2f} G accesses/s ({accesses * 8 * w / t / 1e12:.2f} TB/s of "
              f"payload; plus {accesses * (8 + 8 * w) / t / 1e12:.2f} TB/s sequential index and value streams)",
              flush=True)
    print(f"copy of the value stream: {accesses * 16 * w / tc / 1e12:.2f} TB/s", flush=True)


def account_case(frames: int, sector: int = 64):
    """Per-update memory accounting of the single-edge kernel on the BG1-shaped Z=52 code: decode
    `frames` frames at 1.25 dB with CIRBP (FP32, cap 3E) with the schedule recorded, and for every
    update count the distinct `sector`-byte sectors of the frame state it touches in the layout of
    the benchmark's plan (a global slot per frame: (c2v, pre) pairs in row order, then one 8-byte
    (Lt, L) record per VN): the pairs of every check of n*, the records of n* and of every VN of
    M(n*) \ m*, and the two-hop table entries of n* (shared by all frames).  Counts assume no reuse
    between updates; the block recomputations (64 records each) are counted separately."""
    import numpy as np
    import torch
    from . import ldpc
    from . import synth as S
    code = S.workload_code("c1")
    E, N = code.E, code.N
    rp = np.asarray(code.row_ptr)
    col = np.asarray(code.col)
    col_ptr, col_row, _ = code.csc()
    row_of = np.repeat(np.arange(code.M), np.diff(rp))
    dc = np.diff(rp)
    up = lambda x: (x + 255) // 256 * 256  # noqa: E731
    rec0 = up(2 * E * 4)
    p2 = lambda x: 1 << int(np.ceil(np.log2(x)))  # noqa: E731
    ncnt = np.array([sum(p2(dc[m]) for m in col_row[col_ptr[n]:col_ptr[n + 1]]) for n in range(N)])
    nbr_off = np.concatenate([[0], np.cumsum(ncnt)])[:-1]

    def secs(lo, hi):
        return set(range(lo // sector, (hi - 1) // sector + 1))
    pairs = np.zeros(E)
    recs = np.zeros(E)
    vns = np.zeros(E)
    table = np.zeros(E)
    for e in range(E):
        m, n = row_of[e], col[e]
        checks = col_row[col_ptr[n]:col_ptr[n + 1]]
        ps, touched = set(), {int(n)}
        for i in checks:
            ps |= secs(8 * rp[i], 8 * rp[i + 1])
            if i != m:
                touched |= set(col[rp[i]:rp[i + 1]].tolist())
        rs = set()
        for j in touched:
            rs |= secs(rec0 + 8 * j, rec0 + 8 * j + 8)
        pairs[e], recs[e], vns[e] = len(ps), len(rs), len(touched)
        table[e] = len(secs(8 * nbr_off[n], 8 * (nbr_off[n] + ncnt[n]))) if len(checks) > 1 else 0
    h = ldpc.Code(code)
    _, llr = S.frames(code, frames, 1.25, 7)
    r = ldpc.decode(h, torch.from_numpy(llr).cuda(), ldpc.CIRBP, ldpc.SPA_F32, max_updates=3 * E, gamma=0.1,
                    trace=True)
    torch.cuda.synchronize()
    used = r.updates_used.cpu().numpy()
    tr = r.trace.cpu().numpy()
    t = np.concatenate([tr[f, :used[f]] for f in range(frames)])
    doc = {"frames": frames, "updates": int(len(t)), "sector_bytes": sector,
           "pair_sectors": round(float(pairs[t].mean()), 2), "record_sectors": round(float(recs[t].mean()), 2),
           "touched_vns": round(float(vns[t].mean()), 2), "table_sectors": round(float(table[t].mean()), 2),
           "rows_of_nstar": round(float(np.diff(col_ptr)[col[t]].mean()), 2),
           "degree1_nstar_fraction": round(float((np.diff(col_ptr)[col[t]] == 1).mean()), 4)}
    print(json.dumps(doc), flush=True)


def phase_case(lib: str, which: str):
    """Per-phase cycle sums of the phase-timing build (see the module docstring)."""
    import os
    import numpy as np
    import torch
    from . import ldpc
    from . import synth as S
    ldpc.load(lib)
    prof = torch.zeros(16, dtype=torch.int64, device="cuda")
    if which == "c1":
        code = S.workload_code("c1")
        h = ldpc.Code(code)
        _, llr = S.frames(code, 256, 1.25, 7)
        x = torch.from_numpy(llr).cuda().repeat(256, 1)  # 65536 frames, 256 distinct
        for it in range(2):
            prof.zero_()
            os.environ["LDPCCI_PROF"] = str(prof.data_ptr()) if it == 1 else "0"
            r = ldpc.decode(h, x, ldpc.CIRBP, ldpc.SPA_F32, max_updates=3 * code.E, gamma=0.1)
            torch.cuda.synchronize()
        upd = int(r.updates_used.sum())
        p = prof.cpu().numpy().astype(np.float64)
        names = {7: "loop top", 0: "selection", 1: "propagation", 3: "passes", 5: "groups and late CI",
                 6: "block recomputation"}
        tot = p[:8].sum()
        for i in (7, 0, 1, 3, 5, 6):
            print(f"{names[i]:22s} {p[i] / upd:9.0f} cycles per update {100 * p[i] / tot:5.1f}%", flush=True)
        print(f"total {tot / upd:.0f} cycles per update per wavefront", flush=True)
        return
    code = S.workload_code("c3")
    h = ldpc.Code(code)
    B = 8192
    _, llr = S.frames(code, 256, 1.5, 7)
    x = torch.from_numpy(llr).cuda().repeat(B // 256, 1)  # 8192 frames, 256 distinct
    names = {7: "loop top", 0: "P' and group pass", 1: "fill (list or radix)", 2: "edge choice, propagation",
             3: "sort of touched checks", 4: "touched checks' rows", 5: "CI pass", 6: "Algorithm 6 proposals"}
    for kind, kn in ((ldpc.ME_CIRBP, "ME-CIRBP"), (ldpc.ME_LMD_CIRBP, "ME-LMD-CIRBP")):
        for n_p in (8, 64):
            for it in range(2):
                prof.zero_()
                os.environ["LDPCCI_PROF"] = str(prof.data_ptr()) if it == 1 else "0"
                r = ldpc.decode(h, x, kind, ldpc.SPA_F32, max_updates=3 * code.E, gamma=0.1, n_p=n_p, n_g=16,
                                fill=ldpc.FILL_HASH, seed=2102)
                torch.cuda.synchronize()
            steps = int(r.steps_used.sum())
            p = prof.cpu().numpy().astype(np.float64)
            tot = p[:8].sum()
            print(f"{kn} N_P {n_p}: {steps / B:.0f} steps per frame, {tot / steps:.0f} cycles per step", flush=True)
            for i in (7, 0, 1, 2, 3, 4, 5, 6):
                print(f"   {names[i]:26s} {p[i] / steps:8.0f} cycles per step {100 * p[i] / tot:5.1f}%", flush=True)


def main():
    if sys.argv[1] == "phase":
        phase_case(sys.argv[2], sys.argv[3])
        return
    if sys.argv[1] == "account":
        account_case(int(sys.argv[2]) if len(sys.argv) > 2 else 16, int(sys.argv[3]) if len(sys.argv) > 3 else 64)
        return
    if sys.argv[1] == "copy":
        copy_case(int(sys.argv[2]))
        return
    if sys.argv[1] == "random":
        random_case(int(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4]) if len(sys.argv) > 4 else 8)
        return
    if sys.argv[1] == "traffic":
        traffic_case(sys.argv[2:])
        return
    import torch
    from . import ldpc
    from . import synth as S
    name, sched, arith = sys.argv[1], sys.argv[2], sys.argv[3]
    B = int(sys.argv[4]) if len(sys.argv) > 4 else 1
    eb = float(sys.argv[5]) if len(sys.argv) > 5 else 1.0
    code = S.workload_code(name)
    h = ldpc.Code(code)
    kind = {"cirbp": ldpc.CIRBP, "rbp": ldpc.RBP, "flooding": ldpc.FLOODING, "layered": ldpc.LAYERED,
            "lmdcirbp": ldpc.LMD_CIRBP, "lmdrbp": ldpc.LMDRBP, "slmdrbp": ldpc.SLMDRBP}[sched]
    a = ldpc.MS_FIX if arith == "fix" else ldpc.SPA_F32
    cap = 50 * code.E if kind in (ldpc.FLOODING, ldpc.LAYERED) else (2400 if name == "c0" else 3 * code.E)
    cw, llr = S.frames(code, B, eb, 7)
    t = torch.from_numpy(llr).cuda()
    for _ in range(2):
        dyn = kind not in (ldpc.FLOODING, ldpc.LAYERED)
        r = ldpc.decode(h, t, kind, a, max_updates=cap, check_every=0 if dyn else 1, q_bits=8, frac_bits=2)
        torch.cuda.synchronize()
    print("updates", int(r.updates_used.sum()), "frames", B, flush=True)


if __name__ == "__main__":
    main()
