"""One decode of a named workload, for running under a profiler (rocprofv3 --pmc / --kernel-trace).

    python -m paper_2102_11089_amd.profcase <workload> <schedule> <arith> [frames] [ebn0]
    python -m paper_2102_11089_amd.profcase copy <bytes>
    python -m paper_2102_11089_amd.profcase traffic <out.json> <kernel> <fetch.csv> <write.csv> \
        <copy_fetch.csv> <copy_write.csv> <copy_bytes> [workload text]

workload: c0 (PEG (3,6) n=96), c1 (BG1-shaped Z=52), c4 (PEG (3,6) n=576); schedule: cirbp | rbp |
flooding | layered; arith: f32 | fix.  One untimed warm-up decode, then one decode; prints the
total number of updates so counters can be divided per update.

``copy`` runs two plain device-to-device copies of a buffer of the given size: the reference for
scaling the FETCH_SIZE / WRITE_SIZE counters to bytes.

``traffic`` turns rocprofv3 counter files (``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE`` runs,
``*_counter_collection.csv``) into HBM bytes for the first dispatch whose kernel name contains
<kernel>: each counter (KiB per dispatch) is scaled by the ratio of the copy's known bytes to what
the same counter read for the largest dispatch of the copy run.  Writes a JSON document tagged
with the digest of the library sources it was measured on.
"""
import csv
import json
import sys


def first_counter(path: str, kernel: str) -> float:
    for r in csv.DictReader(open(path)):
        if kernel in r["Kernel_Name"]:
            return float(r["Counter_Value"])
    raise SystemExit(f"no dispatch of {kernel!r} in {path}")


def max_counter(path: str) -> float:
    return max(float(r["Counter_Value"]) for r in csv.DictReader(open(path)))


def traffic_case(argv):
    from .build import sources_digest
    out, kernel, fcsv, wcsv, cfcsv, cwcsv, cbytes = argv[:7]
    workload = argv[7] if len(argv) > 7 else ""
    cbytes = int(cbytes)
    f_kib, w_kib = first_counter(fcsv, kernel), first_counter(wcsv, kernel)
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


def main():
    if sys.argv[1] == "copy":
        copy_case(int(sys.argv[2]))
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
