"""One decode of a named workload, for running under a profiler (rocprofv3 --pmc / --kernel-trace).

    python -m paper_2102_11089_amd.profcase <workload> <schedule> <arith> [frames] [ebn0]
    python -m paper_2102_11089_amd.profcase copy <bytes>

workload: c0 (PEG (3,6) n=96), c1 (BG1-shaped Z=52), c4 (PEG (3,6) n=576); schedule: cirbp | rbp |
flooding | layered; arith: f32 | fix.  One untimed warm-up decode, then one decode; prints the
total number of updates so counters can be divided per update.

``copy`` runs two plain device-to-device copies of a buffer of the given size: the reference for
scaling the FETCH_SIZE / WRITE_SIZE counters to bytes.
"""
import sys

import torch

from . import ldpc
from . import synth as S


def copy_case(nbytes: int):
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
    name, sched, arith = sys.argv[1], sys.argv[2], sys.argv[3]
    B = int(sys.argv[4]) if len(sys.argv) > 4 else 1
    eb = float(sys.argv[5]) if len(sys.argv) > 5 else 1.0
    code = S.workload_code(name)
    h = ldpc.Code(code)
    kind = {"cirbp": ldpc.CIRBP, "rbp": ldpc.RBP, "flooding": ldpc.FLOODING, "layered": ldpc.LAYERED}[sched]
    a = ldpc.MS_FIX if arith == "fix" else ldpc.SPA_F32
    cap = 50 * code.E if kind in (ldpc.FLOODING, ldpc.LAYERED) else (2400 if name == "c0" else 3 * code.E)
    cw, llr = S.frames(code, B, eb, 7)
    t = torch.from_numpy(llr).cuda()
    for _ in range(2):
        r = ldpc.decode(h, t, kind, a, max_updates=cap, check_every=0 if kind in (ldpc.RBP, ldpc.CIRBP) else 1,
                        q_bits=8, frac_bits=2)
        torch.cuda.synchronize()
    print("updates", int(r.updates_used.sum()), "frames", B, flush=True)


if __name__ == "__main__":
    main()
