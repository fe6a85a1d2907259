"""Decodes run by tests/test_gpu_selfcheck.py with the self-checking library (argument: its path).
After every single-edge update the kernels recompute the touched neighbourhood's derived state
from its definition and count mismatches per kind into the buffer LDPCCI_SELFCHECK points to.
Prints one JSON line per case: name, counts (L, Lt, D, check key, VN block, check block, -, updates
checked) and the updates the decode made."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import numpy as np  # noqa: E402
import torch  # noqa: E402

from paper_2102_11089_amd import ldpc  # noqa: E402
from paper_2102_11089_amd import synth as S  # noqa: E402


def many_four_cycles_code():
    from test_gpu_parity import many_four_cycles_code as f
    return f()


def main():
    ldpc.load(sys.argv[1])
    counts = torch.zeros(8, dtype=torch.int64, device="cuda")
    os.environ["LDPCCI_SELFCHECK"] = str(counts.data_ptr())
    kinds = {"cirbp": ldpc.CIRBP, "rbp": ldpc.RBP, "lmdcirbp": ldpc.LMD_CIRBP, "lmdrbp": ldpc.LMDRBP,
             "slmdrbp": ldpc.SLMDRBP}
    stores = {"lds": ldpc.STORE_LDS, "all": ldpc.STORE_GLOBAL_ALL, "frame": ldpc.STORE_GLOBAL_FRAME,
              "rec": ldpc.STORE_GLOBAL_REC, "state": ldpc.STORE_GLOBAL_STATE}
    cases = []
    c0 = S.workload_code("c0")
    for arith in ("fix", "f32"):
        for kn in kinds:
            for st in ("lds", "rec", "state"):
                cases.append((f"c0 {kn} {arith} {st}", c0, kn, arith, st, 64, 2.0, 2400))
    qc = S.qc_24col(24, 12, seed=4)
    for st in stores:
        cases.append((f"qc24 cirbp fix {st}", qc, "cirbp", "fix", st, 64, 2.0, 1500))
    cases.append(("bg1 z4 cirbp fix rec (degree-1 VNs)", S.qc_bg1_shaped(4, seed=3), "cirbp", "fix", "rec", 64, 1.0,
                  3 * S.qc_bg1_shaped(4, seed=3).E))
    cases.append(("overlap32 cirbp fix rec (repeated VNs)", many_four_cycles_code(), "cirbp", "fix", "rec", 64, 1.0, 400))
    cases.append(("overlap32 cirbp f32 lds (repeated VNs)", many_four_cycles_code(), "cirbp", "f32", "lds", 64, 1.0, 400))
    c1 = S.workload_code("c1")
    cases.append(("c1 cirbp f32 default plan", c1, "cirbp", "f32", None, 16, 1.25, 3 * c1.E))
    cases.append(("c1 lmdcirbp f32 default plan", c1, "lmdcirbp", "f32", None, 16, 1.25, 3 * c1.E))
    for name, code, kn, arith, st, B, eb, cap in cases:
        h = ldpc.Code(code)
        a = ldpc.MS_FIX if arith == "fix" else ldpc.SPA_F32
        if st is not None:
            ldpc.set_tuning(h, kinds[kn], a, storage=stores[st], frames_per_cu=2)
        _, llr = S.frames(code, B, eb, 7)
        counts.zero_()
        r = ldpc.decode(h, torch.from_numpy(llr).cuda(), kinds[kn], a, max_updates=cap, q_bits=8, frac_bits=2)
        torch.cuda.synchronize()
        print(json.dumps({"case": name, "counts": counts.cpu().tolist(),
                          "updates": int(r.updates_used.sum())}), flush=True)
        if st is not None:
            ldpc.set_tuning(h, kinds[kn], a, clear=True)
    print("selfcheck cases done", flush=True)


if __name__ == "__main__":
    main()
