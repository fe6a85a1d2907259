"""Write ``c1_fer_0p5db.json``: the oracle's frame errors on seeded frames of the BG1-shaped Z = 52
code (n = 3536) at Eb/N0 0.5 dB, for CIRBP (Algorithm 1, gamma = 0.1, cap 3E, sum-product in FP64)
and for flooding and layered BP (sum-product, at most 50 iterations; Sec. I).

Test infrastructure: calls only the oracle and the seeded input generators.  The GPU test
``test_f32_c1_fer_within_oracle_interval`` regenerates the same frames and checks the GPU's frame
error count against the 95% Clopper-Pearson interval of these counts.

Usage: python tests/golden/make_c1_fer.py [threads]   (about 15 minutes on 8 cores)
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_2102_11089_amd import synth as S  # noqa: E402

FRAMES, EBN0, SEED = 3000, 0.5, 507
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_fer_0p5db.json")


def main(threads: int = 8):
    code = S.workload_code("c1")
    cw, llr = S.frames(code, FRAMES, EBN0, SEED)
    res = {"code": "BG1-shaped QC 46x68, Z=52 (workload_code('c1'))", "ebn0_db": EBN0, "frames": FRAMES,
           "seed": SEED, "generator": "synth.frames(code, frames, ebn0_db, seed)", "decoders": {}}
    for name, kind, cap in (("cirbp", O.CIRBP, 3 * code.E), ("flooding", O.FLOODING, 50 * code.E),
                            ("layered", O.LAYERED, 50 * code.E)):
        t0 = time.time()
        r = O.decode(code, llr, kind, O.SPA, max_updates=cap, gamma=0.1, threads=threads)
        err = np.flatnonzero(np.any(r.bits != cw, axis=1))
        res["decoders"][name] = {"max_updates": int(cap), "gamma": 0.1, "frame_errors": int(err.size),
                                 "error_frames": [int(x) for x in err],
                                 "mean_updates": float(r.updates_used.mean())}
        print(f"{name}: {err.size} frame errors of {FRAMES}, mean updates {r.updates_used.mean():.0f}, "
              f"{time.time() - t0:.0f} s", flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 8)
