#!/usr/bin/env python
"""Decoded frames/s and edge-updates/s of CIRBP against flooding (and layered) BP on one MI355X.

Workload (default): the BG1-shaped 46 x 68 quasi-cyclic code with Z = 52 (n = 3536, m = 2392,
E = 16432, design rate 22/68), seeded circulant shifts; BPSK over AWGN, random codewords, FP32
channel LLRs generated on the GPU and resident in HBM before timing.  Decoders:
  CIRBP     Algorithm 1, gamma = 0.1, sum-product FP32, at most 3E updates (3 iterations);
  flooding  sum-product FP32, at most 50 iterations;
  layered   sum-product FP32, block-row layers, at most 50 iterations.
A step decodes one batch of frames; the value is CIRBP decoded frames per second over the timed
steps.  The same batches are then decoded by flooding and layered BP and reported alongside.

Prints one JSON line.  ``--sweep`` instead prints one JSON line per Eb/N0 point (FER curves).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LDS_PEAK_GBS = 256 * 128 * 2.4  # CUs x bytes/clk/CU x GHz = 78643 GB/s (nominal LDS bandwidth)
METRIC = "decoded frames/s & edge-updates/s at FER 1e-3, CI vs flooding BP, one MI355X"


def lds_bytes_per_update_table(code, s_c=4, s_v=4, s_d=4):
    """Algorithmic LDS bytes of one single-edge CIRBP update through edge e (Table 1 operation
    list): edge choice 2 s_c d_v(n*), propagation 2 s_c + 3 s_v + s_d, and for every touched check
    i in M(n*) \\ m*: d_c(i)(s_c + s_v) V2C reads, 2 s_c (d_c(i) - 1) precompute writes/reads and
    (d_c(i) - 1)(3 s_v + s_d) CI updates."""
    dc = np.diff(code.row_ptr).astype(np.int64)
    col_ptr, col_row, col_eid = code.csc()
    dv = np.diff(col_ptr).astype(np.int64)
    rows = code.row_of_edge()
    # per VN: sum over all its checks of the touched-check bytes; subtract m*'s term per edge
    per_check = dc * (s_c + s_v) + 2 * s_c * (dc - 1) + (dc - 1) * (3 * s_v + s_d)
    per_vn = np.zeros(code.N, dtype=np.int64)
    np.add.at(per_vn, code.col, per_check[rows])
    n = code.col
    return 2 * s_c * dv[n] + 2 * s_c + 3 * s_v + s_d + per_vn[n] - per_check[rows]


def make_batches(code, nb, B, ebn0, seed, device):
    """nb batches of B frames: random codewords (GF(2) encoding on the GPU) and AWGN LLRs."""
    import torch
    from paper_2102_11089_amd import synth as S
    pivots, free, A = code.generator()
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    At = torch.from_numpy(A.T.astype(np.float32)).to(device)  # K x rank
    s2 = S.sigma2_from_ebn0(ebn0, code.design_rate)
    piv = torch.from_numpy(pivots).to(device)
    fre = torch.from_numpy(free).to(device)
    out = []
    for _ in range(nb):
        info = torch.randint(0, 2, (B, len(free)), generator=g, device=device, dtype=torch.int32)
        cw = torch.zeros((B, code.N), dtype=torch.uint8, device=device)
        cw[:, fre] = info.to(torch.uint8)
        par = torch.remainder(torch.round(info.to(torch.float32) @ At), 2).to(torch.uint8)
        cw[:, piv] = par
        x = 1.0 - 2.0 * cw.to(torch.float32)
        y = x + float(np.sqrt(s2)) * torch.randn((B, code.N), generator=g, device=device)
        out.append((cw, (2.0 / s2) * y))
    return out


def check_codewords(code, cw_gpu, k=32):
    H = code.dense().astype(np.int64)
    c = cw_gpu[:k].cpu().numpy().astype(np.int64)
    assert not np.any((H @ c.T) % 2), "encoder produced a non-codeword"


def timed(fn, stream, steps):
    import torch
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    kern_ms = []
    t0 = time.perf_counter()
    for k in range(steps):
        ev0.record(stream)
        fn(k)
        ev1.record(stream)
        ev1.synchronize()
        kern_ms.append(ev0.elapsed_time(ev1))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, kern_ms


def run_decoder(ldpc, h, batches, kind, max_updates, stream, gamma=0.1):
    import torch
    res = []

    def one(k):
        cw, llr = batches[k]
        with torch.cuda.stream(stream):
            r = ldpc.decode(h, llr, kind, ldpc.SPA_F32, max_updates=max_updates, gamma=gamma, stream=stream)
        res.append((cw, r))

    return one, res


def summarize(res, code):
    import torch
    fe = 0
    nf = 0
    upd = 0
    fall = 0
    for cw, r in res:
        fe += int(torch.any(r.bits != cw, dim=1).sum())
        nf += cw.shape[0]
        upd += int(r.updates_used.sum())
        fall += int(r.fallbacks.sum())
    return fe, nf, upd, fall


def cpu_baseline(code, llr_host, cw_host, max_updates, seconds, threads):
    """The oracle (plain C, FP64, linear scans) on the host cores over a bounded sample."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    done = 0
    upd = 0
    while done < len(llr_host) and time.perf_counter() - t0 < seconds:
        chunk = llr_host[done:done + threads]
        r = O.decode(code, chunk, O.CIRBP, O.SPA, max_updates=max_updates, gamma=0.1, threads=threads)
        upd += int(r.updates_used.sum())
        done += len(chunk)
    dt = time.perf_counter() - t0
    return done, upd, dt


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--frames", type=int, default=8192, help="frames per step")
    ap.add_argument("--ebn0", type=float, default=1.25)
    ap.add_argument("--seed", type=int, default=2102)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-baselines", action="store_true")
    ap.add_argument("--sweep", type=str, default="", help="comma list of Eb/N0 points: FER curves")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark decodes on exactly one GPU; frames shard trivially "
                                   "across GPUs but no multi-GPU run is provided", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2102_11089_amd import ldpc
    from paper_2102_11089_amd import synth as S

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    code = S.workload_code("c1")
    h = ldpc.Code(code)
    E = code.E
    cap_ci = 3 * E
    cap_fl = 50 * E
    stream = torch.cuda.Stream(device=dev)

    if args.sweep:
        for eb in [float(x) for x in args.sweep.split(",")]:
            batches = make_batches(code, args.steps, args.frames, eb, args.seed + int(eb * 1000), dev)
            row = {"ebn0": eb, "frames": args.steps * args.frames}
            for name, kind, cap in (("cirbp", ldpc.CIRBP, cap_ci), ("flooding", ldpc.FLOODING, cap_fl),
                                    ("layered", ldpc.LAYERED, cap_fl), ("flooding3", ldpc.FLOODING, 3 * E),
                                    ("layered3", ldpc.LAYERED, 3 * E), ("rbp", ldpc.RBP, cap_ci)):
                one, res = run_decoder(ldpc, h, batches, kind, cap, stream)
                wall, kms = timed(one, stream, args.steps)
                fe, nf, upd, fall = summarize(res, code)
                row[name] = {"fer": fe / nf, "frame_errors": fe, "frames_per_s": nf / (sum(kms) / 1e3),
                             "edge_updates_per_s": upd / (sum(kms) / 1e3), "mean_updates": upd / nf,
                             "fallback_frac": fall / max(upd, 1)}
            print(json.dumps(row), flush=True)
        return

    nb = args.warmup + args.steps
    batches = make_batches(code, nb, args.frames, args.ebn0, args.seed, dev)
    check_codewords(code, batches[0][0])
    torch.cuda.synchronize()

    # warmup
    for name, kind, cap in (("cirbp", ldpc.CIRBP, cap_ci), ("flooding", ldpc.FLOODING, cap_fl),
                            ("layered", ldpc.LAYERED, cap_fl)):
        if name != "cirbp" and args.no_baselines:
            continue
        one, _ = run_decoder(ldpc, h, batches, kind, cap, stream)
        for k in range(args.warmup):
            one(k)
    torch.cuda.synchronize()

    timed_batches = batches[args.warmup:]
    one, res = run_decoder(ldpc, h, timed_batches, ldpc.CIRBP, cap_ci, stream)
    wall, kms = timed(one, stream, args.steps)
    fe, nf, upd, fall = summarize(res, code)
    ci_fps = nf / wall
    ms_per_step = 1e3 * wall / args.steps

    # algorithmic LDS bytes: per-update table summed over a traced decode of the first timed batch
    table = torch.from_numpy(lds_bytes_per_update_table(code)).to(dev)
    cw0, llr0 = timed_batches[0]
    tr_frames = min(2048, llr0.shape[0])
    with torch.cuda.stream(stream):
        rt = ldpc.decode(h, llr0[:tr_frames], ldpc.CIRBP, ldpc.SPA_F32, max_updates=cap_ci, gamma=0.1,
                         trace=True, stream=stream)
    torch.cuda.synchronize()
    used = rt.updates_used
    tr = rt.trace
    mask = torch.arange(tr.shape[1], device=dev)[None, :] < used[:, None]
    bytes_traced = int(table[tr.clamp(min=0).long()][mask].sum())
    bytes_per_update = bytes_traced / max(int(used.sum()), 1)
    kern_s = sum(kms) / 1e3
    achieved_gbs = bytes_per_update * upd / kern_s / 1e9 if kern_s > 0 else 0.0
    del rt, tr, mask

    out = {
        "metric": METRIC,
        "value": round(ci_fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "BG1-shaped QC LDPC 46x68, Z=52 (n=3536, m=2392, E=16432), seeded shifts; BPSK/AWGN "
                        f"Eb/N0 {args.ebn0} dB, random codewords; CIRBP gamma=0.1 sum-product FP32, cap 3E",
            "frames_per_step": args.frames,
            "ebn0_db": args.ebn0,
        },
        "ci": {"fer": fe / nf, "frame_errors": fe, "frames": nf, "frames_per_s": round(ci_fps, 3),
               "edge_updates_per_s": round(upd / wall, 1), "mean_updates_per_frame": upd / nf,
               "fallback_fraction": fall / max(upd, 1), "kernel_ms_per_step": [round(x, 3) for x in kms]},
        "roofline": {"bound": "lds", "achieved": round(achieved_gbs, 2), "peak": LDS_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved_gbs / LDS_PEAK_GBS, 6), "traffic": None,
                     "kernel": "k_dynamic<ArithF32, pre in global scratch>",
                     "bytes_per_update": round(bytes_per_update, 2),
                     "kernel_ms_avg": round(float(np.mean(kms)), 3)},
    }

    if not args.no_baselines:
        for name, kind in (("flooding", ldpc.FLOODING), ("layered", ldpc.LAYERED)):
            one, res_b = run_decoder(ldpc, h, timed_batches, kind, cap_fl, stream)
            wall_b, kms_b = timed(one, stream, args.steps)
            fe_b, nf_b, upd_b, _ = summarize(res_b, code)
            out[name] = {"fer": fe_b / nf_b, "frame_errors": fe_b, "frames_per_s": round(nf_b / wall_b, 3),
                         "edge_updates_per_s": round(upd_b / wall_b, 1),
                         "mean_iterations": upd_b / nf_b / E, "cap_iterations": 50}
        out["ci_over_flooding_frames_per_s"] = round(ci_fps / out["flooding"]["frames_per_s"], 5)

    if not args.no_cpu:
        threads = max(1, min(16, os.cpu_count() or 1))
        cw_h = timed_batches[0][0].cpu().numpy()
        llr_h = timed_batches[0][1][:512].cpu().numpy().astype(np.float64)
        nf_c, upd_c, dt_c = cpu_baseline(code, llr_h, cw_h, cap_ci, args.cpu_seconds, threads)
        out["cpu_baseline"] = {"value": round(nf_c / dt_c, 4), "unit": "frames/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"first {nf_c} frames of the first timed batch, CIRBP gamma=0.1 cap 3E, "
                                         f"FP64, {threads} threads, {dt_c:.1f} s",
                               "edge_updates_per_s": round(upd_c / dt_c, 1)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
