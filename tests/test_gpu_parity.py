"""GPU parity: the HIP decoder (through the C ABI) against the CPU oracle on the same seeded inputs.

* fixed-point min-sum: bit-exact (decoded bits, recorded schedule, updates used, fallbacks, and the
  final c2v / pre / L / Lt / D state);
* FP32 sum-product: replay of the oracle's recorded schedule, every message within
  |gpu - oracle| <= 1e-4 max(|oracle|, 1) (CI within 1e-4 absolute), and free-running frame
  error rates within the oracle's 95% Clopper-Pearson interval.
"""
import numpy as np
import pytest
import torch
from scipy.stats import beta

from oracle import oracle as O
from paper_2102_11089_amd import synth as S

pytestmark = pytest.mark.gpu

KIND = {"flooding": (O.FLOODING, 0), "layered": (O.LAYERED, 1), "rbp": (O.RBP, 2), "cirbp": (O.CIRBP, 3),
        "me": (O.MECIRBP, 4), "replay": (O.REPLAY, 5)}


def say(*a):
    print(*a, flush=True)


def gpu_decode(ldpc, code_h, llr, kind, arith, **kw):
    t = torch.from_numpy(np.ascontiguousarray(llr, dtype=np.float32)).cuda()
    r = ldpc.decode(code_h, t, KIND[kind][1], arith, **kw)
    torch.cuda.synchronize()
    return r


def np_(t):
    return None if t is None else t.cpu().numpy()


def cp_interval(k, n, a=0.05):
    lo = 0.0 if k == 0 else beta.ppf(a / 2, k, n - k + 1)
    hi = 1.0 if k == n else beta.ppf(1 - a / 2, k + 1, n - k)
    return lo, hi


@pytest.fixture(scope="module")
def c0(gpu):
    code = S.workload_code("c0")
    return code, gpu.Code(code)


# ------------------------------------------------------------------------------------------
# fixed point: bit-exact
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["rbp", "cirbp"])
def test_fixed_dynamic_bit_exact_c0(gpu, c0, kind):
    code, ch = c0
    cw, llr = S.frames(code, 1000, 2.0, 100)
    mu = 2400
    say(f"[fixed {kind}] c0 1000 frames, cap {mu}")
    ref = O.decode(code, llr, KIND[kind][0], O.MSFIX, max_updates=mu, gamma=0.1, q_bits=6, frac_bits=1,
                   trace=True, dump=True, threads=8)
    g = gpu_decode(gpu, ch, llr, kind, gpu.MS_FIX, max_updates=mu, gamma=0.1, q_bits=6, frac_bits=1,
                   trace=True, dump=True)
    np.testing.assert_array_equal(np_(g.updates_used), ref.updates_used)
    np.testing.assert_array_equal(np_(g.trace), ref.trace)
    np.testing.assert_array_equal(np_(g.bits), ref.bits)
    np.testing.assert_array_equal(np_(g.llr_out), ref.llr_out.astype(np.float32))
    np.testing.assert_array_equal(np_(g.c2v), ref.c2v)
    np.testing.assert_array_equal(np_(g.pre), ref.pre)
    np.testing.assert_array_equal(np_(g.L), ref.L)
    if kind == "cirbp":
        np.testing.assert_array_equal(np_(g.Lt), ref.Lt)
        np.testing.assert_array_equal(np_(g.D), ref.D)
        np.testing.assert_array_equal(np_(g.fallbacks), ref.counter("fallback"))


@pytest.mark.parametrize("kind", ["flooding", "layered"])
def test_fixed_baselines_bit_exact_c0(gpu, c0, kind):
    code, ch = c0
    cw, llr = S.frames(code, 1000, 2.0, 101)
    mu = 50 * code.E
    say(f"[fixed {kind}] c0 1000 frames")
    ref = O.decode(code, llr, KIND[kind][0], O.MSFIX, max_updates=mu, q_bits=6, frac_bits=1, threads=8)
    g = gpu_decode(gpu, ch, llr, kind, gpu.MS_FIX, max_updates=mu, q_bits=6, frac_bits=1)
    np.testing.assert_array_equal(np_(g.updates_used), ref.updates_used)
    np.testing.assert_array_equal(np_(g.bits), ref.bits)
    np.testing.assert_array_equal(np_(g.llr_out), ref.llr_out.astype(np.float32))


def test_fixed_tie_heavy_inputs(gpu):
    """Many exact ties: integer channel values from a tiny alphabet, exact zeros included; ragged
    code size (N = 200: four VN blocks, the last one partial)."""
    code = S.peg_regular(200, 3, 6, seed=3)
    ch = gpu.Code(code)
    rng = np.random.default_rng(5)
    llr = rng.choice([-1.0, -0.5, 0.0, 0.5, 1.0, 1.5], size=(300, code.N)).astype(np.float32)
    for kind in ("cirbp", "rbp"):
        say(f"[fixed ties {kind}] N=200")
        ref = O.decode(code, llr, KIND[kind][0], O.MSFIX, max_updates=700, gamma=0.05, trace=True, threads=8)
        g = gpu_decode(gpu, ch, llr, kind, gpu.MS_FIX, max_updates=700, gamma=0.05, trace=True)
        np.testing.assert_array_equal(np_(g.trace), ref.trace)
        np.testing.assert_array_equal(np_(g.updates_used), ref.updates_used)
        np.testing.assert_array_equal(np_(g.bits), ref.bits)


def test_fixed_8bit_and_check_every(gpu, c0):
    code, ch = c0
    cw, llr = S.frames(code, 400, 1.5, 102)
    for ce in (0, code.E):
        say(f"[fixed q8 f2 check_every={ce}]")
        ref = O.decode(code, llr, O.CIRBP, O.MSFIX, max_updates=1000, q_bits=8, frac_bits=2, check_every=ce,
                       trace=True, threads=8)
        g = gpu_decode(gpu, ch, llr, "cirbp", gpu.MS_FIX, max_updates=1000, q_bits=8, frac_bits=2,
                       check_every=ce, trace=True)
        np.testing.assert_array_equal(np_(g.trace), ref.trace)
        np.testing.assert_array_equal(np_(g.updates_used), ref.updates_used)
        np.testing.assert_array_equal(np_(g.bits), ref.bits)


def test_fixed_bg1_shaped_full_size_sampled(gpu):
    """The Z=52 BG1-shaped code at full size (state larger than one workgroup's LDS in FP32, here
    fixed point): a few frames, bit-exact."""
    code = S.workload_code("c1")
    ch = gpu.Code(code)
    cw, llr = S.frames(code, 4, 1.25, 103)
    say("[fixed cirbp] c1 4 frames, cap 3000")
    ref = O.decode(code, llr, O.CIRBP, O.MSFIX, max_updates=3000, q_bits=8, frac_bits=2, trace=True, threads=4)
    g = gpu_decode(gpu, ch, llr, "cirbp", gpu.MS_FIX, max_updates=3000, q_bits=8, frac_bits=2, trace=True)
    np.testing.assert_array_equal(np_(g.trace), ref.trace)
    np.testing.assert_array_equal(np_(g.bits), ref.bits)
    say("[fixed layered] c1 16 frames")
    ref = O.decode(code, llr, O.LAYERED, O.MSFIX, max_updates=20 * code.E, q_bits=8, frac_bits=2, threads=4)
    g = gpu_decode(gpu, ch, llr, "layered", gpu.MS_FIX, max_updates=20 * code.E, q_bits=8, frac_bits=2)
    np.testing.assert_array_equal(np_(g.bits), ref.bits)
    np.testing.assert_array_equal(np_(g.updates_used), ref.updates_used)


# ------------------------------------------------------------------------------------------
# FP32: replay tolerance and frame-error-rate interval
# ------------------------------------------------------------------------------------------
def assert_close_msgs(g, ref, what):
    a, b = np_(g), ref
    tol = 1e-4 * np.maximum(np.abs(b), 1.0)
    bad = np.abs(a - b) > tol
    assert not bad.any(), f"{what}: {bad.sum()} of {bad.size} beyond tolerance, max err {np.abs(a - b).max()}"


@pytest.mark.parametrize("name,ntr", [("c0", 400), ("c4", 600)])
def test_f32_replay_within_tolerance(gpu, name, ntr):
    code = S.workload_code(name)
    ch = gpu.Code(code)
    cw, llr = S.frames(code, 64, 2.0, 104)
    say(f"[f32 replay] {name} 64 frames, {ntr} updates")
    rec = O.decode(code, llr, O.CIRBP, O.SPA, max_updates=ntr, check_every=0, trace=True, threads=8)
    ref = O.decode(code, llr, O.REPLAY, O.SPA, max_updates=ntr, replay=rec.trace, dump=True, threads=8)
    g = gpu_decode(gpu, ch, llr, "replay", gpu.SPA_F32, max_updates=ntr, replay=torch.from_numpy(rec.trace),
                   dump=True)
    np.testing.assert_array_equal(np_(g.updates_used), ref.updates_used)
    assert_close_msgs(g.c2v, ref.c2v, "c2v")
    assert_close_msgs(g.pre, ref.pre, "pre")
    assert_close_msgs(g.L, ref.L, "L")
    assert_close_msgs(g.Lt, ref.Lt, "Lt")
    assert np.abs(np_(g.D) - ref.D).max() <= 1e-4


@pytest.mark.parametrize("kind", ["cirbp", "rbp", "flooding", "layered"])
def test_f32_fer_within_interval_c0(gpu, c0, kind):
    code, ch = c0
    cw, llr = S.frames(code, 1000, 2.0, 105)
    mu = 50 * code.E if kind in ("flooding", "layered") else 2400
    say(f"[f32 FER {kind}] c0 1000 frames")
    ref = O.decode(code, llr, KIND[kind][0], O.SPA, max_updates=mu, threads=8)
    g = gpu_decode(gpu, ch, llr, kind, gpu.SPA_F32, max_updates=mu)
    k_ref = int(np.any(ref.bits != cw, axis=1).sum())
    k_gpu = int(np.any(np_(g.bits) != cw, axis=1).sum())
    lo, hi = cp_interval(k_ref, 1000)
    assert lo <= k_gpu / 1000 <= hi, (k_gpu, k_ref, lo, hi)
    # most frames take exactly the same number of updates
    assert np.mean(np_(g.updates_used) == ref.updates_used) > 0.8


@pytest.fixture(scope="module")
def c1_full_length_traces():
    """CIRBP schedules the oracle records on frames of the BG1-shaped Z=52 code at 1.25 dB (cap 3E,
    stop on a valid codeword): the three longest of 24 frames and a median one, each to the update
    where it stopped, and the oracle's replay of them with the final state."""
    code = S.workload_code("c1")
    cw, llr = S.frames(code, 24, 1.25, 106)
    cap = 3 * code.E
    say("[f32 replay] c1: oracle CIRBP on 24 frames (full length)")
    rec = O.decode(code, llr, O.CIRBP, O.SPA, max_updates=cap, gamma=0.1, trace=True, threads=8)
    order = np.argsort(rec.updates_used, kind="stable")
    pick = [int(x) for x in order[-3:]] + [int(order[len(order) // 2])]
    say(f"[f32 replay] c1: frames {pick}, updates {rec.updates_used[pick].tolist()}")
    tr = rec.trace[pick]
    ref = O.decode(code, llr[pick], O.REPLAY, O.SPA, max_updates=cap, replay=tr, dump=True, threads=4)
    assert np.array_equal(ref.updates_used, rec.updates_used[pick])
    return code, llr[pick], tr, ref


@pytest.mark.parametrize("plan", ["default", "benchmark"])
def test_f32_bg1_shaped_full_length_replay(gpu, c1_full_length_traces, plan):
    """Z=52 BG1-shaped code: the oracle's CIRBP schedules replayed to their full length (every
    update the frame made, up to 3E), in the plan a 4-frame decode gets and in the plan the
    benchmark's 65536-frame launch uses (VN records in global memory, QC tables in LDS, 14 frames
    per workgroup): every c2v, pre, L and Lt within 1e-4 max(|oracle|, 1), every CI within 1e-4."""
    code, llr, tr, ref = c1_full_length_traces
    ch = gpu.Code(code)
    cap = 3 * code.E
    if plan == "benchmark":
        gpu.set_tuning(ch, gpu.REPLAY, gpu.SPA_F32, block=14 * 64, storage=gpu.STORE_GLOBAL_REC,
                       topology=gpu.TOPO_QC)
    try:
        pl = gpu.describe_plan(ch, llr.shape[0], gpu.REPLAY)
        say(f"[f32 replay] c1 {plan} plan {pl}")
        if plan == "benchmark":
            bench = gpu.describe_plan(ch, 65536, gpu.CIRBP)
            for k in ("storage", "topology", "block", "frames_per_workgroup"):
                assert pl[k] == bench[k], (k, pl, bench)
        g = gpu_decode(gpu, ch, llr, "replay", gpu.SPA_F32, max_updates=cap, replay=torch.from_numpy(tr),
                       dump=True)
    finally:
        if plan == "benchmark":
            gpu.set_tuning(ch, gpu.REPLAY, gpu.SPA_F32, clear=True)
    assert np.array_equal(np_(g.updates_used), ref.updates_used)
    assert_close_msgs(g.c2v, ref.c2v, "c2v")
    assert_close_msgs(g.pre, ref.pre, "pre")
    assert_close_msgs(g.L, ref.L, "L")
    assert_close_msgs(g.Lt, ref.Lt, "Lt")
    assert np.abs(np_(g.D) - ref.D).max() <= 1e-4
    sure = np.abs(ref.L) > 1e-3  # hard decisions of totals away from zero
    assert np.array_equal(np_(g.bits)[sure], ref.bits[sure])


def test_f32_c1_fer_within_oracle_interval(gpu):
    """Free-running FP32 decodes of the BG1-shaped Z=52 code at 0.5 dB (3000 seeded frames):
    CIRBP (cap 3E), flooding and layered BP (50 iterations) each have frame errors inside the 95%
    Clopper-Pearson interval of the oracle's on the same frames.  The oracle's counts are stored in
    tests/golden/c1_fer_0p5db.json by tests/golden/make_c1_fer.py (oracle and input generators
    only)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "c1_fer_0p5db.json")) as fh:
        gold = json.load(fh)
    code = S.workload_code("c1")
    ch = gpu.Code(code)
    n = gold["frames"]
    cw, llr = S.frames(code, n, gold["ebn0_db"], gold["seed"])
    t = torch.from_numpy(llr).cuda()
    kinds = {"cirbp": gpu.CIRBP, "flooding": gpu.FLOODING, "layered": gpu.LAYERED}
    for name, d in gold["decoders"].items():
        r = gpu.decode(ch, t, kinds[name], gpu.SPA_F32, max_updates=d["max_updates"], gamma=d["gamma"])
        torch.cuda.synchronize()
        err = np.flatnonzero(np.any(np_(r.bits) != cw, axis=1))
        k_ref = d["frame_errors"]
        both = len(set(err.tolist()) & set(d["error_frames"]))
        lo, hi = cp_interval(k_ref, n)
        say(f"[c1 FER {name}] gpu {err.size}, oracle {k_ref} of {n} (both {both}); mean updates gpu "
            f"{np_(r.updates_used).mean():.0f}, oracle {d['mean_updates']:.0f}")
        assert lo <= err.size / n <= hi, (name, err.size, k_ref, lo, hi)


def _syndrome_weights(code, bits):
    """Unsatisfied checks per frame of a (B, N) uint8 CUDA tensor (torch index ops)."""
    col = torch.from_numpy(np.asarray(code.col, dtype=np.int64)).cuda()
    row_of = torch.from_numpy(np.repeat(np.arange(code.M), np.diff(np.asarray(code.row_ptr)))).cuda()
    out = []
    for s0 in range(0, bits.shape[0], 4096):
        b = bits[s0:s0 + 4096].to(torch.int32)
        acc = torch.zeros((b.shape[0], code.M), dtype=torch.int32, device=b.device)
        acc.index_add_(1, row_of, b[:, col])
        out.append((acc % 2).sum(1))
    return torch.cat(out).cpu().numpy()


@pytest.mark.parametrize("kind", ["cirbp", "lmdcirbp", "lmdrbp", "slmdrbp"])
def test_f32_benchmark_launch_sampled_frames(gpu, kind):
    """The launch the benchmark times: 65536 frames of the Z=52 BG1-shaped code at 1.25 dB, FP32,
    cap 3E, default plan.  Sampled frames (and the longest) give the outputs they give when decoded
    alone, in another plan whose FP32 replay the oracle checks above; every frame that stopped
    before the cap satisfies all parity checks."""
    code = S.workload_code("c1")
    ch = gpu.Code(code)
    k = {"cirbp": gpu.CIRBP, "lmdcirbp": gpu.LMD_CIRBP, "lmdrbp": gpu.LMDRBP, "slmdrbp": gpu.SLMDRBP}[kind]
    B, cap = 65536, 3 * code.E
    say(f"[benchmark launch {kind}] plan {gpu.describe_plan(ch, B, k)}")
    say(f"[benchmark launch {kind}] single-frame plan {gpu.describe_plan(ch, 1, k)}")
    cw = torch.from_numpy(S.random_codewords(code, 256, 11)).cuda().repeat(B // 256, 1)
    s2 = S.sigma2_from_ebn0(1.25, code.design_rate)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2102)
    noise = torch.randn(tuple(cw.shape), generator=gen, device="cuda")
    llr = (2.0 / s2) * ((1.0 - 2.0 * cw.to(torch.float32)) + float(np.sqrt(s2)) * noise)
    del noise
    r = gpu.decode(ch, llr, k, gpu.SPA_F32, max_updates=cap, gamma=0.1)
    torch.cuda.synchronize()
    upd = np_(r.updates_used)
    say(f"[benchmark launch {kind}] mean updates {upd.mean():.0f}, at the cap {int((upd >= cap).sum())}")
    unsat = _syndrome_weights(code, r.bits)
    stopped = upd < cap
    assert stopped.mean() > 0.97
    assert (unsat[stopped] == 0).all()
    fe = int((r.bits != cw).any(1).sum().item())
    assert fe < B // 50, fe
    rng = np.random.default_rng(12)
    for f in [int(x) for x in rng.choice(B, 6, replace=False)] + [int(np.argmax(upd))]:
        a = gpu.decode(ch, llr[f:f + 1], k, gpu.SPA_F32, max_updates=cap, gamma=0.1)
        torch.cuda.synchronize()
        assert int(np_(a.updates_used)[0]) == int(upd[f]), f
        assert int(np_(a.fallbacks)[0]) == int(np_(r.fallbacks)[f]), f
        assert torch.equal(a.bits[0], r.bits[f]), f
        assert torch.equal(a.llr_out[0], r.llr_out[f]), f


@pytest.fixture(scope="module")
def c3_launch(gpu):
    """2048 frames of the Z=128 BG1-shaped code at 1.5 dB (the multi-edge benchmark's batch size):
    64 random codewords from the CPU generator, noise from torch's seeded device generator."""
    code = S.workload_code("c3")
    cw = torch.from_numpy(S.random_codewords(code, 64, 13)).cuda().repeat(32, 1)
    s2 = S.sigma2_from_ebn0(1.5, code.design_rate)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1500)
    noise = torch.randn(tuple(cw.shape), generator=gen, device="cuda")
    llr = (2.0 / s2) * ((1.0 - 2.0 * cw.to(torch.float32)) + float(np.sqrt(s2)) * noise)
    return code, gpu.Code(code), cw, llr


@pytest.mark.parametrize("n_p", [8, 64])
@pytest.mark.parametrize("kind", ["me", "melmd"])
def test_me_benchmark_launch_sampled_frames(gpu, c3_launch, kind, n_p):
    """The multi-edge benchmark's launch shape: Z=128, 2048 frames, N_G=16, keyed fill, cap 3E,
    256 persistent workgroups of 1024 lanes, messages in global memory.  A frame decoded alone uses
    the fill key seed ^ f, the key frame f has in the launch.

    FP32 (the benchmark's own launch): two runs of the launch give bit-identical outputs (several
    checks of one step can change the precomputed total of one VN; those changes are summed per VN
    in ascending check order); every frame that stopped before the cap satisfies all parity
    checks; sampled frames and the longest give, decoded alone, exactly the launch's outputs.

    Fixed point (8-bit; the tuning knobs force the same launch shape): sampled frames and the
    longest give bit for bit the outputs they give when decoded alone."""
    code, ch, cw, llr = c3_launch
    k = gpu.ME_CIRBP if kind == "me" else gpu.ME_LMD_CIRBP
    B, cap, seed = llr.shape[0], 3 * code.E, 2102
    kw = dict(max_updates=cap, gamma=0.1, n_p=n_p, n_g=16, fill=gpu.FILL_HASH)
    rng = np.random.default_rng(14 + n_p)
    picks = [int(x) for x in rng.choice(B, 4, replace=False)]

    # FP32, default plan, twice
    plan = gpu.describe_plan(ch, B, k, n_p=n_p, fill=gpu.FILL_HASH)
    say(f"[ME benchmark launch {kind} N_P={n_p}] FP32 plan {plan}")
    assert (plan["block"], plan["grid"], plan["storage_name"]) == (1024, 256, "global_all")
    r = gpu.decode(ch, llr, k, gpu.SPA_F32, seed=seed, **kw)
    r2 = gpu.decode(ch, llr, k, gpu.SPA_F32, seed=seed, **kw)
    torch.cuda.synchronize()
    for name in ("bits", "llr_out", "updates_used", "steps_used"):
        assert torch.equal(getattr(r, name), getattr(r2, name)), f"FP32 rerun differs in {name}"
    del r2
    upd, steps = np_(r.updates_used), np_(r.steps_used)
    unsat = _syndrome_weights(code, r.bits)
    stopped = upd < cap
    assert stopped.mean() > 0.98
    assert (unsat[stopped] == 0).all()
    for f in picks + [int(np.argmax(steps))]:
        a = gpu.decode(ch, llr[f:f + 1], k, gpu.SPA_F32, seed=seed ^ f, **kw)
        torch.cuda.synchronize()
        assert int(np_(a.updates_used)[0]) == int(upd[f]), f
        assert int(np_(a.steps_used)[0]) == int(steps[f]), f
        assert torch.equal(a.bits[0], r.bits[f]), f
        assert torch.equal(a.llr_out[0], r.llr_out[f]), f

    # fixed point, the same launch shape
    gpu.set_tuning(ch, k, gpu.MS_FIX, block=1024, storage=gpu.STORE_GLOBAL)
    try:
        fx = dict(q_bits=8, frac_bits=2, **kw)
        plan = gpu.describe_plan(ch, B, k, gpu.MS_FIX, q_bits=8, frac_bits=2, n_p=n_p, fill=gpu.FILL_HASH)
        say(f"[ME benchmark launch {kind} N_P={n_p}] fixed-point plan {plan}")
        assert (plan["block"], plan["grid"], plan["storage_name"]) == (1024, 256, "global_all")
        r = gpu.decode(ch, llr, k, gpu.MS_FIX, seed=seed, **fx)
        torch.cuda.synchronize()
        upd, steps = np_(r.updates_used), np_(r.steps_used)
        for f in picks + [int(np.argmax(steps))]:
            a = gpu.decode(ch, llr[f:f + 1], k, gpu.MS_FIX, seed=seed ^ f, **fx)
            torch.cuda.synchronize()
            assert int(np_(a.updates_used)[0]) == int(upd[f]), f
            assert int(np_(a.steps_used)[0]) == int(steps[f]), f
            assert torch.equal(a.bits[0], r.bits[f]), f
            assert torch.equal(a.llr_out[0], r.llr_out[f]), f
    finally:
        gpu.set_tuning(ch, k, gpu.MS_FIX, clear=True)


# ------------------------------------------------------------------------------------------
# edge cases
# ------------------------------------------------------------------------------------------
def test_edge_cases(gpu, c0):
    code, ch = c0
    # empty batch
    t = torch.zeros((0, code.N), device="cuda")
    r = gpu.decode(ch, t, gpu.CIRBP, gpu.SPA_F32, max_updates=10)
    assert r.bits.shape == (0, code.N)
    # max_updates = 0, and an already-valid word (strong all-zero channel): 0 updates
    llr = np.full((3, code.N), 5.0, dtype=np.float32)
    for kind in ("cirbp", "rbp", "flooding", "layered"):
        g = gpu_decode(gpu, ch, llr, kind, gpu.SPA_F32, max_updates=100 * code.E)
        assert np.all(np_(g.updates_used) == 0) and not np_(g.bits).any()
    cw, llr = S.frames(code, 8, 1.0, 107)
    g = gpu_decode(gpu, ch, llr, "cirbp", gpu.MS_FIX, max_updates=0)
    assert np.all(np_(g.updates_used) == 0)
    # all-zero channel (every value tied)
    llr = np.zeros((4, code.N), dtype=np.float32)
    ref = O.decode(code, llr, O.CIRBP, O.MSFIX, max_updates=200, trace=True)
    g = gpu_decode(gpu, ch, llr, "cirbp", gpu.MS_FIX, max_updates=200, trace=True)
    np.testing.assert_array_equal(np_(g.trace), ref.trace)
    # single parity check of length 3 (smallest code), FP32 against the oracle
    spc = S.spc_code(3)
    sh = gpu.Code(spc)
    llr = np.array([[1.0, -0.5, 2.0], [0.2, 0.3, -0.1]], dtype=np.float32)
    ref = O.decode(spc, llr, O.CIRBP, O.SPA, max_updates=10, check_every=0, trace=True)
    g = gpu_decode(gpu, sh, llr, "cirbp", gpu.SPA_F32, max_updates=10, check_every=0, trace=True)
    np.testing.assert_array_equal(np_(g.trace), ref.trace)
    np.testing.assert_allclose(np_(g.llr_out), ref.llr_out, rtol=1e-5, atol=1e-5)
    # replay with an invalid edge id stops that frame where the id appears
    rep = torch.tensor([[0, 1, code.E + 5, 2]], dtype=torch.int32)
    cw, llr = S.frames(code, 1, 2.0, 108)
    g = gpu_decode(gpu, ch, llr, "replay", gpu.SPA_F32, max_updates=4, replay=rep)
    assert int(np_(g.updates_used)[0]) == 2


# ------------------------------------------------------------------------------------------
# storage variants: every (pre location, topology source) combination is bit-exact
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("pre", ["lds", "global", "all", "all_lt", "frame", "rec", "state"])
@pytest.mark.parametrize("topo", ["global", "lds", "qc"])
@pytest.mark.parametrize("fpc", [0, 3])
def test_fixed_storage_variants(gpu, pre, topo, fpc):
    """Every storage / topology / launch-shape knob gives the oracle's results bit for bit."""
    code = S.qc_24col(24, 12, seed=4)  # N = 576, quasi-cyclic
    cw, llr = S.frames(code, 200, 2.0, 109)
    ref = O.decode(code, llr, O.CIRBP, O.MSFIX, max_updates=1500, q_bits=8, frac_bits=2, trace=True, dump=True,
                   threads=8)
    store = {"lds": gpu.STORE_LDS, "global": gpu.STORE_GLOBAL, "all": gpu.STORE_GLOBAL_ALL,
             "all_lt": gpu.STORE_GLOBAL_LT, "frame": gpu.STORE_GLOBAL_FRAME, "rec": gpu.STORE_GLOBAL_REC,
             "state": gpu.STORE_GLOBAL_STATE}[pre]
    tp = {"global": gpu.TOPO_GLOBAL, "lds": gpu.TOPO_LDS, "qc": gpu.TOPO_QC}[topo]
    handles = [gpu.Code(code)] if topo == "qc" else [gpu.Code(code), gpu.Code(code, csr=True)]
    for h in handles:
        say(f"[variant pre={pre} topo={topo} frames/CU={fpc}] qc24 Z=24")
        gpu.set_tuning(h, gpu.CIRBP, gpu.MS_FIX, frames_per_cu=fpc, storage=store, topology=tp)
        try:
            g = gpu_decode(gpu, h, llr, "cirbp", gpu.MS_FIX, max_updates=1500, q_bits=8, frac_bits=2, trace=True,
                           dump=True)
        finally:
            gpu.set_tuning(h, gpu.CIRBP, gpu.MS_FIX, clear=True)
        np.testing.assert_array_equal(np_(g.trace), ref.trace)
        np.testing.assert_array_equal(np_(g.bits), ref.bits)
        np.testing.assert_array_equal(np_(g.updates_used), ref.updates_used)
        np.testing.assert_array_equal(np_(g.c2v), ref.c2v)
        np.testing.assert_array_equal(np_(g.D), ref.D)


@pytest.mark.parametrize("store", ["lds", "all", "rec", "state"])
@pytest.mark.parametrize("kind", ["cirbp", "rbp", "replay"])
def test_fixed_degree_one_vns(gpu, store, kind):
    """BG1-shaped base graph lifted by Z = 4 (n = 272): updates of degree-1 VNs (whose only check
    is the updated edge's check) refresh that check's key without a row pass; bit-exact."""
    code = S.qc_bg1_shaped(4, seed=3)
    cw, llr = S.frames(code, 96, 1.0, 113)
    st = {"lds": gpu.STORE_LDS, "all": gpu.STORE_GLOBAL_ALL, "rec": gpu.STORE_GLOBAL_REC,
          "state": gpu.STORE_GLOBAL_STATE}[store]
    say(f"[degree-1 VNs] bg1 Z=4 {kind} store={store}")
    kw = dict(max_updates=2000, q_bits=8, frac_bits=2, trace=True, dump=True)
    rep = None
    if kind == "replay":
        rec = O.decode(code, llr, O.CIRBP, O.MSFIX, max_updates=1500, q_bits=8, frac_bits=2, check_every=0,
                       trace=True, threads=8)
        rep = rec.trace
        kw["max_updates"] = 1500
    ref = O.decode(code, llr, KIND[kind][0], O.MSFIX, threads=8, replay=rep, **kw)
    h = gpu.Code(code)
    gpu.set_tuning(h, KIND[kind][1], gpu.MS_FIX, storage=st, frames_per_cu=2)
    try:
        g = gpu_decode(gpu, h, llr, kind, gpu.MS_FIX, replay=None if rep is None else torch.from_numpy(rep), **kw)
    finally:
        gpu.set_tuning(h, KIND[kind][1], gpu.MS_FIX, clear=True)
    np.testing.assert_array_equal(np_(g.trace), ref.trace)
    np.testing.assert_array_equal(np_(g.updates_used), ref.updates_used)
    np.testing.assert_array_equal(np_(g.bits), ref.bits)
    np.testing.assert_array_equal(np_(g.c2v), ref.c2v)
    np.testing.assert_array_equal(np_(g.pre), ref.pre)
    if kind != "rbp":  # RBP keeps no CIs
        np.testing.assert_array_equal(np_(g.D), ref.D)


def test_fixed_capacity_fallback_large_code(gpu):
    """A code whose check keys alone exceed a CU's LDS (BG1-shaped base lifted by Z = 900:
    m = 41400) decodes with the keys in global memory, bit-exact."""
    code = S.qc_bg1_shaped(900, seed=3)
    h = gpu.Code(code)
    d = gpu.describe_plan(h, 2, gpu.CIRBP, gpu.MS_FIX, q_bits=8, frac_bits=2)
    say(f"[capacity fallback] bg1 Z=900 plan {d}")
    assert d["storage"] == gpu.STORE_GLOBAL_STATE
    cw, llr = S.frames(code, 2, 1.5, 114, zero_codeword=True)
    kw = dict(max_updates=1500, q_bits=8, frac_bits=2, trace=True)
    ref = O.decode(code, llr, O.CIRBP, O.MSFIX, threads=2, **kw)
    g = gpu_decode(gpu, h, llr, "cirbp", gpu.MS_FIX, **kw)
    np.testing.assert_array_equal(np_(g.trace), ref.trace)
    np.testing.assert_array_equal(np_(g.updates_used), ref.updates_used)
    np.testing.assert_array_equal(np_(g.bits), ref.bits)


def many_four_cycles_code():
    """Six checks of degree 16 on 32 VNs with heavy overlap: the two-hop table of a VN lists up to
    27 other VNs more than once (more than the kernels' LDS groups hold), in up to two passes."""
    rows = [[0, 1, 5, 7, 11, 12, 15, 16, 17, 19, 20, 21, 24, 26, 28, 31],
            [3, 4, 5, 8, 9, 12, 14, 15, 16, 17, 18, 20, 23, 24, 25, 30],
            [0, 2, 4, 5, 6, 10, 14, 16, 18, 19, 21, 22, 24, 26, 29, 30],
            [1, 3, 4, 9, 10, 12, 13, 14, 16, 19, 20, 22, 25, 26, 28, 31],
            [1, 2, 3, 5, 6, 8, 9, 10, 11, 12, 18, 21, 22, 28, 29, 30],
            [1, 3, 4, 5, 6, 10, 11, 12, 14, 15, 17, 18, 23, 27, 28, 31]]
    return S.code_from_rows(6, 32, rows, name="overlap32")


@pytest.mark.parametrize("store", ["lds", "rec", "state"])
def test_fixed_repeated_two_hop_vns_bit_exact(gpu, store):
    """VNs met on several checks of the updated VN (4-cycles): their precomputed totals take every
    change of the update, through the LDS groups and through the overflow path."""
    code = many_four_cycles_code()
    h = gpu.Code(code)
    cw, llr = S.frames(code, 200, 1.0, 112)
    st = {"lds": gpu.STORE_LDS, "rec": gpu.STORE_GLOBAL_REC, "state": gpu.STORE_GLOBAL_STATE}[store]
    say(f"[repeated two-hop VNs] overlap32 store={store}")
    ref = O.decode(code, llr, O.CIRBP, O.MSFIX, max_updates=400, check_every=0, q_bits=8, frac_bits=2, trace=True,
                   dump=True, threads=8)
    gpu.set_tuning(h, gpu.CIRBP, gpu.MS_FIX, storage=st, frames_per_cu=2)
    try:
        g = gpu_decode(gpu, h, llr, "cirbp", gpu.MS_FIX, max_updates=400, check_every=0, q_bits=8, frac_bits=2,
                       trace=True, dump=True)
    finally:
        gpu.set_tuning(h, gpu.CIRBP, gpu.MS_FIX, clear=True)
    np.testing.assert_array_equal(np_(g.trace), ref.trace)
    np.testing.assert_array_equal(np_(g.updates_used), ref.updates_used)
    np.testing.assert_array_equal(np_(g.Lt), ref.Lt)
    np.testing.assert_array_equal(np_(g.D), ref.D)
    # FP32: the oracle's schedule replayed, messages and totals within tolerance
    rec = O.decode(code, llr, O.CIRBP, O.SPA, max_updates=300, check_every=0, trace=True, threads=8)
    refr = O.decode(code, llr, O.REPLAY, O.SPA, max_updates=300, replay=rec.trace, dump=True, threads=8)
    gpu.set_tuning(h, gpu.REPLAY, gpu.SPA_F32, storage=st, frames_per_cu=2)
    try:
        gr = gpu_decode(gpu, h, llr, "replay", gpu.SPA_F32, max_updates=300, replay=torch.from_numpy(rec.trace),
                        dump=True)
    finally:
        gpu.set_tuning(h, gpu.REPLAY, gpu.SPA_F32, clear=True)
    assert_close_msgs(gr.Lt, refr.Lt, "Lt")
    assert_close_msgs(gr.L, refr.L, "L")
    assert np.abs(np_(gr.D) - refr.D).max() <= 1e-4


# ------------------------------------------------------------------------------------------
# ME-CIRBP (Algorithms 4 and 5)
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("fill", [0, 1])
@pytest.mark.parametrize("n_p,n_g", [(1, 16), (4, 4), (8, 16), (24, 8)])
def test_fixed_me_bit_exact_c0(gpu, c0, n_p, n_g, fill):
    code, ch = c0
    cw, llr = S.frames(code, 300, 2.0, 110)
    say(f"[fixed me] c0 n_p={n_p} n_g={n_g} fill={fill}")
    kw = dict(max_updates=2400, n_p=n_p, n_g=n_g, fill=fill, seed=77, trace=True, dump=True)
    ref = O.decode(code, llr, O.MECIRBP, O.MSFIX, q_bits=6, frac_bits=1, threads=8, **kw)
    g = gpu_decode(gpu, ch, llr, "me", gpu.MS_FIX, q_bits=6, frac_bits=1, **kw)
    np.testing.assert_array_equal(np_(g.updates_used), ref.updates_used)
    np.testing.assert_array_equal(np_(g.steps_used), ref.steps_used)
    np.testing.assert_array_equal(np_(g.trace), ref.trace)
    np.testing.assert_array_equal(np_(g.bits), ref.bits)
    np.testing.assert_array_equal(np_(g.c2v), ref.c2v)
    np.testing.assert_array_equal(np_(g.pre), ref.pre)
    np.testing.assert_array_equal(np_(g.Lt), ref.Lt)
    np.testing.assert_array_equal(np_(g.D), ref.D)


def test_fixed_me_qc_and_bg1_z128(gpu):
    """Keyed fill against the oracle, traced.  On the Z = 128 code a fill group holds hundreds of
    VNs: at N_P = 8 the fill comes from the short list of keys below the step's threshold, at
    N_P = 64 often from the radix selection (fills the list cannot hold)."""
    c3 = S.workload_code("c3")
    for code, B, eb, n_p, mu in ((S.qc_24col(24, 8, seed=2), 64, 2.5, 16, 3000),
                                 (c3, 2, 1.25, 8, 3000), (c3, 2, 1.25, 32, 4000),
                                 (c3, 2, 1.25, 64, 6000)):
        h = gpu.Code(code)
        cw, llr = S.frames(code, B, eb, 111)
        say(f"[fixed me hash] {code.name} n_p={n_p}")
        kw = dict(max_updates=mu, n_p=n_p, n_g=16, fill=1, seed=5, trace=True)
        ref = O.decode(code, llr, O.MECIRBP, O.MSFIX, q_bits=8, frac_bits=2, threads=4, **kw)
        g = gpu_decode(gpu, h, llr, "me", gpu.MS_FIX, q_bits=8, frac_bits=2, **kw)
        np.testing.assert_array_equal(np_(g.trace), ref.trace)
        np.testing.assert_array_equal(np_(g.updates_used), ref.updates_used)
        np.testing.assert_array_equal(np_(g.bits), ref.bits)


def test_f32_me_fer_within_interval_c0(gpu, c0):
    code, ch = c0
    cw, llr = S.frames(code, 1000, 2.0, 112)
    say("[f32 me] c0 1000 frames n_p=8 hash fill")
    kw = dict(max_updates=2400, n_p=8, n_g=16, fill=1, seed=9)
    ref = O.decode(code, llr, O.MECIRBP, O.SPA, threads=8, **kw)
    g = gpu_decode(gpu, ch, llr, "me", gpu.SPA_F32, **kw)
    k_ref = int(np.any(ref.bits != cw, axis=1).sum())
    k_gpu = int(np.any(np_(g.bits) != cw, axis=1).sum())
    lo, hi = cp_interval(k_ref, 1000)
    assert lo <= k_gpu / 1000 <= hi, (k_gpu, k_ref, lo, hi)


# ------------------------------------------------------------------------------------------
# persistent batched launch over uneven codes and schedules
# ------------------------------------------------------------------------------------------
def _mixed_batch(codes, F, seed, ebn0s=(1.5, 2.5, 3.5), kinds=None):
    from paper_2102_11089_amd import ldpc as L
    rng = np.random.default_rng(seed)
    frames = np.zeros(F, dtype=L.FRAME_DESC)
    llrs, cws, per = [], [], []
    off = 0
    if kinds is None:
        kinds = [L.FLOODING, L.LAYERED, L.RBP, L.CIRBP, L.LMDRBP, L.SLMDRBP, L.LMD_CIRBP]
    for f in range(F):
        ci = int(rng.integers(len(codes)))
        c = codes[ci]
        kind = kinds[int(rng.integers(len(kinds)))]
        cw, llr = S.frames(c, 1, float(rng.choice(ebn0s)), seed * 1000 + f)
        frames[f] = (ci, kind, 0.1, 0, (20 if kind in (L.FLOODING, L.LAYERED) else 3) * c.E, off, off)
        llrs.append(llr[0]); cws.append(cw[0]); per.append((ci, kind, off))
        off += c.N
    return frames, np.concatenate(llrs).astype(np.float32), cws, per, off


@pytest.mark.parametrize("arith", ["fix", "f32"])
def test_batch_uneven_codes_and_schedules(gpu, arith):
    codes = [S.qc_24col(24, 12, seed=1), S.qc_24col(48, 8, seed=1), S.qc_24col(24, 4, seed=1)]
    hs = [gpu.Code(c) for c in codes]
    frames, pool, cws, per, out_len = _mixed_batch(codes, 240, 3)
    a = gpu.MS_FIX if arith == "fix" else gpu.SPA_F32
    say(f"[batch {arith}] 240 frames over 3 codes and 7 schedules")
    bits, llr_out, upd, steps, fall = gpu.decode_batch(hs, frames, torch.from_numpy(pool).cuda(), out_len, arith=a,
                                                       q_bits=8, frac_bits=2)
    torch.cuda.synchronize()
    bits, upd = np_(bits), np_(upd)
    kmap = {gpu.FLOODING: O.FLOODING, gpu.LAYERED: O.LAYERED, gpu.RBP: O.RBP, gpu.CIRBP: O.CIRBP,
            gpu.LMDRBP: O.LMDRBP, gpu.SLMDRBP: O.SLMDRBP, gpu.LMD_CIRBP: O.LMDCIRBP}
    errs_gpu = errs_ref = 0
    for f, (ci, kind, off) in enumerate(per):
        c = codes[ci]
        llr = pool[off:off + c.N][None]
        mu = int(frames[f]["max_updates"])
        if arith == "fix":
            ref = O.decode(c, llr, kmap[kind], O.MSFIX, max_updates=mu, q_bits=8, frac_bits=2)
            assert int(upd[f]) == int(ref.updates_used[0]), (f, kind)
            np.testing.assert_array_equal(bits[off:off + c.N], ref.bits[0])
        elif kind not in (gpu.FLOODING, gpu.LAYERED):  # same per-frame code path as the per-code kernel
            g = gpu.decode(hs[ci], torch.from_numpy(llr).cuda(), int(kind), gpu.SPA_F32, max_updates=mu)
            torch.cuda.synchronize()
            assert int(upd[f]) == int(np_(g.updates_used)[0])
            np.testing.assert_array_equal(bits[off:off + c.N], np_(g.bits)[0])
        else:
            ref = O.decode(c, llr, kmap[kind], O.SPA, max_updates=mu)
            errs_ref += int(np.any(ref.bits[0] != cws[f]))
            errs_gpu += int(np.any(bits[off:off + c.N] != cws[f]))
    assert abs(errs_gpu - errs_ref) <= 2


def _oracle_by_group(codes, frames, pool, per, kmap, arith, **kw):
    """Oracle decodes of a batch's frames, grouped by (code, schedule, cap) so that each group runs
    as one multi-threaded oracle call: per frame (bits, updates_used)."""
    groups = {}
    for f, (ci, kind, off) in enumerate(per):
        groups.setdefault((ci, kind, int(frames[f]["max_updates"])), []).append(f)
    out = {}
    for (ci, kind, mu), fs in groups.items():
        c = codes[ci]
        llr = np.stack([pool[per[f][2]:per[f][2] + c.N] for f in fs])
        r = O.decode(c, llr, kmap[kind], arith, max_updates=mu, gamma=0.1, threads=8, **kw)
        for x, f in enumerate(fs):
            out[f] = (r.bits[x], int(r.updates_used[x]))
    return out


@pytest.mark.parametrize("arith", ["fix", "f32"])
def test_batch_c2_shape_all_codes(gpu, arith):
    """The batched launch at the shape of the batched workload: all 12 codes of the 24-column
    family (Z in {24, 48, 96}, base rows 12, 8, 6, 4: rates 1/2, 2/3, 3/4, 5/6) in one launch, the
    LDS layout sized for the largest (n = 2304), schedules drawn from {flooding (20 iterations), RBP,
    CIRBP (3E)}.  8-bit fixed point: every frame bit for bit equal to the oracle (decoded bits and
    updates used).  FP32: each schedule's frame errors inside the 95% Clopper-Pearson interval of
    the oracle's on the same frames (low Eb/N0, so that errors occur)."""
    codes = [S.qc_24col(Z, mb, seed=1) for Z in (24, 48, 96) for mb in (12, 8, 6, 4)]
    hs = [gpu.Code(c) for c in codes]
    kinds = [gpu.FLOODING, gpu.RBP, gpu.CIRBP]
    if arith == "fix":
        F, ebn0s, a, oa = 480, (1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0), gpu.MS_FIX, O.MSFIX
    else:
        F, ebn0s, a, oa = 1440, (1.0, 1.5), gpu.SPA_F32, O.SPA
    frames, pool, cws, per, out_len = _mixed_batch(codes, F, 21, ebn0s=ebn0s, kinds=kinds)
    say(f"[batch c2 shape {arith}] {F} frames over 12 codes and 3 schedules")
    bits, llr_out, upd, steps, fall = gpu.decode_batch(hs, frames, torch.from_numpy(pool).cuda(), out_len, arith=a,
                                                       q_bits=8, frac_bits=2)
    torch.cuda.synchronize()
    bits, upd = np_(bits), np_(upd)
    kmap = {gpu.FLOODING: O.FLOODING, gpu.RBP: O.RBP, gpu.CIRBP: O.CIRBP}
    ref = _oracle_by_group(codes, frames, pool, per, kmap, oa, q_bits=8, frac_bits=2)
    say(f"[batch c2 shape {arith}] oracle done")
    assert {per[f][0] for f in range(F)} == set(range(12))
    errs = {k: [0, 0, 0] for k in kinds}  # frames, gpu errors, oracle errors
    for f, (ci, kind, off) in enumerate(per):
        n = codes[ci].N
        rb, ru = ref[f]
        if arith == "fix":
            assert int(upd[f]) == ru, (f, ci, kind)
            np.testing.assert_array_equal(bits[off:off + n], rb)
        e = errs[kind]
        e[0] += 1
        e[1] += int(np.any(bits[off:off + n] != cws[f]))
        e[2] += int(np.any(rb != cws[f]))
    for kind, (nf, kg, kr) in errs.items():
        lo, hi = cp_interval(kr, nf)
        say(f"[batch c2 shape {arith}] schedule {kind}: {nf} frames, frame errors gpu {kg}, oracle {kr}")
        assert lo <= kg / nf <= hi, (kind, kg, kr, nf, lo, hi)


def test_batch_rejects_bad_descriptors(gpu):
    codes = [S.qc_24col(24, 12, seed=1)]
    hs = [gpu.Code(codes[0])]
    frames, pool, cws, per, out_len = _mixed_batch(codes, 6, 4)
    frames[1]["code"] = 7          # unknown code
    frames[2]["kind"] = 42         # unknown schedule
    frames[3]["llr_off"] = len(pool) - 10   # LLRs past the end of the pool
    frames[4]["gamma"] = -1.0      # negative threshold
    bits, llr_out, upd, steps, fall = gpu.decode_batch(hs, frames, torch.from_numpy(pool).cuda(), out_len)
    torch.cuda.synchronize()
    u = np_(upd)
    assert list(u[1:5]) == [-1, -1, -1, -1]
    assert u[0] >= 0 and u[5] >= 0


def test_binding_refuses_buffers_that_do_not_match_their_sizes(gpu, c0):
    """The kernels index each buffer by the sizes passed beside it: the binding refuses, before any
    launch, a buffer of another shape, type or device (ValueError)."""
    code, h = c0
    cw, llr = S.frames(code, 4, 2.0, 5)
    t = torch.from_numpy(llr).cuda()
    say("[binding] mismatched buffers refused on the host")
    with pytest.raises(ValueError, match="replay"):
        gpu.decode(h, t, gpu.REPLAY, gpu.SPA_F32, max_updates=4, replay=torch.zeros((2, 4), dtype=torch.int32))
    for bad in (t.double(), t[:, :50], t.cpu(), t[0]):
        with pytest.raises(ValueError, match="llr"):
            gpu.decode(h, bad, gpu.CIRBP, gpu.SPA_F32, max_updates=4)
    frames, pool, _, _, out_len = _mixed_batch([code], 2, 1)
    with pytest.raises(ValueError, match="llr_pool"):
        gpu.decode_batch([h], frames, torch.from_numpy(pool.astype(np.float64)).cuda(), out_len)
    with pytest.raises(ValueError, match="frames"):
        gpu.decode_batch([h], frames.view(np.uint8), torch.from_numpy(pool).cuda(), out_len)
    with pytest.raises(ValueError, match="codewords"):
        gpu.Sweep(h, torch.zeros((2, code.N - 1), dtype=torch.uint8, device="cuda"), [2.0], 0.5, 8, gpu.CIRBP)
    w = torch.ones(code.E, device="cuda")
    tr = torch.randint(0, code.E, (4, 40), dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError, match="trace"):
        gpu.unrolled_forward(h, t, w, tr[:3], 16)
    with pytest.raises(ValueError, match="w:"):
        gpu.unrolled_forward(h, t, w[:-1], tr, 16)
    soft, ck, _ = gpu.unrolled_forward(h, t, w, tr, 16)
    gs = torch.ones((4, code.N), device="cuda")
    with pytest.raises(ValueError, match="grad_soft"):
        gpu.unrolled_backward(h, w, tr, ck, gs[:3], 16)
    with pytest.raises(ValueError, match="ckpt"):
        gpu.unrolled_backward(h, w, tr, ck[: ck.numel() // 2], gs, 16)
    g_llr, g_w = gpu.unrolled_backward(h, w, tr, ck, gs, 16)
    torch.cuda.synchronize()
    assert torch.isfinite(soft).all() and torch.isfinite(g_llr).all() and torch.isfinite(g_w).all()


@pytest.mark.parametrize("store", ["lds", "global", "all", "all_lt", "frame", "rec", "state"])
def test_f32_storage_modes_identical(gpu, store):
    """FP32 results do not depend on where the messages live (same arithmetic, same order)."""
    code = S.workload_code("c4")
    h = gpu.Code(code)
    cw, llr = S.frames(code, 300, 2.0, 111)
    t = torch.from_numpy(llr).cuda()
    gpu.set_tuning(h, gpu.CIRBP, gpu.SPA_F32, clear=True)
    base = gpu.decode(h, t, gpu.CIRBP, gpu.SPA_F32, max_updates=4000, trace=True)
    st = {"lds": gpu.STORE_LDS, "global": gpu.STORE_GLOBAL, "all": gpu.STORE_GLOBAL_ALL,
          "all_lt": gpu.STORE_GLOBAL_LT, "frame": gpu.STORE_GLOBAL_FRAME, "rec": gpu.STORE_GLOBAL_REC,
          "state": gpu.STORE_GLOBAL_STATE}[store]
    gpu.set_tuning(h, gpu.CIRBP, gpu.SPA_F32, storage=st, frames_per_cu=2)
    try:
        r = gpu.decode(h, t, gpu.CIRBP, gpu.SPA_F32, max_updates=4000, trace=True)
        torch.cuda.synchronize()
    finally:
        gpu.set_tuning(h, gpu.CIRBP, gpu.SPA_F32, clear=True)
    for a, b in ((base.trace, r.trace), (base.llr_out, r.llr_out), (base.updates_used, r.updates_used)):
        np.testing.assert_array_equal(np_(a), np_(b))
