"""GPU parity of the differentiable unrolled decoder (damped replay + hand-written adjoint).

The schedules are recorded by the oracle (CIRBP, FP64) or drawn at random from a seed; the HIP
forward must match the oracle's FP64 damped replay within |gpu - ref| <= 1e-4 max(|ref|, 1), and
the adjoint its FP64 reverse-mode gradient within |gpu - ref| <= 1e-3 |ref| + 1e-5 max|ref| per
coordinate (FP32 through a few hundred dependent steps).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2102_11089_amd import synth as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def c4(gpu):
    code = S.workload_code("c4")
    return code, gpu.Code(code)


def oracle_traces(code, llr, T):
    r = O.decode(code, llr, O.CIRBP, O.SPA, max_updates=T, check_every=0, trace=True, threads=16)
    return r.trace


def close(gpu_v, ref, rel, floor):
    err = np.abs(gpu_v - ref)
    bound = rel * np.abs(ref) + floor
    return err.max(), bool(np.all(err <= bound))


def run(gpu, ch, llr, w, tr, K=32, c2v=False):
    t_llr = torch.from_numpy(np.ascontiguousarray(llr, dtype=np.float32)).cuda()
    t_w = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).cuda()
    t_tr = torch.from_numpy(np.ascontiguousarray(tr, dtype=np.int32)).cuda()
    soft, ck, c2v_out = gpu.unrolled_forward(ch, t_llr, t_w, t_tr, K, c2v=c2v)
    return t_llr, t_w, t_tr, soft, ck, c2v_out


def test_forward_matches_oracle(gpu, c4):
    code, ch = c4
    rng = np.random.default_rng(1)
    cw, llr = S.frames(code, 64, 2.0, 21)
    tr = oracle_traces(code, llr, 300)
    w = rng.uniform(0.5, 1.2, code.E)
    say("[unrolled fwd] N=576, 64 frames, T=300")
    _, _, _, soft, _, c2v = run(gpu, ch, llr, w, tr, c2v=True)
    torch.cuda.synchronize()
    L_ref, c2v_ref = O.unrolled_forward(code, llr.astype(np.float64), w.astype(np.float32).astype(np.float64), tr,
                                        threads=16)
    np.testing.assert_allclose(soft.cpu().numpy(), L_ref, rtol=1e-4, atol=1e-4)
    np.testing.assert_allclose(c2v.cpu().numpy(), c2v_ref, rtol=1e-4, atol=1e-4)


def test_unit_weights_equal_gpu_replay(gpu, c4):
    code, ch = c4
    cw, llr = S.frames(code, 32, 2.0, 22)
    tr = oracle_traces(code, llr, 300)
    say("[unrolled w=1] vs replay decode")
    _, _, t_tr, soft, _, _ = run(gpu, ch, llr, np.ones(code.E), tr)
    r = gpu.decode(ch, torch.from_numpy(llr).cuda(), gpu.REPLAY, gpu.SPA_F32, max_updates=300, replay=t_tr,
                   check_every=0, dump=True)
    torch.cuda.synchronize()
    np.testing.assert_allclose(soft.cpu().numpy(), r.L.cpu().numpy(), rtol=1e-4, atol=1e-4)


@pytest.mark.parametrize("K", [1, 7, 32, 128])
def test_gradient_matches_oracle(gpu, c4, K):
    code, ch = c4
    rng = np.random.default_rng(2)
    B, T = 48, 300
    cw, llr = S.frames(code, B, 2.0, 23)
    tr = oracle_traces(code, llr, T)
    w = rng.uniform(0.6, 1.1, code.E).astype(np.float32)
    gL = rng.standard_normal((B, code.N)).astype(np.float32)
    say(f"[unrolled grad] N=576, {B} frames, T={T}, ckpt every {K}")
    _, t_w, t_tr, soft, ck, _ = run(gpu, ch, llr, w, tr, K)
    g_llr, g_w = gpu.unrolled_backward(ch, t_w, t_tr, ck, torch.from_numpy(gL).cuda(), K)
    torch.cuda.synchronize()
    r_llr, r_w = O.unrolled_backward(code, llr.astype(np.float64), w.astype(np.float64), tr, gL.astype(np.float64),
                                     threads=16)
    r_w = r_w.sum(0)
    e1, ok1 = close(g_llr.cpu().numpy(), r_llr, 1e-3, 1e-5 * np.abs(r_llr).max())
    e2, ok2 = close(g_w.cpu().numpy(), r_w, 1e-3, 1e-5 * np.abs(r_w).max())
    say(f"  max |d llr err| {e1:.3g} (max |ref| {np.abs(r_llr).max():.3g}); max |d w err| {e2:.3g} "
        f"(max |ref| {np.abs(r_w).max():.3g})")
    assert ok1 and ok2


def test_gradient_deterministic_and_checkpoint_independent(gpu, c4):
    code, ch = c4
    rng = np.random.default_rng(3)
    B, T = 96, 300
    cw, llr = S.frames(code, B, 2.0, 24)
    tr = rng.integers(0, code.E, size=(B, T)).astype(np.int32)
    w = rng.uniform(0.6, 1.1, code.E).astype(np.float32)
    gs = torch.from_numpy(rng.standard_normal((B, code.N)).astype(np.float32)).cuda()
    res = {}
    for K in (32, 32, 5, 128):
        _, t_w, t_tr, soft, ck, _ = run(gpu, ch, llr, w, tr, K)
        g_llr, g_w = gpu.unrolled_backward(ch, t_w, t_tr, ck, gs, K)
        torch.cuda.synchronize()
        res.setdefault(K, []).append((soft.cpu().numpy(), g_llr.cpu().numpy(), g_w.cpu().numpy()))
    a, b = res[32]
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)  # bitwise reproducible, including grad_w
    for K in (5, 128):
        for x, y in zip(a, res[K][0]):
            np.testing.assert_allclose(x, y, rtol=1e-5, atol=1e-5 * np.abs(y).max())


def test_autograd_function_bce(gpu, c4):
    code, ch = c4
    rng = np.random.default_rng(4)
    B, T = 32, 300
    cw, llr = S.frames(code, B, 2.0, 25)
    tr = torch.from_numpy(oracle_traces(code, llr, T)).cuda()
    x = torch.from_numpy(1.0 - 2.0 * cw.astype(np.float32)).cuda()
    t_llr = torch.from_numpy(llr).cuda().requires_grad_(True)
    t_w = torch.full((code.E,), 1.0, device="cuda").requires_grad_(True)
    soft = gpu.unrolled_decode(ch, t_llr, t_w, tr, 32)
    loss = torch.nn.functional.softplus(-x * soft).mean()
    loss.backward()
    torch.cuda.synchronize()
    # the oracle's own loss gradient, from its own forward
    xs = 1.0 - 2.0 * cw.astype(np.float64)
    L_ref, _ = O.unrolled_forward(code, llr.astype(np.float64), 1.0, tr.cpu().numpy(), threads=16)
    gL = -(xs / (1.0 + np.exp(xs * L_ref))) / L_ref.size
    r_llr, r_w = O.unrolled_backward(code, llr.astype(np.float64), 1.0, tr.cpu().numpy(), gL, threads=16)
    r_w = r_w.sum(0)
    e1, ok1 = close(t_llr.grad.cpu().numpy(), r_llr, 1e-3, 1e-5 * np.abs(r_llr).max())
    e2, ok2 = close(t_w.grad.cpu().numpy(), r_w, 1e-3, 1e-5 * np.abs(r_w).max())
    say(f"[autograd BCE] max err d llr {e1:.3g}, d w {e2:.3g}")
    assert ok1 and ok2


def test_full_size_n576_4096_frames(gpu, c4):
    """The differentiation workload at full size: 4096 frames, T=300, checkpoints every 32.
    grad_w (a sum over all frames) is checked whole; per-frame outputs on a sample."""
    code, ch = c4
    rng = np.random.default_rng(5)
    B, T = 4096, 300
    cw, llr = S.frames(code, B, 2.0, 26)
    say("[unrolled full] recording 4096 x 300 with the oracle")
    tr = oracle_traces(code, llr, T)
    w = rng.uniform(0.8, 1.0, code.E).astype(np.float32)
    x = 1.0 - 2.0 * cw.astype(np.float64)
    say("[unrolled full] oracle forward")
    L_ref, _ = O.unrolled_forward(code, llr.astype(np.float64), w.astype(np.float64), tr, threads=16)
    gL = -(x / (1.0 + np.exp(x * L_ref))) / L_ref.size  # BCE gradient at the oracle's soft output
    say("[unrolled full] GPU forward + backward")
    _, t_w, t_tr, soft, ck, _ = run(gpu, ch, llr, w, tr, 32)
    g_llr, g_w = gpu.unrolled_backward(ch, t_w, t_tr, ck, torch.from_numpy(gL.astype(np.float32)).cuda(), 32)
    torch.cuda.synchronize()
    np.testing.assert_allclose(soft.cpu().numpy(), L_ref, rtol=1e-4, atol=1e-4)
    say("[unrolled full] oracle gradient")
    r_llr, r_w = O.unrolled_backward(code, llr.astype(np.float64), w.astype(np.float64), tr, gL, threads=16)
    r_w = r_w.sum(0)
    sample = rng.choice(B, 64, replace=False)
    e1, ok1 = close(g_llr.cpu().numpy()[sample], r_llr[sample], 1e-3, 1e-5 * np.abs(r_llr).max())
    e2, ok2 = close(g_w.cpu().numpy(), r_w, 1e-3, 1e-5 * np.abs(r_w).max())
    say(f"  max err d llr {e1:.3g} (max {np.abs(r_llr).max():.3g}), d w {e2:.3g} (max {np.abs(r_w).max():.3g})")
    assert ok1 and ok2


def test_edge_cases(gpu, c4):
    code, ch = c4
    rng = np.random.default_rng(6)
    cw, llr = S.frames(code, 4, 2.0, 27)
    tr = rng.integers(0, code.E, size=(4, 70)).astype(np.int32)
    tr[2, 40] = code.E          # invalid id: that frame gets NaN, the others are unaffected
    tr[3, 65] = -1
    w = np.ones(code.E, dtype=np.float32)
    _, t_w, t_tr, soft, ck, _ = run(gpu, ch, llr, w, tr, 16)
    gs = torch.ones((4, code.N), device="cuda")
    g_llr, g_w = gpu.unrolled_backward(ch, t_w, t_tr, ck, gs, 16)
    torch.cuda.synchronize()
    s = soft.cpu().numpy()
    assert np.all(np.isnan(s[2])) and np.all(np.isnan(s[3]))
    assert np.all(np.isfinite(s[:2]))
    assert np.all(np.isnan(g_llr.cpu().numpy()[2:])) and np.all(np.isfinite(g_llr.cpu().numpy()[:2]))
    ref, _ = O.unrolled_forward(code, llr[:2].astype(np.float64), 1.0, tr[:2])
    np.testing.assert_allclose(s[:2], ref, rtol=1e-4, atol=1e-4)
    # T = 0: identity forward, gradient passes straight through, no weight gradient
    t0 = torch.zeros((4, 0), dtype=torch.int32, device="cuda")
    t_llr = torch.from_numpy(llr).cuda()
    soft0, ck0, _ = gpu.unrolled_forward(ch, t_llr, t_w, t0, 32)
    g0, gw0 = gpu.unrolled_backward(ch, t_w, t0, ck0, gs, 32)
    torch.cuda.synchronize()
    assert torch.equal(soft0, t_llr) and torch.equal(g0, gs) and torch.count_nonzero(gw0).item() == 0
    # B = 0
    e = torch.zeros((0, 10), dtype=torch.int32, device="cuda")
    soft_e, ck_e, _ = gpu.unrolled_forward(ch, torch.zeros((0, code.N), device="cuda"), t_w, e, 32)
    g_e, gw_e = gpu.unrolled_backward(ch, t_w, e, ck_e, torch.zeros((0, code.N), device="cuda"), 32)
    torch.cuda.synchronize()
    assert soft_e.shape == (0, code.N) and torch.count_nonzero(gw_e).item() == 0
    # bad checkpoint interval
    with pytest.raises(RuntimeError, match="LDPC_EINVAL"):
        gpu.unrolled_forward(ch, t_llr, t_w, t_tr, 0)
    with pytest.raises(RuntimeError, match="LDPC_EINVAL"):
        gpu.unrolled_forward(ch, t_llr, t_w, t_tr, 129)
