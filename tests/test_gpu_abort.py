"""Stopping decodes and failure paths on the GPU: the process-wide abort flag (every kernel family
starts no frame while it is set and marks those frames updates_used = -1; a decode aborted while
it runs keeps the frames it had started, decoded as without the abort) and the LDPCCI_FAULT hook
(an allocation or launch failure reported as an error code with nothing launched).  The flag is
cleared in every test's teardown, so no other test sees it set."""
import time

import numpy as np
import pytest

from paper_2102_11089_amd import synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture
def clear_abort(gpu):
    gpu.ldpc_request_abort(False)
    yield
    gpu.ldpc_request_abort(False)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("kind", ["cirbp", "lmdcirbp", "flooding", "layered", "me"])
def test_abort_flag_set_before_launch_skips_every_frame(gpu, clear_abort, kind):
    code = S.workload_code("c0")
    h = gpu.Code(code)
    cw, llr = S.frames(code, 64, 2.0, 11)
    k = {"cirbp": gpu.CIRBP, "lmdcirbp": gpu.LMD_CIRBP, "flooding": gpu.FLOODING, "layered": gpu.LAYERED,
         "me": gpu.ME_CIRBP}[kind]
    cap = 50 * code.E if kind in ("flooding", "layered") else 2400
    kw = dict(n_p=4) if kind == "me" else {}
    say(f"[abort] preset, c0 {kind}")
    ref = gpu.decode(h, _cuda(llr), k, gpu.MS_FIX, max_updates=cap, **kw)
    torch.cuda.synchronize()
    gpu.ldpc_request_abort(True)
    r = gpu.decode(h, _cuda(llr), k, gpu.MS_FIX, max_updates=cap, **kw)
    torch.cuda.synchronize()
    assert (r.updates_used.cpu().numpy() == -1).all()
    gpu.ldpc_request_abort(False)
    r2 = gpu.decode(h, _cuda(llr), k, gpu.MS_FIX, max_updates=cap, **kw)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(r2.updates_used.cpu().numpy(), ref.updates_used.cpu().numpy())
    np.testing.assert_array_equal(r2.bits.cpu().numpy(), ref.bits.cpu().numpy())


def test_abort_flag_set_before_batched_launch(gpu, clear_abort):
    code = S.qc_24col(24, 12, seed=1)
    h = gpu.Code(code)
    F = 32
    frames = np.zeros(F, dtype=gpu.FRAME_DESC)
    _, llr = S.frames(code, F, 2.0, 5)
    for f in range(F):
        frames[f] = (0, gpu.CIRBP if f % 2 else gpu.FLOODING, 0.1, 0, 3 * code.E, f * code.N, f * code.N)
    say("[abort] preset, batched launch")
    gpu.ldpc_request_abort(True)
    _, _, upd, _, _ = gpu.decode_batch([h], frames, _cuda(llr.reshape(-1)), F * code.N)
    torch.cuda.synchronize()
    assert (upd.cpu().numpy() == -1).all()


def test_abort_while_running_keeps_started_frames(gpu, clear_abort):
    code = S.workload_code("c1")
    h = gpu.Code(code)
    B = 16384
    cw, llr = S.frames(code, 256, 1.25, 3)
    x = _cuda(np.tile(llr, (B // 256, 1)))
    say("[abort] c1 reference decode")
    ref = gpu.decode(h, x, gpu.CIRBP, gpu.SPA_F32, max_updates=3 * code.E)
    torch.cuda.synchronize()
    t0 = time.time()
    ref2 = gpu.decode(h, x, gpu.CIRBP, gpu.SPA_F32, max_updates=3 * code.E)
    torch.cuda.synchronize()
    full = time.time() - t0
    say(f"[abort] c1 decode aborted after a tenth of {full:.3f} s")
    r = gpu.decode(h, x, gpu.CIRBP, gpu.SPA_F32, max_updates=3 * code.E)
    time.sleep(full / 10)
    gpu.ldpc_request_abort(True)
    torch.cuda.synchronize()
    gpu.ldpc_request_abort(False)
    upd = r.updates_used.cpu().numpy()
    done = upd >= 0
    assert done.any() and not done.all(), int(done.sum())
    assert (upd[~done] == -1).all()
    np.testing.assert_array_equal(upd[done], ref.updates_used.cpu().numpy()[done])
    np.testing.assert_array_equal(r.bits.cpu().numpy()[done], ref.bits.cpu().numpy()[done])
    np.testing.assert_array_equal(ref2.bits.cpu().numpy(), ref.bits.cpu().numpy())


@pytest.mark.parametrize("fault", ["alloc", "launch"])
def test_fault_hook_reports_failure_and_launches_nothing(gpu, clear_abort, monkeypatch, fault):
    code = S.workload_code("c1")
    h = gpu.Code(code)
    cw, llr = S.frames(code, 64, 1.25, 9)
    x = _cuda(llr)
    ref = gpu.decode(h, x, gpu.CIRBP, gpu.SPA_F32, max_updates=3 * code.E)
    torch.cuda.synchronize()
    say(f"[fault] LDPCCI_FAULT={fault}")
    monkeypatch.setenv("LDPCCI_FAULT", fault)
    with pytest.raises(RuntimeError) as ei:
        gpu.decode(h, x, gpu.CIRBP, gpu.SPA_F32, max_updates=3 * code.E)
    assert ("ENOMEM" if fault == "alloc" else "EHIP") in str(ei.value)
    monkeypatch.delenv("LDPCCI_FAULT")
    r = gpu.decode(h, x, gpu.CIRBP, gpu.SPA_F32, max_updates=3 * code.E)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(r.bits.cpu().numpy(), ref.bits.cpu().numpy())
