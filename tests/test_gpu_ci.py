"""CI-metric statistics from the GPU flooding decoder equal those from the oracle's (Sec. III-A)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2102_11089_amd import ci_analysis as C
from paper_2102_11089_amd import synth as S

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("it", [1, 2, 3])
def test_decoded_j_and_f_match_the_oracle(gpu, it):
    code = S.qc_regular(4, 8, 250, seed=1)  # N = 2000
    h = gpu.Code(code)
    cw, llr = S.frames(code, 200, 2.0, 33, zero_codeword=True)
    print(f"[ci] qc48 Z=250 iteration {it}", flush=True)
    t = torch.from_numpy(llr.astype(np.float32)).cuda()
    L, Lt = C.flooding_states(gpu, h, t, it)
    torch.cuda.synchronize()
    gs = [0.0, 0.05, 0.1, 0.2, 0.3]
    e = C.empirical(L.cpu().numpy(), Lt.cpu().numpy(), gs)
    a = O.decode(code, llr.astype(np.float32), O.FLOODING, O.SPA, max_updates=(it - 1) * code.E, check_every=0, threads=8)
    b = O.decode(code, llr.astype(np.float32), O.FLOODING, O.SPA, max_updates=it * code.E, check_every=0, threads=8)
    r = C.empirical(a.llr_out, b.llr_out, gs)
    for k in ("n_correct", "n_incorrect", "n_rise", "n_fall"):
        np.testing.assert_allclose(e[k], r[k], rtol=2e-3, atol=2)
    np.testing.assert_allclose(e["J"], r["J"], rtol=5e-3)
