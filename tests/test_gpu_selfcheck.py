"""The self-checking build (`build.build_selfcheck`, -DLDPC_SELFCHECK) on the GPU: after every
single-edge update the kernel recomputes L, Lt and a stored D of the touched VNs, the keys of the
updated VN's checks and the affected block maxima from their definitions.  Across every
single-edge schedule, both arithmetics, the storage modes, degree-1 VNs, repeated two-hop VNs and
the c1 benchmark plan, no update may leave a mismatch, and every update must have been checked."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
def test_selfcheck_build_finds_no_inconsistent_state():
    sys.path.insert(0, ROOT)
    from paper_2102_11089_amd import build as B
    lib = B.SELFCHECK_LIB
    assert os.path.exists(lib), "the self-checking library is built by build() (paper_2102_11089_amd.build)"
    print("selfcheck cases: running", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "selfcheck_cases.py"), lib],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "selfcheck cases done" in r.stdout
    rows = [json.loads(x) for x in r.stdout.splitlines() if x.startswith("{")]
    assert len(rows) >= 40
    for row in rows:
        c = row["counts"]
        assert c[:6] == [0] * 6, row
        assert c[7] == row["updates"] > 0, row
