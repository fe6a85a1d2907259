"""Host-side logic of bench.py (CPU): the Table-1 byte accounting that prices a roofline, pinned to
its closed form on a (3,6)-regular code (384 B per FP32 CIRBP update, 152 B in fixed point); the
multi-edge and RBP variants of it; the FER-crossing interpolation; the CPU-share detection and the
CPU baseline entry (timed on a trivial job)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2102_11089_amd import synth as S  # noqa: E402


def test_table1_bytes_closed_form_on_a_36_regular_code():
    # B_upd = 2 s_c d_v + 2 s_c + 3 s_v + s_d + sum over the other two checks of
    #         d_c (s_c + s_v) + 2 s_c (d_c - 1) + (d_c - 1)(3 s_v + s_d), with d_v = 3, d_c = 6
    code = S.workload_code("c0")
    assert set(np.diff(code.row_ptr).tolist()) == {6}
    t32 = bench.lds_bytes_per_update_table(code)
    assert (t32 == 24 + 24 + 2 * (48 + 40 + 80)).all() and int(t32[0]) == 384
    tfx = bench.lds_bytes_per_update_table(code, 1, 2, 2)
    assert (tfx == 6 + 10 + 2 * (18 + 10 + 40)).all() and int(tfx[0]) == 152
    # residual schedules keep no CI: propagation 2 s_c + 2 s_v, no CI term per touched VN
    trbp = bench.lds_bytes_per_update_table(code, ci=False)
    assert (trbp == 24 + 16 + 2 * (48 + 40)).all()
    # sLMDRBP: no edge choice either
    assert (bench.lds_bytes_per_update_table(code, ci=False, edge_choice=False) == 16 + 2 * 88).all()


def test_multi_edge_bytes_add_the_proposal_reads():
    code = S.workload_code("c0")
    base = bench.me_bytes_per_update_table(code, False)
    lmd = bench.me_bytes_per_update_table(code, True)
    np.testing.assert_array_equal(base, bench.lds_bytes_per_update_table(code))
    # Algorithm 6: the CI (4 B) of every VN of the updated VN's two other checks, 5 each
    assert (lmd - base == 4 * 2 * 5).all()


def test_table1_bytes_on_an_irregular_code_match_a_direct_sum():
    code = S.qc_bg1_shaped(4, seed=3)
    t = bench.lds_bytes_per_update_table(code)
    col_ptr, col_row, col_eid = code.csc()
    rp = np.asarray(code.row_ptr)
    rows = code.row_of_edge()
    for e in range(0, code.E, 37):
        n, m = int(code.col[e]), int(rows[e])
        dv = col_ptr[n + 1] - col_ptr[n]
        b = 2 * 4 * dv + 2 * 4 + 3 * 4 + 4
        for i in col_row[col_ptr[n]:col_ptr[n + 1]]:
            if i != m:
                dc = rp[i + 1] - rp[i]
                b += dc * 8 + 2 * 4 * (dc - 1) + (dc - 1) * 16
        assert int(t[e]) == b, e


def test_fer_crossing_interpolates_in_log_fer():
    pts = [(1.0, 1e-1), (1.5, 1e-2), (2.0, 1e-4)]
    assert bench.snr_at_fer(pts, 1e-2) == pytest.approx(1.5)
    assert bench.snr_at_fer(pts, 1e-3) == pytest.approx(1.75)
    assert bench.snr_at_fer(pts, 1e-6) is None           # never reached
    assert bench.snr_at_fer([(1.0, 1e-2), (1.5, 0.0)], 1e-3) == 1.5  # zero errors at the next point


def test_host_cpu_reports_the_share(monkeypatch):
    monkeypatch.setenv("OMP_NUM_THREADS", "3")
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and h["affinity"] >= 1 and h["model"]
    assert h["workers"] == min(3, h["affinity"]) and h["workers_from"] == "OMP_NUM_THREADS"
    monkeypatch.delenv("OMP_NUM_THREADS")
    h = bench.host_cpu()
    assert h["workers"] == h["affinity"] and h["workers_from"] == "affinity"


def test_cpu_baseline_entry_fields():
    def jobs():
        while True:
            yield lambda: (1, 10)
    e = bench.cpu_baseline_entry(jobs, 0.3, "trivial jobs")
    assert e["kind"] == "oracle" and e["unit"] == "frames/s" and e["value"] > 0
    assert e["cores"] == e["host"]["workers"]
    assert e["single_thread"]["frames_per_s"] > 0
    assert e["edge_updates_per_s"] == pytest.approx(10 * e["value"], rel=1e-3)
