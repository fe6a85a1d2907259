"""Pins of the seeded input generators (no decoder arithmetic): the counter-based channel noise
of SNR sweeps against the generator's published known-answer vectors, and its distribution."""
import json
import os

import numpy as np

from paper_2102_11089_amd import synth as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox4x32_10_known_answers():
    doc = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))
    for v in doc["vectors"]:
        ctr = np.array([int(x, 16) for x in v["ctr"]], dtype=np.uint64)
        key = np.array([int(x, 16) for x in v["key"]], dtype=np.uint64)
        out = S.philox4x32_10(ctr, key)
        assert [int(x) for x in out] == [int(x, 16) for x in v["out"]]


def test_philox_awgn_llr_statistics():
    code = S.workload_code("c0")
    cw = S.random_codewords(code, 5, 1)
    s2 = S.sigma2_from_ebn0(2.0, 0.5)
    llr = S.philox_awgn_llr(cw, 4000, s2, seed=123456789012345, point=3)
    c = cw[np.arange(4000) % 5]
    x = 1.0 - 2.0 * c
    z = (llr * s2 / 2.0 - x) / np.sqrt(s2)       # recover the normal draws
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    assert abs(np.mean(z ** 4) - 3.0) < 0.05      # Gaussian kurtosis
    # counters differ per point and per seed
    other = S.philox_awgn_llr(cw, 10, s2, seed=123456789012345, point=4)
    assert not np.allclose(other, llr[:10])
    np.testing.assert_array_equal(S.philox_awgn_llr(cw, 10, s2, seed=123456789012345, point=3), llr[:10])
