"""Pins of the damped-replay oracle and its reverse-mode gradient (CPU only).

The forward is pinned to the main oracle's undamped replay (weights 1: the propagation step of the
single-edge schedules, Sec. II-A steps 3-4, which that oracle evaluates with incrementally
maintained precomputed messages) and to the closed form at weights 0.  The gradient is pinned to
central finite differences of the forward, and the derivative of the pairwise check rule to the
identity d(a [+] b)/da = sinh(a [+] b) / sinh(a).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2102_11089_amd import synth as S


@pytest.fixture(scope="module")
def c0():
    return S.workload_code("c0")


def cirbp_traces(code, llr, T):
    r = O.decode(code, llr, O.CIRBP, O.SPA, max_updates=T, check_every=0, trace=True, threads=4)
    assert np.all(r.updates_used == T)
    return r.trace


def test_boxplus_grad_identity_and_fd():
    rng = np.random.default_rng(0)
    for _ in range(400):
        a, b = rng.uniform(-25, 25, 2) * rng.choice([0.01, 0.3, 1.0], 2)
        g = O.boxplus_grad(a, b)
        p = O.boxplus(a, b)
        assert abs(g - np.sinh(p) / np.sinh(a)) <= 1e-9 * max(1.0, abs(g))
        h = 1e-6 * max(1.0, abs(a))
        fd = (O.boxplus(a + h, b) - O.boxplus(a - h, b)) / (2 * h)
        assert abs(g - fd) <= 1e-6
    assert O.boxplus_grad(0.7, np.inf) == 1.0
    # far in the tail: both factors tiny, ratio finite and exact
    assert abs(O.boxplus_grad(40.0, 39.0) - np.exp(O.boxplus(40.0, 39.0) - 40.0)) < 1e-12


@pytest.mark.parametrize("T", [1, 57, 300])
def test_unit_weights_equal_undamped_replay(c0, T):
    cw, llr = S.frames(c0, 24, 2.0, 5)
    tr = cirbp_traces(c0, llr, T)
    L, c2v = O.unrolled_forward(c0, llr, 1.0, tr)
    ref = O.decode(c0, llr, O.REPLAY, O.SPA, max_updates=T, replay=tr, check_every=0, dump=True)
    np.testing.assert_allclose(L, ref.L, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(c2v, ref.c2v, rtol=1e-12, atol=1e-12)


def test_unit_weights_random_schedule_equal_replay(c0):
    rng = np.random.default_rng(3)
    cw, llr = S.frames(c0, 8, 1.0, 6)
    tr = rng.integers(0, c0.E, size=(8, 200)).astype(np.int32)
    L, c2v = O.unrolled_forward(c0, llr, 1.0, tr)
    ref = O.decode(c0, llr, O.REPLAY, O.SPA, max_updates=200, replay=tr, check_every=0, dump=True)
    np.testing.assert_allclose(L, ref.L, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(c2v, ref.c2v, rtol=1e-12, atol=1e-12)


def test_zero_weights_closed_form(c0):
    """w = 0: nothing moves, d/d llr = gL, and d/d w_e sums gL_n p_e(llr) over the steps on e,
    with p_e the tanh-product form of eq. (2) at c2v = 0."""
    rng = np.random.default_rng(4)
    cw, llr = S.frames(c0, 4, 2.0, 7)
    llr = llr.astype(np.float64)
    tr = rng.integers(0, c0.E, size=(4, 120)).astype(np.int32)
    gL = rng.standard_normal((4, c0.N))
    L, c2v = O.unrolled_forward(c0, llr, 0.0, tr)
    np.testing.assert_array_equal(L, llr)
    np.testing.assert_array_equal(c2v, 0.0)
    g_llr, g_w = O.unrolled_backward(c0, llr, 0.0, tr, gL)
    np.testing.assert_array_equal(g_llr, gL)
    row_of = np.repeat(np.arange(c0.M), np.diff(c0.row_ptr))
    expect = np.zeros((4, c0.E))
    for b in range(4):
        for e in tr[b]:
            m = row_of[e]
            others = [k for k in range(c0.row_ptr[m], c0.row_ptr[m + 1]) if k != e]
            p = 2 * np.arctanh(np.prod(np.tanh(llr[b, c0.col[others]] / 2)))
            expect[b, e] += gL[b, c0.col[e]] * p
    np.testing.assert_allclose(g_w, expect, rtol=1e-10, atol=1e-12)


def _fd_check(code, llr, w, tr, gL, coords_llr, coords_w):
    llr = np.asarray(llr, dtype=np.float64)
    g_llr, g_w = O.unrolled_backward(code, llr, w, tr, gL)
    gw_tot = g_w.sum(0)

    def loss(llr_, w_):
        L, _ = O.unrolled_forward(code, llr_, w_, tr)
        return float(np.sum(gL * L))

    scale = max(np.abs(g_llr).max(), np.abs(gw_tot).max())
    for (b, n) in coords_llr:
        h = 1e-6 * max(1.0, abs(llr[b, n]))
        lp, lm = llr.copy(), llr.copy()
        lp[b, n] += h
        lm[b, n] -= h
        fd = (loss(lp, w) - loss(lm, w)) / (2 * h)
        assert abs(fd - g_llr[b, n]) <= 1e-6 * max(abs(g_llr[b, n]), 1e-2 * scale), (b, n, fd, g_llr[b, n])
    for e in coords_w:
        h = 1e-6 * max(1.0, abs(w[e]))
        wp, wm = w.copy(), w.copy()
        wp[e] += h
        wm[e] -= h
        fd = (loss(llr, wp) - loss(llr, wm)) / (2 * h)
        assert abs(fd - gw_tot[e]) <= 1e-6 * max(abs(gw_tot[e]), 1e-2 * scale), (e, fd, gw_tot[e])


def test_gradient_matches_central_differences_c0(c0):
    rng = np.random.default_rng(8)
    B, T = 3, 300
    cw, llr = S.frames(c0, B, 2.0, 9)
    tr = cirbp_traces(c0, llr, T)
    w = rng.uniform(0.5, 1.2, c0.E)
    gL = rng.standard_normal((B, c0.N))
    used = np.unique(tr)
    coords_llr = [(int(rng.integers(B)), int(rng.integers(c0.N))) for _ in range(64)]
    coords_w = rng.choice(used, 64, replace=False)
    _fd_check(c0, llr, w, tr, gL, coords_llr, coords_w)


def test_gradient_matches_central_differences_n576():
    code = S.workload_code("c4")
    rng = np.random.default_rng(10)
    B, T = 2, 300
    cw, llr = S.frames(code, B, 2.0, 11)
    tr = cirbp_traces(code, llr, T)
    w = rng.uniform(0.7, 1.1, code.E)
    gL = -(1 - 2.0 * cw) / (1 + np.exp((1 - 2.0 * cw) * llr))  # BCE-like weights
    used = np.unique(tr)
    coords_llr = [(int(rng.integers(B)), int(rng.integers(code.N))) for _ in range(64)]
    coords_w = rng.choice(used, 64, replace=False)
    _fd_check(code, llr, w, tr, gL, coords_llr, coords_w)


def test_unused_edges_have_zero_weight_gradient(c0):
    rng = np.random.default_rng(12)
    cw, llr = S.frames(c0, 2, 2.0, 13)
    tr = cirbp_traces(c0, llr, 80)
    g_llr, g_w = O.unrolled_backward(c0, llr, rng.uniform(0.5, 1.5, c0.E), tr, rng.standard_normal((2, c0.N)))
    for b in range(2):
        unused = np.setdiff1d(np.arange(c0.E), tr[b])
        assert np.all(g_w[b, unused] == 0.0)
