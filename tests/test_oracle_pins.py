"""Pins of the CPU oracle against facts fixed by the paper and by mathematics (no GPU).

Each test names the passage it checks.  References that do not come from the oracle itself:
brute-force enumeration of codewords (bitwise MAP / max-log marginals, ML), closed-form operation
counts (Table 1), hand-worked fixtures (Algorithm 4), exact special cases and symmetries.
"""
import json
import os

import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
from paper_2102_11089_amd import synth as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def sigmoid(x):
    """p0(L) = e^L / (1 + e^L), the posterior of bit 0 (Sec. III-A)."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(x >= 0, 1.0 / (1.0 + np.exp(-np.abs(x))), np.exp(-np.abs(x)) / (1.0 + np.exp(-np.abs(x))))


# ------------------------------------------------------------------------------------------
# check rule (eq. (2)) and CI (eq. (9))
# ------------------------------------------------------------------------------------------
def test_spc_one_flooding_pass_is_bitwise_map():
    """On a single parity check, ch_n + C2V_{0->n} is the exact a-posteriori LLR (eq. (2)-(3));
    reference: enumeration of all even-weight words."""
    rng = np.random.default_rng(0)
    for N in (2, 3, 5, 8, 12):
        code = S.spc_code(N)
        H = code.dense()
        cws = brute.codewords(H)
        for _ in range(5):
            llr = rng.normal(1.0, 2.0, size=N) * rng.choice([1, 4], size=N)
            r = O.decode(code, llr, O.FLOODING, O.SPA, max_updates=code.E, check_every=0)
            assert r.updates_used[0] == code.E
            np.testing.assert_allclose(r.llr_out[0], brute.bitwise_map_llr(H, llr, cws), rtol=1e-10, atol=1e-10)


def test_boxplus_matches_tanh_rule_moderate_inputs():
    """Jacobian-log form of eq. (2) equals the literal tanh product where the latter is well conditioned."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, b = rng.uniform(-15, 15, size=2)
        assert abs(O.boxplus(a, b) - O.c2v_tanh([a, b])) <= 1e-9 * max(1.0, abs(O.boxplus(a, b)))
    # large magnitudes: tanh(x/2) rounds to 1 in the literal form, the pairwise form keeps the
    # exact value min + log1p(e^-(a+b)) - log1p(e^-|a-b|)
    assert O.boxplus(60.0, 80.0) == pytest.approx(60.0 - np.log1p(np.exp(-20.0)), abs=1e-12)
    assert O.boxplus(-60.0, 80.0) == pytest.approx(-60.0 + np.log1p(np.exp(-20.0)), abs=1e-12)
    assert O.boxplus(0.0, 5.0) == 0.0


def test_ci_spa_is_posterior_difference():
    """D = |p0(L) - p0(Lt)| (eq. (9)); the oracle's tanh form must agree with p0 computed directly."""
    rng = np.random.default_rng(2)
    for _ in range(500):
        L, Lt = rng.normal(0, 8, size=2)
        d = O.ci_spa(L, Lt)
        assert abs(d - abs(sigmoid(L) - sigmoid(Lt))) < 1e-14
        assert 0.0 <= d < 1.0
    assert O.ci_spa(3.0, 3.0) == 0.0


# ------------------------------------------------------------------------------------------
# initial precompute and the first selection (Algorithm 1 initialisation and selection, RBP step 2)
# ------------------------------------------------------------------------------------------
def test_first_selection_on_spc_matches_bruteforce():
    """On a single check the precomputed C2V into n is the extrinsic MAP LLR, so Lt_n is the
    exact a-posteriori LLR: n* = argmax_n |p0(ch_n) - p0(MAP_n)| (lowest index on ties), and RBP
    picks argmax_n |MAP_n - ch_n|."""
    rng = np.random.default_rng(3)
    for N in (3, 6, 9):
        code = S.spc_code(N)
        H = code.dense()
        cws = brute.codewords(H)
        for _ in range(10):
            llr = rng.normal(0.5, 2.0, size=N)
            mp = brute.bitwise_map_llr(H, llr, cws)
            ci = np.abs(sigmoid(llr) - sigmoid(mp))
            r = O.decode(code, llr, O.CIRBP, O.SPA, max_updates=1, gamma=0.0, trace=True, check_every=0)
            assert r.trace[0, 0] == int(np.argmax(ci))  # edge id = VN index on one row
            r = O.decode(code, llr, O.RBP, O.SPA, max_updates=1, trace=True, check_every=0)
            assert r.trace[0, 0] == int(np.argmax(np.abs(mp - llr)))


# ------------------------------------------------------------------------------------------
# every schedule reaches the exact marginals on cycle-free graphs
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("kind", [O.FLOODING, O.LAYERED, O.RBP, O.CIRBP, O.MECIRBP])
def test_cycle_free_graphs_reach_bitwise_map(kind):
    """BP on a tree converges to the exact bitwise-MAP LLRs whatever the schedule (sum-product)."""
    rng = np.random.default_rng(10 + kind)
    for seed in range(6):
        code = S.random_tree_code(int(rng.integers(2, 6)), seed=seed)
        H = code.dense()
        llr = rng.normal(1.0, 2.5, size=code.N)
        # ME-CIRBP uses the keyed random fill of Algorithm 4: with the lowest-index fill the same
        # low-CI VNs would be chosen for ever once every CI falls in the lowest group
        r = O.decode(code, llr, kind, O.SPA, max_updates=60 * code.E, check_every=0, gamma=0.1,
                     n_p=2, n_g=8, fill=O.FILL_HASH, seed=seed)
        np.testing.assert_allclose(r.llr_out[0], brute.bitwise_map_llr(H, llr), rtol=1e-9, atol=1e-9)


def maxlog_marginals(H, ch):
    """Max-log marginals: max_{c: c_n=0} S(c) - max_{c: c_n=1} S(c), S(c) = sum (1-2c_k) ch_k / 2."""
    cws = brute.codewords(H)
    score = 0.5 * ((1.0 - 2.0 * cws) @ ch)
    return np.array([score[cws[:, n] == 0].max() - score[cws[:, n] == 1].max() for n in range(H.shape[1])])


@pytest.mark.parametrize("kind", [O.FLOODING, O.LAYERED, O.RBP, O.CIRBP, O.MECIRBP])
def test_cycle_free_graphs_min_sum_reaches_maxlog(kind):
    """Min-sum (Sec. V) on a tree converges to the max-log marginals; integer channel, no saturation
    (16-bit messages), so the match is exact."""
    rng = np.random.default_rng(20 + kind)
    for seed in range(6):
        code = S.random_tree_code(int(rng.integers(2, 6)), seed=100 + seed)
        H = code.dense()
        ch = rng.integers(-12, 13, size=code.N).astype(np.float64)
        r = O.decode(code, ch, kind, O.MSFIX, q_bits=16, frac_bits=0, max_updates=60 * code.E,
                     check_every=0, gamma=0.1, n_p=2, n_g=8, fill=O.FILL_HASH, seed=seed)
        np.testing.assert_array_equal(r.llr_out[0], maxlog_marginals(H, ch))


# ------------------------------------------------------------------------------------------
# first flooding iteration on a loopy code: every check is an independent SPC
# ------------------------------------------------------------------------------------------
def test_first_flooding_iteration_loopy_code():
    code = S.workload_code("c0")
    rng = np.random.default_rng(4)
    llr = rng.normal(1.5, 2.0, size=code.N)
    expect = llr.copy()
    for m in range(code.M):
        vs = code.col[code.row_ptr[m]:code.row_ptr[m + 1]]
        H1 = np.ones((1, len(vs)), dtype=np.uint8)
        expect[vs] += brute.bitwise_map_llr(H1, llr[vs]) - llr[vs]
    r = O.decode(code, llr, O.FLOODING, O.SPA, max_updates=code.E, check_every=0)
    np.testing.assert_allclose(r.llr_out[0], expect, rtol=1e-10, atol=1e-10)


# ------------------------------------------------------------------------------------------
# Table 1: per-update operation counts (closed form on a (3,6)-regular code)
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("arith", [O.SPA, O.MSFIX])
def test_table1_counts_regular_code(arith):
    code = S.workload_code("c0")
    cw, llr = S.frames(code, 40, 1.0, 5)
    for kind in (O.RBP, O.CIRBP):
        r = O.decode(code, llr, kind, arith, max_updates=600, gamma=0.1)
        u = r.updates_used
        assert np.all(r.counter("prop") == u)
        assert np.all(r.counter("v2c") == 2 * u)        # d_v - 1
        assert np.all(r.counter("pre") == 10 * u)       # (d_v - 1)(d_c - 1)
        assert np.all(r.counter("ci") == 10 * u)        # (d_v - 1)(d_c - 1)
        assert np.all(r.counter("ci_self") == u)
        if kind == O.RBP:
            assert np.all(r.counter("cmp") == (code.E - 1) * u)
        else:
            k = r.counter("fallback")
            # N - 1 + 1 comparisons for the CI argmax and the threshold test, then E - 1 or d_v - 1
            assert np.all(r.counter("cmp") == code.N * u + k * (code.E - 1) + (u - k) * 2)


# ------------------------------------------------------------------------------------------
# special cases and equivalences
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("arith", [O.SPA, O.MSFIX])
def test_cirbp_large_gamma_is_rbp(arith):
    """D < 1 always (eq. (9)), so gamma > 1 makes every CIRBP update the RBP fallback."""
    code = S.workload_code("c0")
    cw, llr = S.frames(code, 30, 2.0, 6)
    a = O.decode(code, llr, O.CIRBP, arith, max_updates=800, gamma=1.01, trace=True)
    b = O.decode(code, llr, O.RBP, arith, max_updates=800, trace=True)
    np.testing.assert_array_equal(a.trace, b.trace)
    np.testing.assert_array_equal(a.bits, b.bits)
    np.testing.assert_array_equal(a.updates_used, b.updates_used)
    assert np.all(a.counter("fallback") == a.updates_used)


def test_cirbp_gamma_zero_never_falls_back():
    code = S.workload_code("c0")
    cw, llr = S.frames(code, 30, 2.0, 7)
    for arith in (O.SPA, O.MSFIX):
        r = O.decode(code, llr, O.CIRBP, arith, max_updates=800, gamma=0.0)
        assert np.all(r.counter("fallback") == 0)


def test_me_single_vn_equals_cirbp_gamma_zero_fixed_point():
    """With N_P = 1 and one group per CI level, Algorithm 4 returns the lowest-index VN of maximum
    CI, so Algorithm 5 is Algorithm 1 with gamma = 0 (bit-exact in fixed point)."""
    code = S.workload_code("c0")
    cw, llr = S.frames(code, 40, 2.0, 8)
    a = O.decode(code, llr, O.MECIRBP, O.MSFIX, max_updates=900, n_p=1, n_g=65535, trace=True)
    b = O.decode(code, llr, O.CIRBP, O.MSFIX, max_updates=900, gamma=0.0, trace=True)
    np.testing.assert_array_equal(a.trace, b.trace)
    np.testing.assert_array_equal(a.updates_used, b.updates_used)
    np.testing.assert_array_equal(a.llr_out, b.llr_out)


def test_me_disjoint_selection_equals_sequential():
    """When the selected VNs have pairwise disjoint two-hop neighbourhoods, one ME step equals the
    single-edge updates applied one after the other (replayed in the same order)."""
    # two disconnected copies of a small code: each VN's neighbourhood stays in its copy
    base = S.workload_code("c0")
    rows = []
    for off in (0, base.N):
        for m in range(base.M):
            rows.append(list(base.col[base.row_ptr[m]:base.row_ptr[m + 1]] + off))
    code = S.code_from_rows(2 * base.M, 2 * base.N, rows)
    rng = np.random.default_rng(9)
    checked = 0
    for trial in range(30):
        llr = rng.normal(1.0, 2.0, size=code.N)
        # one ME step with N_P = 2 and a single group chooses the two lowest indices 0 and 1 ...
        # instead force one VN per copy: N_G large, and keep only trials whose selection splits
        me = O.decode(code, llr, O.MECIRBP, O.SPA, max_updates=2, n_p=2, n_g=1 << 20, trace=True,
                      check_every=0, dump=True)
        e = me.trace[0, :2]
        n = code.col[e]
        if not ((n[0] < base.N) ^ (n[1] < base.N)):
            continue
        rep = O.decode(code, llr, O.REPLAY, O.SPA, max_updates=2, replay=e[None], dump=True)
        np.testing.assert_allclose(me.c2v, rep.c2v, atol=1e-12)
        np.testing.assert_allclose(me.L, rep.L, atol=1e-12)
        np.testing.assert_allclose(me.Lt, rep.Lt, atol=1e-12)
        np.testing.assert_allclose(me.D, rep.D, atol=1e-12)
        checked += 1
    assert checked >= 5


@pytest.mark.parametrize("arith", [O.SPA, O.MSFIX])
def test_replay_reproduces_schedule(arith):
    code = S.workload_code("c0")
    cw, llr = S.frames(code, 20, 2.0, 10)
    a = O.decode(code, llr, O.CIRBP, arith, max_updates=1000, trace=True, dump=True)
    for f in range(20):
        t = int(a.updates_used[f])
        rep = O.decode(code, llr[f], O.REPLAY, arith, max_updates=t, replay=a.trace[f:f + 1, :t], dump=True)
        np.testing.assert_array_equal(rep.llr_out[0], a.llr_out[f])
        np.testing.assert_array_equal(rep.c2v[0], a.c2v[f])


def test_replay_ends_at_an_invalid_edge_id():
    """A recorded order padded with -1 after the frame stopped (the layout of a trace row) replays
    to that point and no further: same updates used, same final state as the recording."""
    code = S.workload_code("c0")
    cw, llr = S.frames(code, 12, 2.0, 12)
    a = O.decode(code, llr, O.CIRBP, O.SPA, max_updates=1000, trace=True, dump=True)
    assert (a.updates_used < 1000).any()
    rep = O.decode(code, llr, O.REPLAY, O.SPA, max_updates=1000, replay=a.trace, dump=True)
    np.testing.assert_array_equal(rep.updates_used, a.updates_used)
    np.testing.assert_array_equal(rep.llr_out, a.llr_out)
    np.testing.assert_array_equal(rep.c2v, a.c2v)
    bad = a.trace.copy()
    bad[:, 5] = code.E  # out of range from the sixth update on
    rep = O.decode(code, llr, O.REPLAY, O.SPA, max_updates=1000, replay=bad)
    np.testing.assert_array_equal(rep.updates_used, np.minimum(a.updates_used, 5))


def test_stop_rule_first_valid_codeword():
    """Sec. II-A: decoding stops at the first update after which the hard decisions form a codeword
    (here tested after every update); checked with H from scratch on replayed prefixes."""
    code = S.workload_code("c0")
    Hd = code.dense().astype(np.int64)
    cw, llr = S.frames(code, 30, 2.5, 11)
    a = O.decode(code, llr, O.CIRBP, O.SPA, max_updates=1500, trace=True)
    for f in range(30):
        t = int(a.updates_used[f])
        if t == 1500:
            continue
        assert not np.any((Hd @ a.bits[f]) % 2)
        if t == 0:
            assert not np.any((Hd @ (llr[f] < 0).astype(np.int64)) % 2)
            continue
        prev = O.decode(code, llr[f], O.REPLAY, O.SPA, max_updates=t - 1, replay=a.trace[f:f + 1, :t - 1])
        assert np.any((Hd @ prev.bits[0]) % 2)


# ------------------------------------------------------------------------------------------
# invariants
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("kind", [O.RBP, O.CIRBP, O.MECIRBP])
@pytest.mark.parametrize("arith", [O.SPA, O.MSFIX])
def test_incremental_state_equals_definitions(kind, arith):
    """After every update the maintained precomputed messages, Lt, D and syndrome equal their
    definitions recomputed from (c2v, L); 0 <= D < 1 (eq. (9))."""
    code = S.workload_code("c0")
    cw, llr = S.frames(code, 6, 1.5, 12)
    O.decode(code, llr, kind, arith, max_updates=400, selfcheck=True, n_p=4)


def test_sign_symmetry_spa():
    """Sum-product decoding commutes with flipping the channel signs on a codeword's support: the
    outputs flip on that support and the schedule is unchanged (exact arithmetic symmetry)."""
    code = S.workload_code("c0")
    cw, llr = S.frames(code, 20, 2.0, 13)
    flip = (1.0 - 2.0 * cw)
    llr0 = llr * flip  # channel for the all-zero codeword with the same noise
    for kind in (O.RBP, O.CIRBP, O.MECIRBP, O.FLOODING, O.LAYERED):
        mu = 50 * code.E if kind in (O.FLOODING, O.LAYERED) else 1200
        a = O.decode(code, llr, kind, O.SPA, max_updates=mu, n_p=4, trace=kind >= O.RBP)
        b = O.decode(code, llr0, kind, O.SPA, max_updates=mu, n_p=4, trace=kind >= O.RBP)
        np.testing.assert_array_equal(a.updates_used, b.updates_used)
        np.testing.assert_array_equal(a.llr_out, b.llr_out * flip)
        if kind >= O.RBP:
            np.testing.assert_array_equal(a.trace, b.trace)


def test_fixed_point_ci_table_tracks_posteriors():
    """The p0 look-up table used in fixed point (Sec. V-B) approximates D = |p0(L) - p0(Lt)| to
    within one table step: |D_q / 65534 - D(L 2^-f, Lt 2^-f)| <= 1 / 65534."""
    code = S.workload_code("c0")
    cw, llr = S.frames(code, 10, 1.0, 14)
    r = O.decode(code, llr, O.CIRBP, O.MSFIX, max_updates=300, dump=True, frac_bits=1)
    L = r.L * 0.5
    Lt = r.Lt * 0.5
    D = np.abs(sigmoid(np.clip(L, -64, 64)) - sigmoid(np.clip(Lt, -64, 64)))
    assert np.all(np.abs(r.D / 65534.0 - D) <= 1.0 / 65534 + 1e-12)
    assert np.all(r.D == np.round(r.D)) and np.all(r.D >= 0) and np.all(r.D <= 65534)


def test_high_snr_decodes_without_errors():
    code = S.workload_code("c0")
    for zero in (True, False):
        cw, llr = S.frames(code, 300, 8.0, 15, zero_codeword=zero)
        for kind in (O.CIRBP, O.RBP, O.FLOODING, O.LAYERED, O.MECIRBP):
            for arith in (O.SPA, O.MSFIX):
                mu = 50 * code.E if kind in (O.FLOODING, O.LAYERED) else 2400
                r = O.decode(code, llr, kind, arith, max_updates=mu, n_p=4, threads=4)
                assert np.array_equal(r.bits, cw), (kind, arith, zero)


def test_ml_and_map_lower_bound_bp():
    """No decoder beats ML in frame errors or bitwise MAP in bit errors (statistical, K = 12)."""
    code = S.peg_regular(24, 3, 6, seed=5)
    H = code.dense()
    cws = brute.codewords(H)
    cw, llr = S.frames(code, 1500, 1.5, 16)
    ml_err = sum(np.any(brute.ml_codeword(H, l, cws) != c) for l, c in zip(llr, cw))
    map_bits = np.array([brute.bitwise_map_llr(H, l, cws) < 0 for l in llr])
    map_ber = np.mean(map_bits != cw)
    for kind in (O.CIRBP, O.RBP, O.FLOODING):
        mu = 50 * code.E if kind == O.FLOODING else 20 * code.E
        r = O.decode(code, llr, kind, O.SPA, max_updates=mu, threads=4)
        bp_err = np.sum(np.any(r.bits != cw, axis=1))
        assert ml_err <= bp_err + 3
        assert map_ber <= np.mean(r.bits != cw) + 1e-3


# ------------------------------------------------------------------------------------------
# Algorithm 4 (golden, worked by hand)
# ------------------------------------------------------------------------------------------
def test_alg4_hand_worked_cases():
    g = json.load(open(os.path.join(GOLDEN, "alg4_select.json")))
    D = np.array(g["D"])
    bins = np.minimum(np.floor(D * g["n_g"]).astype(np.int32), g["n_g"] - 1)
    for case in g["cases"]:
        assert list(O.alg4_select(bins, g["n_g"], case["n_p"])) == case["expect"], case["why"]


def test_splitmix64_published_reference_values():
    """SplitMix64 (Steele, Lea, Flood 2014), reference outputs of the generator seeded with 0:
    the first three outputs of the stream are the function applied to 0, gamma, 2 gamma."""
    g = 0x9E3779B97F4A7C15
    assert O.splitmix64(0) == 0xE220A8397B1DCDAF
    assert O.splitmix64(g) == 0x6E789E6AA1B965F4
    assert O.splitmix64((2 * g) & (2**64 - 1)) == 0x06C45D188009454F


def test_alg4_keyed_fill_takes_smallest_keys():
    g = json.load(open(os.path.join(GOLDEN, "alg4_select.json")))
    D = np.array(g["D"])
    bins = np.minimum(np.floor(D * g["n_g"]).astype(np.int32), g["n_g"] - 1)
    keys = np.array([O.fill_key(7, 0, 3, n) for n in range(len(D))], dtype=np.uint64)
    # n_p = 4: Q(1) = {1, 2, 4}, one more from G2 = {5, 6}: the one with the smaller key
    expect = sorted([1, 2, 4] + [5 if keys[5] < keys[6] else 6])
    assert list(O.alg4_select_keyed(bins, g["n_g"], 4, keys)) == expect
    # n_p = 2: two of G3 = {1, 2, 4} with the smallest keys
    top = sorted([1, 2, 4], key=lambda n: (int(keys[n]), n))[:2]
    assert list(O.alg4_select_keyed(bins, g["n_g"], 2, keys)) == sorted(top)


# ------------------------------------------------------------------------------------------
# LMD schedules (Sec. IV, Algorithms 2 and 3; degree-1 rule of Sec. V)
# ------------------------------------------------------------------------------------------
LMD_KINDS = (O.LMDRBP, O.SLMDRBP, O.LMDCIRBP)


def _spc_extrinsic(x):
    """C2V messages of one check whose incoming V2C messages are x: the extrinsic part of the
    exact single-parity-check posterior, by codeword enumeration."""
    d = len(x)
    H1 = np.ones((1, d), dtype=np.uint8)
    return brute.bitwise_map_llr(H1, x) - np.asarray(x, dtype=np.float64)


def _lmd_first_two(code, ch, kind):
    """The first two edges an LMD schedule sends, from the definitions alone: every precomputed
    C2V message by enumeration on its check, Lt_n = ch_n + sum of precomputed messages into n,
    D_n = |p0(L_n) - p0(Lt_n)| (eq. (9)).  Returns (e1, e2, margin): margin is the smallest gap
    between the winning value and the runner-up in the argmaxes taken, so that callers can skip
    cases that rounding could decide."""
    rows = code.row_of_edge()
    E = code.E
    rp, col = code.row_ptr, code.col

    def precompute(v2c_of):
        pre = np.zeros(E)
        for m in range(code.M):
            sl = slice(rp[m], rp[m + 1])
            pre[sl] = _spc_extrinsic(v2c_of(m, col[sl]))
        return pre

    margins = []

    def argmax(vals, ids):
        # largest value, lowest id on ties (the ids are ascending edge ids or VN indices)
        vals = np.asarray(vals, dtype=np.float64)
        order = np.lexsort((np.asarray(ids), -vals))
        u = np.unique(vals)
        if len(u) > 1:
            margins.append(u[-1] - u[-2])
        return int(np.asarray(ids)[order[0]])

    pre0 = precompute(lambda m, vs: ch[vs])
    c2v = np.zeros(E)
    Lt0 = ch + np.bincount(col, weights=pre0, minlength=code.N)
    D0 = np.abs(sigmoid(ch) - sigmoid(Lt0))
    res0 = np.abs(pre0 - c2v)

    def into(n, res):
        es = np.nonzero(col == n)[0]
        return argmax(res[es], es)

    if kind == O.LMDCIRBP:
        e1 = into(argmax(D0, np.arange(code.N)), res0)
    else:
        e1 = argmax(res0, np.arange(E))
    ms, ns = int(rows[e1]), int(col[e1])
    c2v[e1] = pre0[e1]
    L = ch.copy()
    L[ns] = ch[ns] + pre0[e1]
    touched = [int(r) for r in rows[col == ns] if r != ms]
    pre1 = pre0.copy()
    for m in touched:
        sl = slice(rp[m], rp[m + 1])
        vs = col[sl]
        pre1[sl] = _spc_extrinsic(np.where(vs == ns, L[ns], ch[vs]))  # c2v into row m is 0
    res1 = np.abs(pre1 - c2v)
    Lt1 = ch + np.bincount(col, weights=pre1, minlength=code.N)
    D1 = np.abs(sigmoid(L) - sigmoid(Lt1))
    cand_rows = touched if touched else [ms]  # degree-1 n*: search N(m*) \ n* (Sec. V)
    cand = np.array([e for m in cand_rows for e in range(rp[m], rp[m + 1]) if col[e] != ns])
    if kind == O.LMDCIRBP:
        vs = col[cand]
        e2 = into(argmax(D1[vs], vs), res1)
    else:
        e = argmax(res1[cand], cand)
        e2 = e if kind == O.SLMDRBP else into(int(col[e]), res1)
    return e1, e2, min(margins) if margins else np.inf


def _small_mixed_code():
    """Four checks of degree 4 on 10 VNs, any two checks sharing one VN: VNs 3, 6, 8 and 9 have
    degree 1, the others degree 2 (no 4-cycles)."""
    return S.code_from_rows(4, 10, [[0, 1, 2, 3], [0, 4, 5, 6], [1, 4, 7, 8], [2, 5, 7, 9]])


@pytest.mark.parametrize("kind", LMD_KINDS)
def test_lmd_first_two_choices_match_enumeration(kind):
    """Algorithms 2 and 3: the global first choice and the local second one (after the latest
    update, among the messages of the checks that just received new V2C messages; from m* itself
    when n* has degree 1), recomputed by codeword enumeration on each check."""
    rng = np.random.default_rng(40 + kind)
    seen_deg1 = seen_deg2 = 0
    for code in (_small_mixed_code(), S.workload_code("c0")):
        deg = np.bincount(code.col, minlength=code.N)
        for trial in range(25 if code.N < 20 else 8):
            ch = rng.normal(0.8, 2.0, size=code.N)
            e1, e2, margin = _lmd_first_two(code, ch, kind)
            if margin < 1e-9:
                continue
            r = O.decode(code, ch, kind, O.SPA, max_updates=2, check_every=0, trace=True)
            assert list(r.trace[0, :2]) == [e1, e2], (code.name, trial)
            if deg[code.col[e1]] == 1:
                seen_deg1 += 1
            else:
                seen_deg2 += 1
    assert seen_deg1 >= 3 and seen_deg2 >= 10


@pytest.mark.parametrize("kind", LMD_KINDS)
@pytest.mark.parametrize("arith", [O.SPA, O.MSFIX])
def test_lmd_on_a_single_check_follows_the_global_schedule(kind, arith):
    """On one check every VN has degree 1, so the LMD search covers N(m*) \\ n* (Sec. V); an update
    changes no other message there and leaves the sent edge with residual 0 and its VN with D = 0.
    While unsent edges keep positive residuals and CIs, the local maximum is the global one:
    LMDRBP and sLMDRBP send what RBP sends and LMD-CIRBP what CIRBP with gamma = 0 sends.  In
    fixed point (small integer channel values, min-sum) most residuals tie, which pins the
    lowest-index rule for ties."""
    rng = np.random.default_rng(50 + kind + 10 * arith)
    for N in (3, 5, 8):
        code = S.spc_code(N)
        for _ in range(6):
            if arith == O.SPA:
                ch = rng.normal(0.5, 2.0, size=N)
            else:
                ch = rng.choice([-3.0, -2.0, -1.0, 1.0, 2.0, 3.0], size=N)
            ref_kind = O.CIRBP if kind == O.LMDCIRBP else O.RBP
            a = O.decode(code, ch, kind, arith, max_updates=N, check_every=0, trace=True, frac_bits=0)
            b = O.decode(code, ch, ref_kind, arith, max_updates=N, check_every=0, trace=True, gamma=0.0,
                         frac_bits=0)
            np.testing.assert_array_equal(a.trace, b.trace)
            assert sorted(a.trace[0]) == list(range(N))  # every edge once


@pytest.mark.parametrize("arith", [O.SPA, O.MSFIX])
def test_table1_counts_lmd_regular_code(arith):
    """Table 1 on a (3,6)-regular code: after each propagation sLMDRBP makes
    (d_v - 1)(d_c - 1) - 1 = 9 comparisons, LMDRBP and LMD-CIRBP (d_v - 1) d_c - 1 = 11; the
    first choice is global (E - 1 residual comparisons, or N - 1 CI comparisons plus d_v - 1)."""
    code = S.workload_code("c0")
    cw, llr = S.frames(code, 40, 1.0, 5)
    first = {O.LMDRBP: code.E - 1, O.SLMDRBP: code.E - 1, O.LMDCIRBP: code.N - 1 + 2}
    per = {O.LMDRBP: 11, O.SLMDRBP: 9, O.LMDCIRBP: 11}
    for kind in LMD_KINDS:
        r = O.decode(code, llr, kind, arith, max_updates=600)
        u = r.updates_used
        assert np.all(r.counter("prop") == u)
        assert np.all(r.counter("pre") == 10 * u)
        assert np.all(r.counter("cmp") == np.where(u > 0, first[kind], 0) + per[kind] * u)
        assert np.all(r.counter("fallback") == 0)


@pytest.mark.parametrize("kind", LMD_KINDS)
@pytest.mark.parametrize("arith", [O.SPA, O.MSFIX])
def test_lmd_incremental_state_equals_definitions(kind, arith):
    """The state kept by the LMD schedules equals its definitions after every update (the same
    self-check as the other single-edge schedules), on a code with degree-1 VNs too."""
    for name in ("c0", "bg"):
        code = S.workload_code("c0") if name == "c0" else S.qc_bg1_shaped(4, seed=3)
        cw, llr = S.frames(code, 4, 1.5, 17, zero_codeword=True)
        O.decode(code, llr, kind, arith, max_updates=300, selfcheck=True)


def test_lmd_sign_symmetry_spa():
    """As for the other schedules: flipping the channel signs on a codeword's support flips the
    outputs there and leaves the LMD schedule unchanged."""
    code = S.workload_code("c0")
    cw, llr = S.frames(code, 20, 2.0, 18)
    flip = (1.0 - 2.0 * cw)
    for kind in LMD_KINDS:
        a = O.decode(code, llr, kind, O.SPA, max_updates=1200, trace=True)
        b = O.decode(code, llr * flip, kind, O.SPA, max_updates=1200, trace=True)
        np.testing.assert_array_equal(a.trace, b.trace)
        np.testing.assert_array_equal(a.llr_out, b.llr_out * flip)


def test_lmd_high_snr_decodes_without_errors():
    code = S.workload_code("c0")
    cw, llr = S.frames(code, 300, 8.0, 19)
    for kind in LMD_KINDS:
        for arith in (O.SPA, O.MSFIX):
            r = O.decode(code, llr, kind, arith, max_updates=2400, threads=4)
            assert np.array_equal(r.bits, cw), (kind, arith)


# ------------------------------------------------------------------------------------------
# ME-LMD-CIRBP (Algorithm 6)
# ------------------------------------------------------------------------------------------
def test_alg4_with_excluded_vns_hand_worked():
    """Algorithm 6 refills P' with Algorithm 4 run on the VNs outside P' (hand-worked cases)."""
    g = json.load(open(os.path.join(GOLDEN, "alg4_select.json")))
    D = np.array(g["D"])
    bins = np.minimum(np.floor(D * g["n_g"]).astype(np.int32), g["n_g"] - 1)
    for case in g["excl_cases"]:
        excl = np.zeros(len(D), dtype=np.uint8)
        excl[case["excl"]] = 1
        assert list(O.alg4_select_excl(bins, g["n_g"], case["n_p"], excl)) == case["expect"], case["why"]


def test_me_lmd_single_vn_equals_lmd_cirbp_fixed_point():
    """With N_P = 1 and one group per CI level, Algorithm 4 picks the VN of largest CI (lowest index
    on ties) and every later set is the single proposal p' of Algorithm 3: Algorithm 6 is LMD-CIRBP,
    bit-exact in fixed point (an ME step's recomputation of m*'s row changes nothing there)."""
    code = S.workload_code("c0")
    cw, llr = S.frames(code, 40, 2.0, 21)
    a = O.decode(code, llr, O.MELMDCIRBP, O.MSFIX, max_updates=900, n_p=1, n_g=65535, trace=True, dump=True)
    b = O.decode(code, llr, O.LMDCIRBP, O.MSFIX, max_updates=900, trace=True, dump=True)
    np.testing.assert_array_equal(a.trace, b.trace)
    np.testing.assert_array_equal(a.updates_used, b.updates_used)
    np.testing.assert_array_equal(a.llr_out, b.llr_out)
    np.testing.assert_array_equal(a.D, b.D)


def test_me_lmd_disjoint_copies_follow_lmd_cirbp_each():
    """Two disconnected copies of a code, N_P = 2: when the first set takes one VN per copy, the
    proposals stay one per copy, so each copy runs LMD-CIRBP on its own (fixed point, exact CI
    groups).  Ties for the first set are avoided by keeping only trials that split."""
    base = S.workload_code("c0")
    rows = []
    for off in (0, base.N):
        for m in range(base.M):
            rows.append(list(base.col[base.row_ptr[m]:base.row_ptr[m + 1]] + off))
    code = S.code_from_rows(2 * base.M, 2 * base.N, rows)
    rng = np.random.default_rng(22)
    T = 120
    checked = 0
    for trial in range(30):
        llr = rng.normal(1.0, 2.0, size=code.N)
        me = O.decode(code, llr, O.MELMDCIRBP, O.MSFIX, max_updates=T, n_p=2, n_g=65535, check_every=0,
                      trace=True)
        e0 = me.trace[0, :2]
        if not ((code.col[e0[0]] < base.N) and (code.col[e0[1]] >= base.N)):
            continue
        a = O.decode(base, llr[:base.N], O.LMDCIRBP, O.MSFIX, max_updates=T // 2, check_every=0, trace=True)
        b = O.decode(base, llr[base.N:], O.LMDCIRBP, O.MSFIX, max_updates=T // 2, check_every=0, trace=True)
        np.testing.assert_array_equal(me.trace[0, 0::2], a.trace[0])
        np.testing.assert_array_equal(me.trace[0, 1::2] - base.E, b.trace[0])
        checked += 1
    assert checked >= 5


@pytest.mark.parametrize("fill", [O.FILL_LOWEST, O.FILL_HASH])
def test_me_lmd_every_step_updates_n_p_distinct_vns(fill):
    """Repeated proposals are merged and Algorithm 4 refills the set, so every step updates exactly
    N_P distinct VNs."""
    code = S.workload_code("c0")
    cw, llr = S.frames(code, 20, 1.5, 23)
    n_p = 8
    r = O.decode(code, llr, O.MELMDCIRBP, O.SPA, max_updates=800, n_p=n_p, n_g=16, fill=fill, seed=5,
                 check_every=0, trace=True)
    assert np.all(r.updates_used == 800) and np.all(r.steps_used == 100)
    vn = code.col[r.trace]
    for f in range(vn.shape[0]):
        steps = vn[f].reshape(-1, n_p)
        assert all(len(set(s)) == n_p for s in steps)
        assert np.all(np.diff(steps, axis=1) > 0)  # ascending VN order within a step


@pytest.mark.parametrize("arith", [O.SPA, O.MSFIX])
def test_me_lmd_incremental_state_equals_definitions(arith):
    for code in (S.workload_code("c0"), S.qc_bg1_shaped(4, seed=3)):
        cw, llr = S.frames(code, 4, 1.5, 24, zero_codeword=True)
        O.decode(code, llr, O.MELMDCIRBP, arith, max_updates=400, selfcheck=True, n_p=4, n_g=8, fill=O.FILL_HASH)


def test_me_lmd_sign_symmetry_and_high_snr():
    code = S.workload_code("c0")
    cw, llr = S.frames(code, 20, 2.0, 25)
    flip = (1.0 - 2.0 * cw)
    a = O.decode(code, llr, O.MELMDCIRBP, O.SPA, max_updates=1200, n_p=4, trace=True)
    b = O.decode(code, llr * flip, O.MELMDCIRBP, O.SPA, max_updates=1200, n_p=4, trace=True)
    np.testing.assert_array_equal(a.trace, b.trace)
    np.testing.assert_array_equal(a.llr_out, b.llr_out * flip)
    cw, llr = S.frames(code, 200, 8.0, 26)
    for arith in (O.SPA, O.MSFIX):
        r = O.decode(code, llr, O.MELMDCIRBP, arith, max_updates=2400, n_p=4, fill=O.FILL_HASH, threads=4)
        assert np.array_equal(r.bits, cw)
