"""CI-metric analysis (Sec. III-A, Properties 1-2, Appendix A): the Gaussian-approximation model
against published values and Monte Carlo of the same model, and the decoder's empirical J(gamma)
against the model (no GPU)."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import oracle as O
from paper_2102_11089_amd import ci_analysis as C
from paper_2102_11089_amd import synth as S


def test_phi_matches_published_approximations():
    """Chung, Richardson, Urbanke (2001) approximate Phi by exp(-0.4527 x^0.86 + 0.0218) for
    0 < x < 10 and by sqrt(pi / x) e^(-x/4) (1 - 10 / (7x)) for large x; the quadrature of the
    definition stays within the approximations' own accuracy."""
    for x in (0.1, 0.5, 1.0, 2.0, 5.0, 9.9):
        assert abs(C.phi(x) / math.exp(-0.4527 * x ** 0.86 + 0.0218) - 1) < 0.01, x
    for x in (10.0, 20.0, 40.0):
        approx = math.sqrt(math.pi / x) * math.exp(-x / 4) * (1 - 10 / (7 * x))
        assert abs(C.phi(x) / approx - 1) < 0.03, x
    assert C.phi(0.0) == 1.0 and C.phi(math.inf) == 0.0


def test_phi_monte_carlo_and_inverse():
    rng = np.random.default_rng(1)
    for mu in (0.3, 1.5, 4.0):
        u = rng.normal(mu, math.sqrt(2 * mu), 2_000_000)
        mc = float(np.mean(1.0 - np.tanh(u / 2)))
        assert abs(C.phi(mu) - mc) < 5e-3 * max(mc, 0.05)
    for mu in (1e-3, 0.2, 3.0, 30.0, 300.0):
        assert abs(C.phi_inv(C.phi(mu)) / mu - 1) < 1e-6


def test_ga_de_threshold_of_the_36_ensemble():
    """GA-DE of the (3,6)-regular ensemble: below about 1.16 dB (the GA threshold reported by
    Chung et al.; the exact DE threshold is 1.11 dB) the C2V mean stays bounded, above it grows
    without bound."""
    below = C.ga_de(3, 6, C.channel_mean(1.0, 0.5), 400)
    above = C.ga_de(3, 6, C.channel_mean(1.35, 0.5), 300)
    assert below[-1] < 10 and abs(below[-1] - below[-2]) < 1e-3
    assert above[-1] > 1e3


def _model_mc(mu_l, mu_lt, n, seed):
    rng = np.random.default_rng(seed)
    L = rng.normal(mu_l, math.sqrt(2 * mu_l), n)
    dL = rng.normal(mu_lt - mu_l, math.sqrt(2 * (mu_lt - mu_l)), n)
    return L, L + dL


@pytest.mark.parametrize("it", [1, 2, 3])
def test_ga_j_matches_monte_carlo_of_the_model(it):
    """The integrals for J(gamma) equal a Monte Carlo draw of the same Gaussian model."""
    ml, mlt = C.ga_totals(4, 8, C.channel_mean(2.0, 0.5), it)
    gs = [0.0, 0.05, 0.1, 0.2, 0.3, 0.4]
    L, Lt = _model_mc(ml, mlt, 3_000_000, it)
    mc = C.empirical(L, Lt, gs)["J"]
    np.testing.assert_allclose(C.ga_j(gs, ml, mlt), mc, rtol=0.03)


def test_property1_j_decreases_under_the_model():
    gs = np.linspace(0.0, 0.6, 13)
    for eb in (1.5, 2.0, 3.0):
        for it in (1, 2, 3):
            ml, mlt = C.ga_totals(4, 8, C.channel_mean(eb, 0.5), it)
            J = C.ga_j(gs, ml, mlt)
            assert np.all(np.diff(J) < 0), (eb, it)


def test_property2_f_exceeds_one_and_grows():
    """Appendix B: for P0 = tau < 1/2, F(gamma) > 1, strictly increasing on [0, tau), infinite from
    tau on; the closed form equals a Monte Carlo of the model."""
    for tau in (0.1, 0.3, 0.45):
        for mu_dl in (0.5, 1.5, 4.0):
            gs = np.linspace(0.0, tau, 12, endpoint=False)
            F = C.ga_f(gs, tau, mu_dl)
            assert np.all(F > 1) and np.all(np.diff(F) > 0)
            assert np.isinf(C.ga_f([tau, tau + 0.05], tau, mu_dl)).all()
    rng = np.random.default_rng(3)
    tau, mu_dl = 0.3, 1.5
    lt = np.log(tau / (1 - tau)) + rng.normal(mu_dl, math.sqrt(2 * mu_dl), 2_000_000)
    pt = special.expit(lt)
    for g in (0.0, 0.1, 0.2):
        m = np.abs(pt - tau) >= g
        mc = np.sum(m & (pt >= tau)) / np.sum(m & (pt < tau))
        assert abs(C.ga_f([g], tau, mu_dl)[0] / mc - 1) < 0.03


def test_empirical_counts_by_hand():
    L = np.array([2.0, -1.0, 0.5, -3.0, 0.0])
    Lt = np.array([1.0, 1.0, 0.5, -4.0, -0.1])
    e = C.empirical(L, Lt, [0.0, 0.2])
    # D = |p0(L) - p0(Lt)|: [0.150, 0.462, 0, 0.0294, 0.025]; correct = [1, 0, 1, 0, 1]
    assert list(e["n_correct"]) == [3, 0] and list(e["n_incorrect"]) == [2, 1]
    assert list(e["n_rise"]) == [1, 1] and list(e["n_fall"]) == [1, 0]
    assert e["J"][0] == 1.5 and e["F"][0] == 1.0 and e["J"][1] == 0.0 and np.isinf(e["F"][1])


def test_decoded_j_follows_the_ga_model():
    """Sec. III-A: on a girth-6 (4,8)-regular code at 2 dB, J(gamma) measured from flooding decoding
    (the oracle's) for the first three iterations almost coincides with the GA-DE curves."""
    code = S.qc_regular(4, 8, 250, seed=1)  # N = 2000
    cw, llr = S.frames(code, 300, 2.0, 32, zero_codeword=True)
    gs = [0.0, 0.05, 0.1, 0.2, 0.3]
    mu0 = C.channel_mean(2.0, 0.5)
    for it, tol in ((1, 0.05), (2, 0.06), (3, 0.07)):
        a = O.decode(code, llr, O.FLOODING, O.SPA, max_updates=(it - 1) * code.E, check_every=0, threads=8)
        b = O.decode(code, llr, O.FLOODING, O.SPA, max_updates=it * code.E, check_every=0, threads=8)
        e = C.empirical(a.llr_out, b.llr_out, gs)
        ml, mlt = C.ga_totals(4, 8, mu0, it)
        np.testing.assert_allclose(e["J"], C.ga_j(gs, ml, mlt), rtol=tol)
        assert np.all(e["F"] > 1) and np.all(np.diff(e["F"]) > 0)


def test_irregular_ga_reduces_to_the_regular_recursion():
    mu0 = C.channel_mean(2.0, 0.5)
    np.testing.assert_array_equal(C.ga_de_irregular({4: 1.0}, {8: 1.0}, mu0, 6), C.ga_de(4, 8, mu0, 6))
    gs = [0.0, 0.1, 0.3]
    ml, mlt = C.ga_totals(4, 8, mu0, 2)
    t = C.ga_de(4, 8, mu0, 2)
    np.testing.assert_allclose(C.ga_j_mixture(gs, {4: 1.0}, mu0, t[0], t[1]), C.ga_j(gs, ml, mlt), rtol=1e-12)


def test_degree_mixture_j_matches_monte_carlo():
    """The degree-mixture J(gamma) equals a Monte Carlo draw of the same model (VN degree drawn by
    its node fraction, then L and Lt - L from that degree's Gaussians)."""
    node = {1: 0.5, 3: 0.3, 9: 0.2}
    mu0, tp, tc = 2.0, 0.4, 0.9
    gs = [0.0, 0.05, 0.1, 0.2, 0.3]
    rng = np.random.default_rng(4)
    n = 3_000_000
    d = rng.choice(list(node), p=list(node.values()), size=n)
    ml, md = mu0 + d * tp, d * (tc - tp)
    L = rng.normal(ml, np.sqrt(2 * ml))
    Lt = L + rng.normal(md, np.sqrt(2 * md))
    mc = C.empirical(L, Lt, gs)["J"]
    np.testing.assert_allclose(C.ga_j_mixture(gs, node, mu0, tp, tc), mc, rtol=0.03)


def test_degree_profile_of_a_known_code():
    code = S.code_from_rows(2, 4, [[0, 1, 2], [1, 2, 3]])
    node, lam, rho = C.degree_profile(code)
    assert node == {1: 0.5, 2: 0.5} and lam == {1: 2 / 6, 2: 4 / 6} and rho == {3: 1.0}


def test_decoded_j_on_the_workload_codes():
    """Sec. III-A on the workload codes: on the BG1-shaped Z=52 code at 1.25 dB, J(gamma) measured
    from the oracle's flooding decodes follows the GA-DE model of its degree profile (Chung et al.'s
    irregular recursion, J mixed over VN degrees) for the first two iterations; on both c1 and the
    (3,6) n=96 code J decreases in gamma (Property 1) and F exceeds 1 and grows (Property 2)."""
    gs = [0.0, 0.05, 0.1, 0.2, 0.3]
    for name, eb, frames in (("c1", 1.25, 200), ("c0", 2.0, 3000)):
        code = S.workload_code(name)
        node, lam, rho = C.degree_profile(code)
        cw, llr = S.frames(code, frames, eb, 42, zero_codeword=True)
        mu0 = C.channel_mean(eb, code.design_rate)
        t = np.concatenate([[0.0], C.ga_de_irregular(lam, rho, mu0, 2)])
        for it in (1, 2):
            a = O.decode(code, llr, O.FLOODING, O.SPA, max_updates=(it - 1) * code.E, check_every=0, threads=8)
            b = O.decode(code, llr, O.FLOODING, O.SPA, max_updates=it * code.E, check_every=0, threads=8)
            e = C.empirical(a.llr_out, b.llr_out, gs)
            assert np.all(np.diff(e["J"]) < 0) and np.all(e["F"] > 1) and np.all(np.diff(e["F"]) > 0), (name, it)
            if name == "c1":
                np.testing.assert_allclose(e["J"], C.ga_j_mixture(gs, node, mu0, t[it - 1], t[it]), rtol=0.06)
