"""Analysis of the conditional-innovation metric (Sec. III-A, Properties 1 and 2, Appendix A).

The CI of a VN is D = |p0(L) - p0(Lt)| (eq. (9)), with L its total LLR and Lt the total it would
have after the pending update.  Under the all-zero codeword, a decision is correct iff p0(L) >= 1/2.

* Property 1: J(gamma) = Pr(correct | D >= gamma) / Pr(incorrect | D >= gamma) decreases in gamma.
* Property 2: for an incorrect decision, F(gamma) = Pr(p0(Lt) >= p0(L) | D >= gamma) /
  Pr(p0(Lt) < p0(L) | D >= gamma) exceeds 1 and grows with gamma.

Two ways to evaluate them:

* ``ga_*``: the Gaussian-approximation density evolution (GA-DE) model of Appendix A for a
  (d_v, d_c)-regular ensemble under flooding.  Messages are consistent Gaussians N(mu, 2 mu); the
  means follow mu_C = Phi^-1(1 - [1 - Phi(mu_V)]^(d_c - 1)), mu_V = mu_0 + (d_v - 1) mu_C, with Phi
  as defined by Chung, Richardson and Urbanke (2001), evaluated here from that definition by
  quadrature.  L ~ N(mu_L, 2 mu_L) with mu_L = mu_0 + d_v mu_C at iteration l; the precomputed
  total is the next iteration's, and the difference is modelled as an independent
  N(mu_dL, 2 mu_dL), mu_dL = mu_Lt - mu_L.  J is the ratio of its two conditional probabilities
  integrated over the whole range of L (see the readings of the paper in the design notes).
* ``empirical``: counts over decoded frames.  At flooding iteration l (l = 1, 2, ...) L is the
  total after l - 1 iterations and Lt the total after l, which is what the iteration's precomputed
  messages give; ``flooding_states`` obtains both from the GPU flooding decoder (no early stop).

The GA functions are plain numerical analysis (numpy/scipy) and the statistics are counts over
decoder outputs; neither is part of the decoding path.
"""
from __future__ import annotations

import math
from functools import lru_cache
from typing import Dict, Sequence

import numpy as np
from scipy import integrate, special

# ----------------------------------------------------------------------------------------------
# Gaussian approximation
# ----------------------------------------------------------------------------------------------


@lru_cache(maxsize=65536)
def phi(mu: float) -> float:
    """Phi(mu) = 1 - E[tanh(u / 2)], u ~ N(mu, 2 mu) (Chung, Richardson, Urbanke 2001, Definition 1);
    Phi(0) = 1.  Evaluated as E[2 / (1 + e^u)], which keeps its small values accurate."""
    mu = float(mu)
    if mu <= 0.0:
        return 1.0
    if math.isinf(mu):
        return 0.0
    s = math.sqrt(2.0 * mu)

    def f(z):  # z ~ N(0, 1), u = mu + s z
        u = mu + s * z
        return 2.0 * special.expit(-u) * math.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)

    lo, hi = -12.0, 12.0
    z0 = -mu / s  # where u = 0: the integrand's knee
    pts = [z0] if lo < z0 < hi else None
    val, _ = integrate.quad(f, lo, hi, limit=400, epsabs=0.0, epsrel=1e-11, points=pts)
    return val


def phi_inv(y: float) -> float:
    """The mu >= 0 with Phi(mu) = y, y in (0, 1] (Phi decreases strictly): bisection in log mu."""
    if y >= 1.0:
        return 0.0
    if y <= 0.0:
        return math.inf
    lo, hi = 1e-12, 1.0
    while phi(hi) > y:
        hi *= 2.0
        if hi > 1e6:
            return math.inf
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if phi(mid) > y:
            lo = mid
        else:
            hi = mid
        if hi / lo < 1.0 + 1e-13:
            break
    return math.sqrt(lo * hi)


def channel_mean(ebn0_db: float, rate: float) -> float:
    """mu_0 = 2 / sigma^2 with sigma^2 = 1 / (2 R 10^(Eb/N0 / 10))."""
    return 4.0 * rate * 10.0 ** (ebn0_db / 10.0)


def ga_de(dv: int, dc: int, mu0: float, iters: int) -> np.ndarray:
    """C2V means mu_C after iterations 1..iters of flooding (Appendix A recursion); inf once the
    error probability underflows (decoding has converged)."""
    mu_v = mu0
    out = []
    for _ in range(iters):
        # 1 - (1 - Phi)^(dc - 1), accurate for tiny Phi
        mu_c = phi_inv(-math.expm1((dc - 1) * math.log1p(-phi(mu_v))))
        out.append(mu_c)
        mu_v = mu0 + (dv - 1) * mu_c
    return np.array(out)


def degree_profile(code):
    """(VN degrees and their node fractions, edge-perspective VN and CN degree distributions
    lambda_i and rho_j) of a code: lambda_i / rho_j = fraction of edges at VNs / CNs of degree i / j."""
    dv = np.bincount(code.col, minlength=code.N)
    dc = np.diff(code.row_ptr)
    E = float(code.E)
    vd, vn = np.unique(dv, return_counts=True)
    lam = {int(d): float(c * d) / E for d, c in zip(vd, vn)}
    cd, cn = np.unique(dc, return_counts=True)
    rho = {int(d): float(c * d) / E for d, c in zip(cd, cn)}
    return {int(d): float(c) / code.N for d, c in zip(vd, vn)}, lam, rho


def ga_de_irregular(lam: dict, rho: dict, mu0: float, iters: int) -> np.ndarray:
    """Mean C2V message t_l after iterations 1..iters for an irregular ensemble (Chung, Richardson,
    Urbanke 2001): t_l = sum_j rho_j Phi^-1(1 - [1 - sum_i lambda_i Phi(mu_0 + (i - 1) t_{l-1})]^(j-1)),
    t_0 = 0.  For a single VN and CN degree it is the regular recursion of Appendix A."""
    t = 0.0
    out = []
    for _ in range(iters):
        inner = sum(l * phi(mu0 + (i - 1) * t) for i, l in lam.items())
        t = sum(r * phi_inv(-math.expm1((j - 1) * math.log1p(-inner))) for j, r in rho.items())
        out.append(t)
    return np.array(out)


def ga_j_mixture(gammas: Sequence[float], node_frac: dict, mu0: float, t_prev: float, t_cur: float) -> np.ndarray:
    """J(gamma) when VNs of degree d (node fraction w_d) have L ~ N(mu_0 + d t_prev, 2 (...)) and
    Lt - L ~ N(d (t_cur - t_prev), 2 (...)): the correct and incorrect parts are summed over the
    degrees before the ratio is taken."""
    num = np.zeros(len(gammas))
    den = np.zeros(len(gammas))
    for d, w in node_frac.items():
        ml, mlt = mu0 + d * t_prev, mu0 + d * t_cur
        n_d, d_d = _ga_parts(gammas, ml, mlt)
        num += w * n_d
        den += w * d_d
    with np.errstate(divide="ignore"):
        return num / den


def ga_totals(dv: int, dc: int, mu0: float, iteration: int):
    """(mu_L, mu_Lt) at flooding iteration l >= 1: the totals after l - 1 iterations (the current
    ones) and after l (what the iteration's precomputed messages give)."""
    if iteration < 1:
        raise ValueError("iterations count from 1")
    mc = np.concatenate([[0.0], ga_de(dv, dc, mu0, iteration)])
    return mu0 + dv * mc[iteration - 1], mu0 + dv * mc[iteration]


def _q(x):
    return 0.5 * special.erfc(np.asarray(x, dtype=np.float64) / math.sqrt(2.0))


def _logit(p):
    with np.errstate(divide="ignore"):
        return np.log(p) - np.log1p(-p)


def ga_pr_d_given_l(gamma: float, l, mu_dl: float):
    """Pr(D >= gamma | L = l) with Lt = l + dL, dL ~ N(mu_dl, 2 mu_dl) (Appendix A)."""
    tau = special.expit(np.asarray(l, dtype=np.float64))
    s = math.sqrt(2.0 * mu_dl)
    a = _logit(np.maximum(tau - gamma, 0.0))  # -inf when tau <= gamma
    b = _logit(np.minimum(tau + gamma, 1.0))  # +inf when tau + gamma >= 1
    return 1.0 - _q((a - l - mu_dl) / s) + _q((b - l - mu_dl) / s)


def _ga_parts(gammas: Sequence[float], mu_l: float, mu_lt: float):
    """Pr(correct, D >= gamma) and Pr(incorrect, D >= gamma) of the Gaussian model, each an
    integral over L ~ N(mu_L, 2 mu_L)."""
    mu_dl = mu_lt - mu_l
    if not mu_dl > 0.0:
        raise ValueError("the model needs mu_Lt > mu_L")
    sl = math.sqrt(2.0 * mu_l)
    dens = lambda l: math.exp(-((l - mu_l) ** 2) / (4.0 * mu_l)) / math.sqrt(4.0 * math.pi * mu_l)
    lo, hi = mu_l - 14.0 * sl, mu_l + 14.0 * sl
    num, den = [], []
    for g in gammas:
        f = lambda l: float(ga_pr_d_given_l(g, l, mu_dl)) * dens(l)
        a, _ = integrate.quad(f, 0.0, max(hi, 1.0), limit=400, epsabs=0.0, epsrel=1e-9)
        b, _ = integrate.quad(f, min(lo, -1.0), 0.0, limit=400, epsabs=0.0, epsrel=1e-9)
        num.append(a)
        den.append(b)
    return np.array(num), np.array(den)


def ga_j(gammas: Sequence[float], mu_l: float, mu_lt: float) -> np.ndarray:
    """J(gamma) of the Gaussian model: the ratio of Pr(correct, D >= gamma) and
    Pr(incorrect, D >= gamma), each an integral over L ~ N(mu_L, 2 mu_L)."""
    num, den = _ga_parts(gammas, mu_l, mu_lt)
    with np.errstate(divide="ignore"):
        return np.where(den > 0, num / np.where(den > 0, den, 1.0), np.inf)


def ga_f(gammas: Sequence[float], tau: float, mu_dl: float) -> np.ndarray:
    """F(gamma) of the Gaussian model for one incorrect decision P0 = tau < 1/2 (Appendix B):
    Pr(P0t >= tau + gamma) / Pr(P0t <= tau - gamma); infinite for gamma >= tau."""
    lt = _logit(tau)
    s = math.sqrt(2.0 * mu_dl)
    out = []
    for g in gammas:
        up = 0.0 if tau + g >= 1.0 else float(_q((_logit(tau + g) - lt - mu_dl) / s))
        down = 0.0 if g >= tau else float(1.0 - _q((_logit(tau - g) - lt - mu_dl) / s))
        out.append(math.inf if down == 0.0 else up / down)
    return np.array(out)


# ----------------------------------------------------------------------------------------------
# statistics over decoded frames
# ----------------------------------------------------------------------------------------------
def empirical(L: np.ndarray, Lt: np.ndarray, gammas: Sequence[float]) -> Dict[str, np.ndarray]:
    """J(gamma) and F(gamma) counted over every (frame, VN) pair, all-zero codeword.

    Returns counts per gamma: correct/incorrect decisions with D >= gamma, and among the incorrect
    ones those whose p0 would rise (p0(Lt) >= p0(L)) or fall; J and F are their ratios (inf when
    the denominator is 0, nan when both are)."""
    L = np.asarray(L, dtype=np.float64).ravel()
    Lt = np.asarray(Lt, dtype=np.float64).ravel()
    p, pt = special.expit(L), special.expit(Lt)
    D = np.abs(p - pt)
    correct = p >= 0.5
    rise = pt >= p
    res = {k: [] for k in ("gamma", "n_correct", "n_incorrect", "n_rise", "n_fall")}
    for g in gammas:
        m = D >= g
        res["gamma"].append(g)
        res["n_correct"].append(int(np.sum(m & correct)))
        res["n_incorrect"].append(int(np.sum(m & ~correct)))
        res["n_rise"].append(int(np.sum(m & ~correct & rise)))
        res["n_fall"].append(int(np.sum(m & ~correct & ~rise)))
    out = {k: np.array(v) for k, v in res.items()}
    with np.errstate(divide="ignore", invalid="ignore"):
        out["J"] = out["n_correct"] / out["n_incorrect"]
        out["F"] = out["n_rise"] / out["n_fall"]
    return out


def flooding_states(ldpc, code_h, llr, iteration: int, arith=None, stream=None):
    """(L, Lt) of every frame at flooding iteration l >= 1, from the GPU decoder: the totals after
    l - 1 and after l iterations (check_every = 0, so no frame stops early)."""
    if iteration < 1:
        raise ValueError("iterations count from 1")
    arith = ldpc.SPA_F32 if arith is None else arith
    E = code_h.E
    a = ldpc.decode(code_h, llr, ldpc.FLOODING, arith, max_updates=(iteration - 1) * E, check_every=0, stream=stream)
    b = ldpc.decode(code_h, llr, ldpc.FLOODING, arith, max_updates=iteration * E, check_every=0, stream=stream)
    return a.llr_out, b.llr_out
