"""Pins for the CPU oracle: what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints, hand-worked trees, closed forms, textbook methods (backward
induction, a lattice recursion), identities, published known-answer vectors,
and brute force over tiny trees.  CPU only.
"""
import itertools
import json
import math
import os
from dataclasses import replace
from fractions import Fraction

import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


PAYOFFS = ("asian_call", "asian_put", "lookback_float", "lookback_fixed_put",
           "euro_call", "euro_put")


# ---------------------------------------------------------------- trees


def test_two_step_tree_by_hand(orc):
    g = _gold("two_step_tree.json")
    for case in g["cases"]:
        base = orc.Option(case["S"], case["u"], case["p"], case["r"], case["T"],
                          case["K"], case["N"], "asian_call")
        disc = math.exp(-case["r"] * case["T"])
        # path prices and probabilities (Algorithm 1 grid, path probability)
        for bits_s, pv in case["paths"].items():
            bits = [int(c) for c in bits_s]
            assert orc.prob_of_path(base, bits) == pytest.approx(
                float(Fraction(pv["prob"])), rel=1e-15)
        for payoff, v in case["values"].items():
            o = replace(base, payoff=payoff)
            want = disc * float(Fraction(v["value"]))
            assert orc.price_naive(o) == pytest.approx(want, rel=1e-14), payoff
            assert orc.price_dfs(o, 1) == pytest.approx(want, rel=1e-14), payoff


def test_rank_partition_is_msb_first(orc):
    g = _gold("rank_partition.json")
    N, r = g["N"], g["r"]
    for m_s, paths in g["blocks"].items():
        m = int(m_s)
        for i, bits_s in enumerate(paths):
            assert orc.path_of_index(m * 2 ** (N - r) + i, N) == [int(c) for c in bits_s]


def test_paper_section5_exact_values(orc):
    """Section 5 prints 82.115 (Asian put) and 93.196 (fixed lookback put).
    Reproduced only with Seydel's u = beta + sqrt(beta^2 - 1)."""
    g = _gold("paper_section5_exact.json")
    P = g["params"]
    tol = 0.5 * 10 ** -g["printed_decimals"]
    lb = orc.make_option(P["S"], P["K"], P["sigma"], P["r"], P["T"], P["N"],
                         "lookback_fixed_put", P["scheme"])
    v_dp, _ = orc.lookback_dp(lb)
    assert abs(v_dp - g["values"]["lookback_fixed_put"]) <= tol
    ap = replace(lb, payoff="asian_put")
    v = orc.price_dfs(ap)
    assert abs(v - g["values"]["asian_put"]) <= tol


def test_paper_u_formula_reading(orc):
    """The printed '+1' under the root gives a lookback value far from the
    printed 93.196; the reading '-1' (Seydel) reproduces it (test above)."""
    g = _gold("paper_section5_exact.json")
    P = g["params"]
    dt = P["T"] / P["N"]
    beta = 0.5 * (math.exp(-P["r"] * dt) + math.exp((P["r"] + P["sigma"] ** 2) * dt))
    u_plus = beta + math.sqrt(beta * beta + 1.0)
    d = 1.0 / u_plus
    p = (math.exp(P["r"] * dt) - d) / (u_plus - d)
    o = orc.Option(P["S"], u_plus, p, P["r"], P["T"], P["K"], P["N"], "lookback_fixed_put")
    v, _ = orc.lookback_dp(o)
    assert abs(v - g["values"]["lookback_fixed_put"]) > 0.5


# ---------------------------------------------------------- closed forms


@pytest.mark.parametrize("N", [1, 2, 5, 12, 18])
@pytest.mark.parametrize("scheme", ["crr", "seydel"])
def test_martingale_discounted_terminal(orc, N, scheme):
    """A3 with risk-neutral p: e^{-rT} E[S_N] = S.  A European call with K=0
    pays S_N, so its value must be S."""
    o = orc.make_option(100.0, 0.0, 0.25, 0.05, 1.5, N, "euro_call", scheme)
    assert orc.price_naive(o) == pytest.approx(100.0, rel=1e-13)
    assert orc.price_dfs(o, 2) == pytest.approx(100.0, rel=1e-13)


@pytest.mark.parametrize("N", [1, 3, 10, 16])
def test_asian_mean_closed_form(orc, N):
    """E[(1/N) sum_{t=1..N} S_t] = (S/N) sum_t g^t with g = pu + (1-p)/u; an
    Asian call with K=0 pays the mean."""
    S, r, T = 80.0, 0.03, 0.7
    o = orc.make_option(S, 0.0, 0.35, r, T, N, "asian_call")
    g = o.p * o.u + (1 - o.p) / o.u
    mean = S / N * sum(g ** t for t in range(1, N + 1))
    assert orc.price_naive(o) == pytest.approx(math.exp(-r * T) * mean, rel=1e-13)


@pytest.mark.parametrize("N", [4, 11, 17])
def test_asian_put_call_parity(orc, N):
    """C - P = e^{-rT} (E[A] - K): an exact identity of the Asian payoffs."""
    S, K, r, T = 100.0, 103.0, 0.05, 1.0
    c = orc.make_option(S, K, 0.2, r, T, N, "asian_call")
    p = replace(c, payoff="asian_put")
    g = c.p * c.u + (1 - c.p) / c.u
    mean = S / N * sum(g ** t for t in range(1, N + 1))
    lhs = orc.price_naive(c) - orc.price_naive(p)
    assert lhs == pytest.approx(math.exp(-r * T) * (mean - K), rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("N", [1, 2, 7, 15, 20])
@pytest.mark.parametrize("payoff", ["euro_call", "euro_put"])
def test_european_backward_induction(orc, N, payoff):
    """Path enumeration (eq. (f13)) = eq. (f8) closed sum = backward induction
    on the Algorithm 1 grid."""
    o = orc.make_option(100.0, 95.0, 0.3, 0.04, 2.0, N, payoff)
    bi = orc.euro_backward(o)
    assert orc.euro_closed(o) == pytest.approx(bi, rel=1e-13)
    assert orc.price_dfs(o, 3) == pytest.approx(bi, rel=1e-13)


@pytest.mark.parametrize("N", [1, 2, 9, 16, 22])
@pytest.mark.parametrize("payoff", ["lookback_float", "lookback_fixed_put"])
def test_lookback_lattice_recursion(orc, N, payoff):
    """Enumeration equals a lattice recursion over (level, running extreme),
    a different method summing in a different order."""
    o = orc.make_option(100.0, 110.0, 0.4, 0.05, 1.0, N, payoff)
    dp, _ = orc.lookback_dp(o)
    assert orc.price_dfs(o) == pytest.approx(dp, rel=1e-13)


def test_lookback_second_moment_dp(orc):
    """E[V^2] from the recursion equals the exact stratum decomposition's
    Var[V] + E[V]^2 (eq. (mc14) pieces)."""
    o = orc.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 14, "lookback_float")
    dp, m2 = orc.lookback_dp(o)
    ex = orc.exact_strata(o, 5)
    assert ex["var_total"] + ex["mean"] ** 2 == pytest.approx(m2, rel=1e-12)
    assert math.exp(-o.r * o.T) * ex["mean"] == pytest.approx(dp, rel=1e-13)


# ---------------------------------------------------------- brute force


def _brute(o):
    """Tiny trees: every path written out, prices as S u^(2U_t - t)."""
    tot = 0.0
    for bits in itertools.product((0, 1), repeat=o.N):
        U, path = 0, []
        for t, b in enumerate(bits, start=1):
            U += b
            path.append(o.S * o.u ** (2 * U - t))
        w = o.p ** U * (1 - o.p) ** (o.N - U)
        mean = sum(path) / o.N
        v = {"asian_call": max(mean - o.K, 0.0), "asian_put": max(o.K - mean, 0.0),
             "lookback_float": max(path) - path[-1],
             "lookback_fixed_put": max(o.K - min(path), 0.0),
             "euro_call": max(path[-1] - o.K, 0.0),
             "euro_put": max(o.K - path[-1], 0.0)}[o.payoff]
        tot += w * v
    return math.exp(-o.r * o.T) * tot


@pytest.mark.parametrize("N", [1, 2, 3, 6, 10])
@pytest.mark.parametrize("payoff", PAYOFFS)
def test_brute_force_tiny(orc, N, payoff):
    o = orc.make_option(50.0, 52.0, 0.45, 0.02, 0.5, N, payoff)
    assert orc.price_naive(o) == pytest.approx(_brute(o), rel=1e-12, abs=1e-13)


# ------------------------------------------------ enumerators agree


@pytest.mark.parametrize("payoff", PAYOFFS)
def test_naive_equals_dfs(orc, payoff):
    o = orc.make_option(100.0, 100.0, 0.2, 0.05, 1.0, 18, payoff)
    assert orc.price_dfs(o, 4) == pytest.approx(orc.price_naive(o), rel=1e-14)


def test_dfs_independent_of_thread_count(orc):
    o = orc.make_option(100.0, 100.0, 0.2, 0.05, 1.0, 21, "asian_call")
    vals = {orc.price_dfs(o, t) for t in (1, 3, 8)}
    assert len(vals) == 1


def test_subtree_blocks_partition_the_sum(orc):
    """eqs. (f14)-(f15): blocks of the first d steps partition B^N; a block is
    the index range [z 2^(N-d), (z+1) 2^(N-d))."""
    o = orc.make_option(100.0, 100.0, 0.2, 0.05, 1.0, 12, "lookback_float")
    d = 4
    parts = [orc.subtree_sum(o, d, z) for z in range(2 ** d)]
    for z in (0, 5, 15):
        lo, hi = z * 2 ** (o.N - d), (z + 1) * 2 ** (o.N - d)
        assert parts[z] == pytest.approx(orc.range_naive(o, lo, hi), rel=1e-14)
    total = math.exp(-o.r * o.T) * sum(parts)
    assert total == pytest.approx(orc.price_naive(o), rel=1e-14)


def test_path_probabilities_sum_to_one(orc):
    """eq. (f11) summed over i: the 2^N path probabilities add to 1."""
    o = orc.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 10, "asian_call")
    tot = sum(orc.prob_of_path(o, orc.path_of_index(x, 10)) for x in range(2 ** 10))
    assert tot == pytest.approx(1.0, rel=1e-14)


# ------------------------------------------------------------- params


def test_params_crr_and_risk_neutral_drift(orc):
    u, p = orc.params(0.2, 0.05, 1.0, 32, "crr")
    assert u == pytest.approx(math.exp(0.2 * math.sqrt(1 / 32)), rel=1e-15)
    # A3: p u + (1-p) d = e^{r dt}
    assert p * u + (1 - p) / u == pytest.approx(math.exp(0.05 / 32), rel=1e-14)


def test_params_reject_arbitrage(orc):
    with pytest.raises(ValueError):
        orc.params(0.01, 0.5, 1.0, 2, "crr")  # e^{r dt} > u: p > 1


# ------------------------------------------------------------- Philox


def test_philox_known_answers(orc):
    g = _gold("philox_kat.json")
    for v in g["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        assert orc.philox4x32_10(ctr, key) == [int(x, 16) for x in v["out"]]


def test_up_threshold(orc):
    assert orc.up_threshold(0.5) == 2 ** 31
    assert orc.up_threshold(0.25) == 2 ** 30
    p = 0.5167980141148621
    assert orc.up_threshold(p) == math.floor(p * 2 ** 32)


def test_bernoulli_frequency(orc):
    p = 0.37
    thr = orc.up_threshold(p)
    n, ups = 0, 0
    for m in range(400):
        b = orc.mc_suffix_bits(12345, 0, 7, m, 50, thr)
        n += len(b)
        ups += sum(b)
    sd = math.sqrt(p * (1 - p) / n)
    assert abs(ups / n - p) < 5 * sd


# --------------------------------------------------------- Monte Carlo


def test_total_variance_decomposition(orc):
    """eq. (mc14): Var[V] = sum P Var[V|D] + Var_D E[V|D], exactly."""
    o = orc.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 12, "asian_call")
    for r in (0, 3, 7, 12):
        ex = orc.exact_strata(o, r)
        assert ex["within"] + ex["between"] == pytest.approx(ex["var_total"], rel=1e-12)
        assert ex["mean"] * math.exp(-o.r * o.T) == pytest.approx(orc.price_naive(o), rel=1e-13)
    assert orc.exact_strata(o, 12)["within"] == pytest.approx(0.0, abs=1e-12)
    assert orc.exact_strata(o, 0)["between"] == pytest.approx(0.0, abs=1e-9)


def test_stratified_mc_unbiased_and_variance(orc):
    """Over many seeds: the Partitioned estimator averages to the exact value,
    its spread matches sum W^2 Var[V|D]/R_m (eq. (mc13) first line, equal
    allocation), and the 1/(R_m - 1) variance estimate is unbiased for it."""
    o = orc.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 12, "asian_call")
    r, Rm, reps = 4, 16, 300
    ex = orc.exact_strata(o, r)
    want_var = ex["within_sq"] / Rm
    est, vub = [], []
    for s in range(reps):
        th, _, ub = orc.mc_stratified_range(o, r, Rm, 1000 + s, 0, 0, 2 ** r)
        est.append(th)
        vub.append(ub)
    mean = sum(est) / reps
    emp = sum((e - mean) ** 2 for e in est) / (reps - 1)
    assert abs(mean - ex["mean"]) < 4 * math.sqrt(want_var / reps)
    assert emp == pytest.approx(want_var, rel=0.25)
    assert sum(vub) / reps == pytest.approx(want_var, rel=0.1)
    # Partitioned beats basic MC at equal sample count (eq. (mc15)).
    assert want_var <= ex["var_total"] / (Rm * 2 ** r)


def test_variance_estimator_normalisations(orc):
    """With R_m = 4 the plug-in s^2 (1/R_m, the paper's form) is biased low by
    (R_m - 1)/R_m = 3/4 and the 1/(R_m - 1) form is unbiased."""
    o = orc.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 10, "asian_put")
    r, Rm, reps = 3, 4, 600
    want = orc.exact_strata(o, r)["within_sq"] / Rm
    pi = ub = 0.0
    for s in range(reps):
        _, a, b = orc.mc_stratified_range(o, r, Rm, 777 + s, 1, 0, 2 ** r)
        pi += a / reps
        ub += b / reps
    assert ub == pytest.approx(want, rel=0.08)
    assert pi == pytest.approx(0.75 * want, rel=0.08)


def test_plain_mc_is_r0(orc):
    """r = 0: a single stratum, the basic estimator and its 1/R^2 variance."""
    o = orc.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 10, "lookback_float")
    th, vpi, _ = orc.mc_stratified_range(o, 0, 4096, 99, 0, 0, 1)
    ex = orc.exact_strata(o, 0)
    assert abs(th - ex["mean"]) < 5 * math.sqrt(ex["var_total"] / 4096)
    assert vpi == pytest.approx(ex["var_total"] / 4096, rel=0.15)


def test_plain_mc_variance_from_strata(orc):
    """The stratified draws also estimate E[V^2] (sum_z P(D_z) mean_m V^2,
    unbiased), hence the variance plain MC would have with as many paths,
    (E[V^2] - E[V]^2) / paths, eq. (mc2).  Over many seeds the E[V^2]
    estimate averages to the exact one (var_total + mean^2 by enumeration);
    with one stratum the plain-MC variance is the plug-in variance itself;
    stratification never has the larger variance (eq. (mc15))."""
    o = orc.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 12, "lookback_float")
    r, Rm, reps = 4, 16, 200
    ex = orc.exact_strata(o, r)
    second = [orc.mc_stratified_second(o, r, Rm, 4000 + s, 0, 0, 2 ** r) for s in range(reps)]
    mean2 = sum(second) / reps
    sd = math.sqrt(sum((x - mean2) ** 2 for x in second) / (reps - 1))
    assert abs(mean2 - (ex["var_total"] + ex["mean"] ** 2)) < 4 * sd / math.sqrt(reps)
    # one stratum: the plain-MC variance equals the plug-in variance
    disc2 = math.exp(-2 * o.r * o.T)
    _, vpi, _ = orc.mc_stratified(o, 0, 4096, 99, 0)
    assert orc.mc_stratified_plain_var(o, 0, 4096, 99, 0) == pytest.approx(vpi, rel=1e-12)
    # stratified vs plain at equal paths, exact and estimated
    vp = [orc.mc_stratified_plain_var(o, r, Rm, 4000 + s, 0) for s in range(40)]
    assert sum(vp) / 40 == pytest.approx(disc2 * ex["var_total"] / (Rm * 2 ** r), rel=0.1)
    assert ex["within_sq"] / Rm <= ex["var_total"] / (Rm * 2 ** r)


def test_proportional_second_moment(orc):
    """Proportional allocation's draws estimate E[V^2] without bias too."""
    o = orc.make_option(100.0, 95.0, 0.3, 0.05, 1.0, 12, "asian_call")
    r, R, reps = 4, 512, 150
    ex = orc.exact_strata(o, r)
    sec = [orc.mc_proportional_second(o, r, R, 600 + s, 2) for s in range(reps)]
    m = sum(sec) / reps
    sd = math.sqrt(sum((x - m) ** 2 for x in sec) / (reps - 1))
    assert abs(m - (ex["var_total"] + ex["mean"] ** 2)) < 4 * sd / math.sqrt(reps)


def test_mc_ranges_add_up(orc):
    o = orc.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 14, "asian_put")
    full = orc.mc_stratified_range(o, 6, 8, 5, 3, 0, 64)
    a = orc.mc_stratified_range(o, 6, 8, 5, 3, 0, 20)
    b = orc.mc_stratified_range(o, 6, 8, 5, 3, 20, 64)
    for i in range(3):
        assert a[i] + b[i] == pytest.approx(full[i], rel=1e-14)
    sa = orc.mc_stratified_second(o, 6, 8, 5, 3, 0, 20)
    sb = orc.mc_stratified_second(o, 6, 8, 5, 3, 20, 64)
    assert sa + sb == pytest.approx(orc.mc_stratified_second(o, 6, 8, 5, 3, 0, 64), rel=1e-14)


# ------------------------------------------- Shared-Sample, proportional


def test_shared_sample_identities_and_theorem1(orc):
    """eq. (mc17): Var[V] = Var_Y E[V|Y] + E_Y Var[V|Y]; Theorem 1 (R_m = R):
    sum P^2 Var[V|D] <= Var_Y E[V|Y] <= Var[V]."""
    for payoff in ("asian_put", "lookback_fixed_put", "asian_call"):
        o = orc.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 12, payoff)
        for r in (1, 3, 5, 8, 11):
            ex = orc.exact_strata(o, r)
            assert ex["shared"] + ex["within_y"] == pytest.approx(ex["var_total"], rel=1e-12)
            assert ex["within_sq"] <= ex["shared"] <= ex["var_total"]


def test_shared_sample_unbiased_and_variance(orc):
    o = orc.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 10, "asian_put")
    r, R, reps = 4, 32, 300
    ex = orc.exact_strata(o, r)
    want = ex["shared"] / R
    est, vub, vpi = [], [], []
    for s in range(reps):
        th, pi, ub = orc.mc_shared(o, r, R, 5000 + s, 2)
        est.append(th); vub.append(ub); vpi.append(pi)
    mean = sum(est) / reps
    emp = sum((e - mean) ** 2 for e in est) / (reps - 1)
    assert abs(mean - ex["mean"]) < 4 * math.sqrt(want / reps)
    assert emp == pytest.approx(want, rel=0.25)
    assert sum(vub) / reps == pytest.approx(want, rel=0.12)
    assert sum(vpi) / reps == pytest.approx(want * (R - 1) / R, rel=0.12)


def test_proportional_allocation(orc):
    """R_m = R P(D_m): unbiased, and its variance is (1/R) sum P Var[V|D]
    (eq. (mc13)); the paper's 1/R^2 estimator estimates it."""
    o = orc.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 10, "lookback_float")
    r, R, reps = 3, 4096, 120
    ex = orc.exact_strata(o, r)
    want = ex["within"] / R
    est, vpaper = [], []
    for s in range(reps):
        th, pi, ub, paper, n = orc.mc_proportional(o, r, R, 900 + s, 4)
        assert abs(n - R) <= 2 ** r
        est.append(th); vpaper.append(paper)
    mean = sum(est) / reps
    assert abs(mean - ex["mean"]) < 4 * math.sqrt(want / reps)
    assert sum(vpaper) / reps == pytest.approx(want, rel=0.1)


def test_proportional_single_draw_strata(orc):
    """Every stratum at R_m = 1 (R far below 2^r): the estimate is one draw
    per stratum, the plug-in variance is 0 and the 1/(R_m - 1) form is
    undefined (NaN); a stratum whose P(D_m) R rounds to zero still gets its
    one draw."""
    o = orc.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 8, "asian_call")
    th, pi, ub, paper, n = orc.mc_proportional(o, 4, 1, 5, 0)
    assert n == 16 and pi == 0.0 and math.isnan(ub)
    # same draws as equal allocation with R_m = 1
    th_eq, _, _ = orc.mc_stratified_range(o, 4, 1, 5, 0, 0, 16)
    assert th == pytest.approx(th_eq, rel=1e-15)


def _paper45():
    return _gold("paper_tables_4_5.json")


def test_paper_table4_reading_is_proportional(orc):
    """Table 4's variances follow R_m = R P(D_m) (the text), not R/M per
    stratum (its header): at M = 64 the proportional estimator averages near
    the printed 0.194, equal allocation far below it."""
    g = _paper45()
    P = g["params"]
    o = orc.make_option(P["S"], P["K"], P["sigma"], P["r"], P["T"], P["N"], "asian_put", P["scheme"])
    disc2 = math.exp(-2 * P["r"] * P["T"])
    t4 = g["table4_partitioned_R1024"]
    for M, printed in zip(t4["M"], t4["var_asian_put"]):
        if M not in (1, 8, 64):
            continue
        r = int(math.log2(M))
        reps = 60
        vals = [disc2 * orc.mc_proportional(o, r, 1024, 70 + s, 1)[3] for s in range(reps)]
        assert sum(vals) / reps == pytest.approx(printed, rel=0.12), M
    equal = [disc2 * orc.mc_stratified_range(o, 6, 16, 70 + s, 1, 0, 64)[1] for s in range(60)]
    assert sum(equal) / 60 < 0.85 * 0.194


def test_paper_table5_shared_sample(orc):
    """Table 5's Shared-Sample variances (R = 1024) against the estimator's
    average over repetitions (printed values are averages of 1000
    repetitions; tolerance 12%)."""
    g = _paper45()
    P = g["params"]
    o = orc.make_option(P["S"], P["K"], P["sigma"], P["r"], P["T"], P["N"], "asian_put", P["scheme"])
    disc2 = math.exp(-2 * P["r"] * P["T"])
    t5 = g["table5_shared_sample_R1024"]
    for M, printed in zip(t5["M"], t5["var_asian_put"]):
        if M not in (2, 16, 64):
            continue
        r = int(math.log2(M))
        reps = 24
        vals = [disc2 * orc.mc_shared(o, r, 1024, 300 + s, 3)[1] for s in range(reps)]
        assert sum(vals) / reps == pytest.approx(printed, rel=0.12), M


def test_suffix_draws_half_words_and_ties(orc):
    """Suffix steps read 16-bit halves of the Philox block (high half for
    even steps, low half for odd ones, eight steps per block); a step whose
    half equals the threshold's high half is decided by the high half of a
    fallback block with counter (2^31 + j, m, z, stream).  Checked against
    Philox outputs computed directly, with the threshold chosen to force a
    tie at step 3 and at step 12 (second block)."""
    seed, stream, z, m = 0x1234_5678_9ABC_DEF0, 7, 4242, 99
    key = [seed & 0xFFFFFFFF, seed >> 32]
    blocks = [orc.philox4x32_10([b, m, z, stream], key) for b in range(2)]
    halves = []
    for j in range(16):
        w = blocks[j // 8][(j % 8) // 2]
        halves.append(w >> 16 if j % 2 == 0 else w & 0xFFFF)
    for tie_step in (3, 12):
        h = halves[tie_step]
        g = orc.philox4x32_10([0x80000000 + tie_step, m, z, stream], key)[0] >> 16
        for lo in (0, 1, g, g + 1, 0xFFFF):
            if lo > 0xFFFF:
                continue
            thr = (h << 16) | lo
            bits = orc.mc_suffix_bits(seed, stream, z, m, 16, thr)
            for j in range(16):
                if halves[j] == h:
                    fb = orc.philox4x32_10([0x80000000 + j, m, z, stream], key)[0] >> 16
                    assert bits[j] == (1 if fb < lo else 0), (tie_step, lo, j)
                else:
                    assert bits[j] == (1 if halves[j] < h else 0), (tie_step, lo, j)
            assert bits[tie_step] == (1 if g < lo else 0)


def test_mc_ranges_split_the_estimators(orc):
    """The range forms (used to spread the oracle's MC work over host
    threads) add up to the whole estimators: proportional allocation over
    strata ranges, Shared-Sample over draw ranges (its estimate is the mean
    of the h_i, eq. (mc16), with the 1/R^2 variance of the h_i)."""
    o = orc.make_option(100.0, 100.0, 0.2, 0.05, 1.0, 16, "asian_call")
    r, R, seed = 6, 3000, 17
    whole = orc.mc_proportional(o, r, R, seed, 2)
    cuts = [0, 5, 17, 40, 64]
    parts = [orc.mc_proportional_range(o, r, R, seed, 2, a, b) for a, b in zip(cuts, cuts[1:])]
    for k in range(4):
        tot = sum(p[k] for p in parts)
        assert abs(tot - whole[k]) <= 1e-14 * abs(whole[k]) + 1e-300, (k, tot, whole[k])
    assert sum(p[4] for p in parts) == whole[4]
    theta, vpi, _ = orc.mc_shared(o, r, 40, seed, 2)
    h = orc.mc_shared_draws(o, r, seed, 2, 0, 13) + orc.mc_shared_draws(o, r, seed, 2, 13, 40)
    mean = sum(h) / len(h)
    assert abs(mean - theta) <= 1e-14 * abs(theta)
    v = sum((x - mean) ** 2 for x in h) / len(h) ** 2
    assert abs(v - vpi) <= 1e-12 * vpi
    # a draw's h_i does not depend on the range it is computed in
    assert orc.mc_shared_draws(o, r, seed, 2, 13, 14)[0] == h[13]
