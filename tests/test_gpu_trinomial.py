"""Trinomial trees on the GPU (bt_price_exact_trinomial) against the
oracle's sum over 3^N paths.  Tolerances as for the binomial tree: FP64
1e-12 relative (floor 1e-15 S), FP32 with Kahan sums 1e-6 (floor 1e-9 S)."""
import json
import os

import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PAYOFFS = ("asian_call", "asian_put", "lookback_float", "lookback_fixed_put", "euro_call", "euro_put")
LAM = 1.224744871391589


def close(got, want, S, precision):
    if precision == "fp64":
        return abs(got - want) <= max(1e-12 * abs(want), 1e-15 * S)
    return abs(got - want) <= max(1e-6 * abs(want), 1e-9 * S)


def pair(gbt, orc, N, payoff, sigma=0.3, r=0.03, T=1.0, K=97.0, lam=LAM):
    u, pu, pd = gbt.bt_params_trinomial(sigma, r, T, N, lam)
    g = gbt.Option(100.0, u, pu, r, T, K, N, payoff)
    o = orc.Option(100.0, u, pu, r, T, K, N, payoff)
    return g, o, pd


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
@pytest.mark.parametrize("payoff", PAYOFFS)
@pytest.mark.parametrize("N", [1, 2, 3, 6, 9, 13])
def test_small_trees(gbt, orc, N, payoff, precision):
    g, o, pd = pair(gbt, orc, N, payoff)
    want = orc.price_tri_naive(o, pd) if N <= 9 else orc.price_tri(o, pd)
    got = gbt.bt_price_exact_trinomial(g, pd, precision)
    assert got["paths"] == 3 ** N
    assert close(got["value"], want, 100.0, precision), (got["value"], want)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_splits_and_chunks(gbt, orc, precision):
    g, o, pd = pair(gbt, orc, 12, "lookback_fixed_put", K=105.0)
    want = orc.price_tri(o, pd)
    for k in (1, 3, 7, 12):
        for chunk in (4, 64, 1024):
            r = gbt.bt_price_exact_trinomial(g, pd, precision, tune={"k": k, "chunk": chunk})
            assert r["split"] == k
            assert close(r["value"], want, 100.0, precision), (k, chunk, r["value"], want)


@pytest.mark.parametrize("payoff", PAYOFFS)
def test_binomial_limit(gbt, payoff):
    """Middle probability 0: the 3^N sum equals the binomial 2^N one."""
    g = gbt.make_option(100.0, 97.0, 0.3, 0.04, 1.0, 14, payoff)
    want = gbt.bt_price_exact(g, "fp64")["value"]
    got = gbt.bt_price_exact_trinomial(g, 1.0 - g.p, "fp64")["value"]
    assert abs(got - want) <= max(1e-12 * abs(want), 1e-15 * 100.0)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_n20_full_size(gbt, precision):
    """N=20 (3^20 = 3.49e9 paths), three payoffs, against oracle values
    stored by tests/golden/make_oracle_values.py."""
    gold = json.load(open(os.path.join(GOLD, "oracle_values.json")))
    rows = gold["exact_tri"]
    assert len(rows) == 3
    for e in rows:
        sp = e["spec"]
        u, pu, pd = gbt.bt_params_trinomial(sp["sigma"], sp["r"], sp["T"], sp["N"], sp["lam"])
        g = gbt.Option(sp["S"], u, pu, sp["r"], sp["T"], sp["K"], sp["N"], sp["payoff"])
        got = gbt.bt_price_exact_trinomial(g, pd, precision)
        assert got["paths"] == 3 ** 20
        assert close(got["value"], e["value"], sp["S"], precision), (sp["payoff"], got["value"], e["value"])


def test_trinomial_plan_stages(gbt, orc):
    g, o, pd = pair(gbt, orc, 11, "asian_put")
    one = gbt.bt_price_exact_trinomial(g, pd, "fp64")["value"]
    plan = gbt.Plan([g], "fp64", p_down=pd)
    for _ in range(2):
        plan.tables()
        plan.enumerate()
        plan.reduce()
        assert plan.results()[0]["value"] == one
    plan.close()


def test_trinomial_plan_of_several_options_matches_one_option_plans(gbt):
    """Options of different depths, strikes and payoffs sharing p_down in
    one plan: each value equals its one-option price bit for bit."""
    u, pu, pd = gbt.bt_params_trinomial(0.25, 0.04, 1.0, 12, 1.224744871391589)
    opts = [gbt.Option(100.0, u, pu, 0.04, 1.0, 100.0, 12, "asian_call"),
            gbt.Option(95.0, u, pu, 0.04, 1.0, 100.0, 12, "lookback_float"),
            gbt.Option(100.0, u, pu, 0.04, 1.0, 97.0, 9, "lookback_fixed_put"),
            gbt.Option(104.0, u, pu, 0.04, 1.0, 100.0, 14, "euro_put")]
    for precision in ("fp64", "fp32_kahan"):
        one = [gbt.bt_price_exact_trinomial(o, pd, precision)["value"] for o in opts]
        plan = gbt.Plan(opts, precision, p_down=pd)
        plan.tables()
        plan.enumerate()
        plan.reduce()
        assert [r["value"] for r in plan.results()] == one
        plan.close()
