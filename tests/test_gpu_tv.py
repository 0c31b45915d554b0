"""Time-varying moves on the GPU (bt_price_exact_tv) against the oracle's
eq. (f13) with per-step u_t, p_t.  Tolerances as for the fixed tree: FP64
1e-12 relative (floor 1e-15 S), FP32 with Kahan sums 1e-6 (floor 1e-9 S)."""
import json
import os
import random

import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PAYOFFS = ("asian_call", "asian_put", "lookback_float", "lookback_fixed_put", "euro_call", "euro_put")


def close(got, want, S, precision):
    if precision == "fp64":
        return abs(got - want) <= max(1e-12 * abs(want), 1e-15 * S)
    return abs(got - want) <= max(1e-6 * abs(want), 1e-9 * S)


def steps_from_sigmas(bt, sigmas, r, T):
    N = len(sigmas)
    uv = [bt.bt_params(s, r, T, N) for s in sigmas]
    return [u for u, _ in uv], [p for _, p in uv]


def random_steps(N, seed):
    g = random.Random(seed)
    return [g.uniform(1.02, 1.25) for _ in range(N)], [g.uniform(0.25, 0.75) for _ in range(N)]


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
@pytest.mark.parametrize("payoff", PAYOFFS)
@pytest.mark.parametrize("N", [1, 2, 3, 7, 12, 17])
def test_small_trees(gbt, orc, N, payoff, precision):
    u, p = random_steps(N, 100 + N)
    g = gbt.Option(100.0, 1.1, 0.5, 0.03, 1.0, 97.0, N, payoff)
    o = orc.Option(100.0, 1.1, 0.5, 0.03, 1.0, 97.0, N, payoff)
    want = orc.price_tv_naive(o, u, p)
    got = gbt.bt_price_exact_tv(g, u, p, precision)
    assert got["paths"] == 2 ** N
    assert close(got["value"], want, 100.0, precision), (got["value"], want)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_splits_and_chunks(gbt, orc, precision):
    N = 15
    u, p = random_steps(N, 7)
    g = gbt.Option(90.0, 1.1, 0.5, 0.02, 1.5, 100.0, N, "asian_put")
    want = orc.price_tv(orc.Option(90.0, 1.1, 0.5, 0.02, 1.5, 100.0, N, "asian_put"), u, p, 4)
    for k in (1, 4, 9, 15):
        for chunk in (4, 64, 512):
            r = gbt.bt_price_exact_tv(g, u, p, precision, tune={"k": k, "chunk": chunk})
            assert r["split"] == k
            assert close(r["value"], want, 90.0, precision), (k, chunk, r["value"], want)


def test_constant_steps_match_the_fixed_tree(gbt):
    g = gbt.make_option(100.0, 100.0, 0.25, 0.05, 1.0, 20, "lookback_float")
    fixed = gbt.bt_price_exact(g, "fp64")["value"]
    tv = gbt.bt_price_exact_tv(g, [g.u] * 20, [g.p] * 20, "fp64")["value"]
    assert abs(tv - fixed) <= 1e-13 * abs(fixed)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_term_structure_n24(gbt, orc, precision):
    from paper_1701_03512_amd import workloads
    sig = workloads.term_structure_sigmas(24, jitter=0.03)
    u, p = steps_from_sigmas(gbt, sig, 0.05, 1.0)
    for payoff in ("asian_call", "lookback_fixed_put"):
        g = gbt.Option(100.0, 1.1, 0.5, 0.05, 1.0, 100.0, 24, payoff)
        want = orc.price_tv(orc.Option(100.0, 1.1, 0.5, 0.05, 1.0, 100.0, 24, payoff), u, p)
        got = gbt.bt_price_exact_tv(g, u, p, precision)["value"]
        assert close(got, want, 100.0, precision), (payoff, got, want)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_term_structure_n32_full_size(gbt, precision):
    """N=32 (2^32 paths), volatility ramp 0.15 -> 0.30, three payoffs, against
    oracle values stored by tests/golden/make_oracle_values.py."""
    gold = json.load(open(os.path.join(GOLD, "oracle_values.json")))
    rows = gold["exact_tv"]
    assert len(rows) == 3
    for e in rows:
        sp = e["spec"]
        u, p = steps_from_sigmas(gbt, sp["sigma_t"], sp["r"], sp["T"])
        g = gbt.Option(sp["S"], 1.1, 0.5, sp["r"], sp["T"], sp["K"], sp["N"], sp["payoff"])
        got = gbt.bt_price_exact_tv(g, u, p, precision)
        assert got["paths"] == 2 ** 32
        assert close(got["value"], e["value"], sp["S"], precision), (sp["payoff"], got["value"], e["value"])


def test_fp32_weight_range_refused(gbt):
    N = 40
    u = [1.05] * N
    p = [0.001] * N
    g = gbt.Option(100.0, 1.1, 0.5, 0.0, 1.0, 100.0, N, "asian_call")
    with pytest.raises(gbt.BtError) as e:
        gbt.bt_price_exact_tv(g, u, p, "fp32_kahan")
    assert e.value.code == gbt.BT_ERANGE


def test_tv_plan_stages_match_the_one_call(gbt):
    N = 18
    u, p = random_steps(N, 21)
    g = gbt.Option(100.0, 1.1, 0.5, 0.01, 1.0, 105.0, N, "lookback_fixed_put")
    one = gbt.bt_price_exact_tv(g, u, p, "fp64")["value"]
    plan = gbt.Plan([g], "fp64", u_t=u, p_t=p)
    for _ in range(2):
        plan.tables()
        plan.enumerate()
        plan.reduce()
        assert plan.results()[0]["value"] == one
    plan.close()


def test_tv_plan_of_several_options_matches_one_option_plans(gbt):
    """Options of one depth sharing a term structure in one plan: each value
    equals its one-option price bit for bit; differing depths are refused."""
    N = 20
    u, p = random_steps(N, 33)
    opts = [gbt.Option(100.0, 1.1, 0.5, 0.02, 1.0, 100.0, N, "asian_call"),
            gbt.Option(90.0, 1.1, 0.5, 0.02, 1.5, 95.0, N, "asian_put"),
            gbt.Option(110.0, 1.1, 0.5, 0.03, 1.0, 0.0, N, "lookback_float"),
            gbt.Option(100.0, 1.1, 0.5, 0.01, 0.5, 104.0, N, "lookback_fixed_put")]
    for precision in ("fp64", "fp32_kahan"):
        one = [gbt.bt_price_exact_tv(o, u, p, precision)["value"] for o in opts]
        plan = gbt.Plan(opts, precision, u_t=u, p_t=p)
        plan.tables()
        plan.enumerate()
        plan.reduce()
        assert [r["value"] for r in plan.results()] == one
        plan.close()
    bad = [opts[0], gbt.Option(100.0, 1.1, 0.5, 0.02, 1.0, 100.0, N - 1, "asian_call")]
    with pytest.raises(gbt.BtError) as e:
        gbt.Plan(bad, "fp64", u_t=u, p_t=p)
    assert e.value.code == gbt.BT_EINVAL
