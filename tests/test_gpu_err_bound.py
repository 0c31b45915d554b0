"""The per-result error bound (bt_result.err_bound) of exact pricing.

Validity: on small trees the exact value of eq. (f13) is computed in rational
arithmetic from the option's own FP64 inputs, so |value - exact| <= err_bound
is checked with nothing else rounding.  On full-size workloads the oracle
stands in for the exact value and its own rounding bound is added
(tests/bounds.py).  Tightness: the FP32 form of a binomial tree states at
most 1e-6 of the value on the benchmark workloads (the target accuracy of
the compensated form)."""
import json
import math
import os

import pytest

import bounds

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PAYOFFS = ("asian_call", "asian_put", "lookback_float", "lookback_fixed_put",
           "euro_call", "euro_put")

_exact_cache = {}


def _exact(g, payoff):
    key = (g.S, g.u, g.p, g.K, g.N, payoff)
    if key not in _exact_cache:
        _exact_cache[key] = bounds.exact_binomial(g.S, g.u, g.p, g.K, g.N, payoff)
    return _exact_cache[key]


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
@pytest.mark.parametrize("payoff", PAYOFFS)
@pytest.mark.parametrize("N", [1, 2, 5, 9, 12])
def test_bound_holds_against_exact_rational(gbt, N, payoff, precision):
    """r = 0 (no discount): the value against eq. (f13) in exact arithmetic,
    under the default split and two others."""
    g = gbt.make_option(100.0, 104.0, 0.3, 0.0, 1.0, N, payoff)
    exact = _exact(g, payoff)
    for tune in (None, {"k": 1}, {"k": max(1, N // 2), "chunk": 4}):
        r = gbt.bt_price_exact(g, precision, tune=tune)
        assert r["status"] == 0 and math.isfinite(r["err_bound"]) and r["err_bound"] >= 0
        err = abs(r["value"] - exact)
        assert err <= r["err_bound"], (tune, float(err), r["err_bound"])


@pytest.mark.parametrize("payoff", PAYOFFS)
def test_fp32_bound_counts_only_paths_that_reach_the_money(gbt, payoff):
    """The FP32 binomial bound sums input rounding over the paths that can
    pay, so it stays within 1e-6 of the value however far the strike is out
    of the money, and is exactly zero when no path pays (the value is then
    exactly zero too).  Checked against eq. (f13) in exact arithmetic."""
    N = 12
    g0 = gbt.make_option(100.0, 100.0, 0.3, 0.0, 1.0, N, payoff)
    top, bottom = 100.0 * g0.u ** N, 100.0 * g0.u ** -N  # the extreme prices
    calls = payoff in ("asian_call", "euro_call")
    strikes = [1.5 * top] if calls else [bottom / 1.5]  # no path pays
    # strikes that leave a sliver of paying paths, near the extreme path
    if payoff in ("asian_call", "euro_call"):
        strikes += [0.97 * top if payoff == "euro_call" else 0.9 * sum(100.0 * g0.u ** t
                                                                     for t in range(1, N + 1)) / N]
    elif payoff in ("asian_put", "euro_put", "lookback_fixed_put"):
        strikes += [1.05 * bottom]
    for K in strikes:
        g = gbt.make_option(100.0, K, 0.3, 0.0, 1.0, N, payoff)
        exact = _exact(g, payoff)
        for tune in (None, {"k": 4, "chunk": 16}):
            r = gbt.bt_price_exact(g, "fp32_kahan", tune=tune)
            assert r["status"] == 0
            assert abs(r["value"] - exact) <= r["err_bound"], (K, tune, r, float(exact))
            if exact == 0:
                assert r["value"] == 0.0 and r["err_bound"] == 0.0, (K, tune, r)
            else:
                assert r["err_bound"] <= 1e-6 * float(exact), (K, tune, r, float(exact))


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_bound_holds_and_is_tight_at_n32(gbt, precision):
    """The N=32 workload (three payoffs) against the stored oracle values."""
    gold = json.load(open(os.path.join(GOLD, "oracle_values.json")))
    rows = [e for e in gold["exact"] if e["spec"]["N"] in (20, 32)]
    for e in rows:
        sp = e["spec"]
        g = gbt.make_option(sp["S"], sp["K"], sp["sigma"], sp["r"], sp["T"], sp["N"], sp["payoff"])
        r = gbt.bt_price_exact(g, precision)
        ob = bounds.oracle_rounding(e["value"], g.S, g.K, g.r, g.T, g.N,
                                    bounds.forward_growth(g.u, g.p, g.N))
        err = abs(r["value"] - e["value"])
        assert err <= r["err_bound"] + ob, (sp, err, r["err_bound"], ob)
        limit = 1e-12 if precision == "fp64" else 1e-6
        assert r["err_bound"] <= limit * abs(r["value"]), (sp, r["err_bound"] / r["value"])


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_bound_time_varying_and_trinomial(gbt, precision):
    """Time-varying N=32 and trinomial N=20 workloads against the stored
    oracle values.  Their FP32 form keeps the path weight in the FP32
    multiplier and chains 32 multiply-adds per run, so its bound is about
    2.5e-6 of the value."""
    from paper_1701_03512_amd import workloads
    gold = json.load(open(os.path.join(GOLD, "oracle_values.json")))
    limit = 1e-12 if precision == "fp64" else 3e-6
    for e in gold["exact_tv"]:
        sp = e["spec"]
        steps = [gbt.bt_params(s, sp["r"], sp["T"], sp["N"], sp["scheme"]) for s in sp["sigma_t"]]
        u_t, p_t = [a for a, _ in steps], [b for _, b in steps]
        opt = gbt.Option(sp["S"], u_t[0], p_t[0], sp["r"], sp["T"], sp["K"], sp["N"], sp["payoff"])
        r = gbt.bt_price_exact_tv(opt, u_t, p_t, precision)
        ob = bounds.oracle_rounding(e["value"], sp["S"], sp["K"], sp["r"], sp["T"], sp["N"],
                                    bounds.forward_growth(None, None, sp["N"], u_t, p_t))
        assert abs(r["value"] - e["value"]) <= r["err_bound"] + ob, (sp["payoff"], r, e["value"])
        assert r["err_bound"] <= limit * abs(r["value"])
    for e in gold["exact_tri"]:
        sp = e["spec"]
        u, pu, pd = gbt.bt_params_trinomial(sp["sigma"], sp["r"], sp["T"], sp["N"], sp["lam"])
        opt = gbt.Option(sp["S"], u, pu, sp["r"], sp["T"], sp["K"], sp["N"], sp["payoff"])
        r = gbt.bt_price_exact_trinomial(opt, pd, precision)
        ob = bounds.oracle_rounding(e["value"], sp["S"], sp["K"], sp["r"], sp["T"], sp["N"],
                                    bounds.forward_growth(u, pu, sp["N"], p_down=pd))
        assert abs(r["value"] - e["value"]) <= r["err_bound"] + ob, (sp["payoff"], r, e["value"])
        assert r["err_bound"] <= limit * abs(r["value"])
    assert workloads  # recipes come from the same module as the stored values


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_bound_in_batch_equals_bound_alone(gbt, precision):
    """The bound is computed from the option's own tables and sums in a
    fixed order, so it is the same bits alone and in a batch."""
    from paper_1701_03512_amd import workloads
    specs = workloads.random_options(24, seed=3, n_lo=8, n_hi=20, payoffs=PAYOFFS)
    opts = [gbt.make_option(s["S"], s["K"], s["sigma"], s["r"], s["T"], s["N"], s["payoff"])
            for s in specs]
    batch = gbt.bt_price_batch(opts, precision)
    for o, b in zip(opts, batch):
        one = gbt.bt_price_exact(o, precision)
        assert b["err_bound"] == one["err_bound"] and b["value"] == one["value"]
