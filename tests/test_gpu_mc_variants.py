"""Proportional allocation and the Shared-Sample estimator on the GPU
(through bt_price_mc) against the CPU oracle on the same Philox draws:
1e-12 relative with FP64 paths, 1e-6 with FP32 paths."""
import math

import pytest

pytestmark = pytest.mark.gpu


def close(got, want, precision, floor):
    if math.isnan(want):
        return math.isnan(got)
    tol = 1e-12 if precision == "fp64" else 1e-6
    return abs(got - want) <= tol * abs(want) + floor


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
@pytest.mark.parametrize("payoff", ["asian_call", "asian_put", "lookback_float", "lookback_fixed_put"])
def test_proportional_matches_oracle(gbt, orc, payoff, precision):
    g = gbt.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 14, payoff)
    o = orc.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 14, payoff)
    disc = math.exp(-o.r * o.T)
    for r, R in ((3, 1000), (6, 4096), (9, 65536), (12, 9000)):
        res = gbt.bt_price_mc(g, "proportional", r, R, seed=21, stream_id=4, precision=precision)
        th, vpi, vub, vpaper, n = orc.mc_proportional(o, r, R, 21, 4)
        assert res["paths"] == n
        fl = 1e-15 * 100 if precision == "fp64" else 1e-9 * 100
        assert close(res["value"], disc * th, precision, fl), (r, R, res["value"], disc * th)
        assert close(res["var_est"], disc * disc * vpaper, precision, fl * 1e-3), (r, R)
        assert close(res["var_unbiased"], disc * disc * vub, precision, fl * 1e-3), (r, R)
        sec = orc.mc_proportional_second(o, r, R, 21, 4)
        vpl = disc * disc * (sec - th * th) / n
        assert close(res["var_plain"], vpl, precision, fl * 1e-3), (r, R, res["var_plain"], vpl)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_proportional_many_items_n64(gbt, orc, precision):
    """N=64 with 2^16 strata and R = 2^22 (about 64 draws per stratum, the
    up-count order of the lane kernel over 1024 work items) against the
    oracle on the same draws."""
    g = gbt.make_option(100.0, 100.0, 0.2, 0.05, 1.0, 64, "asian_call")
    o = orc.make_option(100.0, 100.0, 0.2, 0.05, 1.0, 64, "asian_call")
    disc = math.exp(-o.r * o.T)
    r, R = 16, 2 ** 22
    res = gbt.bt_price_mc(g, "proportional", r, R, seed=8, stream_id=1, precision=precision)
    th, vpi, vub, vpaper, n = orc.mc_proportional(o, r, R, 8, 1)
    assert res["paths"] == n
    fl = 1e-15 * 100 if precision == "fp64" else 1e-9 * 100
    assert close(res["value"], disc * th, precision, fl), (res["value"], disc * th)
    assert close(res["var_est"], disc * disc * vpaper, precision, fl * 1e-3)
    assert close(res["var_unbiased"], disc * disc * vub, precision, fl * 1e-3)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
@pytest.mark.parametrize("payoff", ["asian_call", "asian_put", "lookback_float", "lookback_fixed_put",
                                    "euro_call"])
def test_shared_sample_matches_oracle(gbt, orc, payoff, precision):
    g = gbt.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 14, payoff)
    o = orc.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 14, payoff)
    disc = math.exp(-o.r * o.T)
    for r, R in ((2, 50), (6, 1024), (10, 3000)):
        res = gbt.bt_price_mc(g, "shared_sample", r, R, seed=8, stream_id=3, precision=precision)
        th, vpi, vub = orc.mc_shared(o, r, R, 8, 3)
        assert res["paths"] == R * 2 ** r
        fl = 1e-15 * 100 if precision == "fp64" else 1e-9 * 100
        assert close(res["value"], disc * th, precision, fl), (r, R, res["value"], disc * th)
        assert close(res["var_est"], disc * disc * vpi, precision, 1e-6 * disc * disc * vpi), (r, R)
        assert math.isnan(res["var_plain"])


def test_shared_sample_paper_table5_n32(gbt):
    """N=32 Asian put (Section 5 parameters), R = 1024 shared draws, M = 64
    strata: the variance estimate averages near the printed 0.123
    (Table 5), and Partitioned MC with R_m = R estimates a smaller variance
    (Theorem 1)."""
    g = gbt.make_option(20.0, 100.0, 3.0, 0.06, 1.0, 32, "asian_put", "seydel")
    vs = [gbt.bt_price_mc(g, "shared_sample", 6, 1024, seed=100 + i)["var_est"] for i in range(64)]
    assert sum(vs) / len(vs) == pytest.approx(0.123, rel=0.12)
    part = gbt.bt_price_mc(g, "partitioned", 6, 1024, seed=7)
    assert part["var_est"] < sum(vs) / len(vs)
    assert abs(part["value"] - 82.115) < 5 * part["std_err"]


def test_proportional_paper_table4_n32(gbt):
    """Table 4 (R = 2^10, M = 64 strata, proportional): the 1/R^2 variance
    estimate averages near the printed 0.194 (the oracle's average over
    these repetitions sits about 9% below it)."""
    g = gbt.make_option(20.0, 100.0, 3.0, 0.06, 1.0, 32, "asian_put", "seydel")
    vs = [gbt.bt_price_mc(g, "proportional", 6, 1024, seed=200 + i)["var_est"] for i in range(400)]
    assert sum(vs) / len(vs) == pytest.approx(0.194, rel=0.12)


def test_shared_sample_full_size(gbt):
    """N=64 floating lookback, 2^20 strata x 1024 shared draws (2^30 paths at
    enumeration speed) against the exact lattice value."""
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")))
    e = gold["lookback_dp"][0]
    sp = e["spec"]
    g = gbt.make_option(sp["S"], sp["K"], sp["sigma"], sp["r"], sp["T"], sp["N"], sp["payoff"])
    for precision in ("fp64", "fp32_kahan"):
        res = gbt.bt_price_mc(g, "shared_sample", 20, 1024, seed=3, precision=precision)
        assert res["paths"] == 2 ** 30
        assert abs(res["value"] - e["value"]) < 5 * math.sqrt(res["var_unbiased"])


def test_estimator_argument_checks(gbt):
    g = gbt.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 30, "asian_call")
    with pytest.raises(gbt.BtError):
        gbt.bt_price_mc(g, "shared_sample", 27, 16, seed=1)      # r > 26
    with pytest.raises(gbt.BtError):
        gbt.bt_price_mc(g, "proportional", 5, 2 ** 31, seed=1)   # R > 2^30


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_proportional_single_draw_strata(gbt, orc, precision):
    """R below the stratum count: one draw per stratum, unbiased form NaN,
    as in the oracle."""
    g = gbt.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 8, "asian_call")
    o = orc.make_option(100.0, 100.0, 0.3, 0.05, 1.0, 8, "asian_call")
    res = gbt.bt_price_mc(g, "proportional", 4, 1, seed=5, stream_id=0, precision=precision)
    th, pi, ub, vpaper, n = orc.mc_proportional(o, 4, 1, 5, 0)
    assert res["paths"] == n == 16 and vpaper == 0.0
    assert close(res["value"], math.exp(-o.r * o.T) * th, precision, 1e-13)
    assert res["var_est"] == 0.0 and math.isnan(res["var_unbiased"]) and math.isnan(ub)
