"""Partitioned Monte Carlo on the GPU (through the C ABI) against the CPU
oracle, which draws the same Philox4x32-10 streams: sampled suffix bits are
compared exactly; estimates and variance estimates to 1e-12 relative with
FP64 paths and 1e-6 with FP32 paths.  At full size (N=64, 2^24 strata x 64
draws) the estimate is checked against the exact value of a lattice
recursion, and at N=32 against exact enumeration (the estimator's validation
case)."""
import json
import math
import os

import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rel_ok(got, want, precision, scale=1.0):
    tol = 1e-12 if precision == "fp64" else 1e-6
    return abs(got - want) <= tol * max(abs(want), 1e-300) + (1e-15 if precision == "fp64" else 1e-9) * scale


def pair(bt, orc, S, K, sigma, r, T, N, payoff):
    g = bt.make_option(S, K, sigma, r, T, N, payoff)
    o = orc.make_option(S, K, sigma, r, T, N, payoff)
    return g, o


def test_suffix_bits_bit_exact(gbt, orc):
    p = 0.5167980141148621
    thr = orc.up_threshold(p)
    for (seed, stream, z, m, L) in [(0, 0, 0, 0, 40), (0x5EED1701, 3, 12345, 63, 40),
                                    (2 ** 64 - 1, 2 ** 32 - 1, 2 ** 24 - 1, 7, 64), (9, 1, 5, 4096, 7)]:
        assert gbt.bt_mc_debug_bits(seed, stream, z, m, L, p) == orc.mc_suffix_bits(seed, stream, z, m, L, thr)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
@pytest.mark.parametrize("payoff", ["asian_call", "asian_put", "lookback_float",
                                    "lookback_fixed_put", "euro_call", "euro_put"])
def test_stratified_matches_oracle(gbt, orc, payoff, precision):
    g, o = pair(gbt, orc, 100.0, 100.0, 0.3, 0.05, 1.0, 14, payoff)
    for (r, Rm) in [(4, 16), (6, 64), (3, 100), (9, 1)]:
        res = gbt.bt_price_stratified(g, r, Rm, seed=77, stream_id=5, precision=precision)
        v, vpi, vub = orc.mc_stratified(o, r, Rm, 77, 5)
        assert res["paths"] == Rm * 2 ** r and res["split"] == r
        assert rel_ok(res["value"], v, precision, g.S), (r, Rm, res["value"], v)
        assert rel_ok(res["var_est"], vpi, precision, 1e-6), (r, Rm, res["var_est"], vpi)
        if Rm > 1:
            assert rel_ok(res["var_unbiased"], vub, precision, 1e-6)
        vpl = orc.mc_stratified_plain_var(o, r, Rm, 77, 5)
        assert rel_ok(res["var_plain"], vpl, precision, 1e-6), (r, Rm, res["var_plain"], vpl)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_plain_mc_matches_oracle(gbt, orc, precision):
    g, o = pair(gbt, orc, 100.0, 105.0, 0.25, 0.05, 1.0, 20, "asian_call")
    for R in (1000, 8192, 20000):
        res = gbt.bt_price_stratified(g, 0, R, seed=3, stream_id=1, precision=precision)
        v, vpi, vub = orc.mc_stratified(o, 0, R, 3, 1)
        assert rel_ok(res["value"], v, precision, g.S), (R, res["value"], v)
        assert rel_ok(res["var_est"], vpi, precision, 1e-6), (R, res["var_est"], vpi)
        assert res["var_plain"] == res["var_est"]  # basic MC is plain MC


def test_stratified_n32_against_exact(gbt):
    """Validation at N=32: r=24 prefix strata x 64 draws of the last 8 steps
    vs the exact enumeration value; and the estimated variance is below the
    basic-MC variance at the same count (eq. (mc15))."""
    gold = json.load(open(os.path.join(GOLD, "oracle_values.json")))
    for e in gold["exact"]:
        sp = e["spec"]
        if sp["N"] != 32:
            continue
        g = gbt.make_option(sp["S"], sp["K"], sp["sigma"], sp["r"], sp["T"], 32, sp["payoff"])
        for precision in ("fp64", "fp32_kahan"):
            res = gbt.bt_price_stratified(g, 24, 64, seed=0x5EED1701, stream_id=0, precision=precision)
            se = math.sqrt(res["var_unbiased"])
            assert abs(res["value"] - e["value"]) < 5 * se, (sp["payoff"], res["value"], e["value"], se)
        plain = gbt.bt_price_stratified(g, 0, 2 ** 22, seed=11, stream_id=0, precision="fp64")
        strat = gbt.bt_price_stratified(g, 16, 64, seed=11, stream_id=0, precision="fp64")
        assert strat["var_est"] < plain["var_est"]
        # the plain-MC variance the stratified draws imply agrees with the
        # basic run's own estimate (both at 2^22 paths)
        assert strat["var_plain"] == pytest.approx(plain["var_est"], rel=0.05)


@pytest.mark.parametrize("precision", ["fp32_kahan", "fp64"])
def test_stratified_full_size_lookback(gbt, precision):
    """N=64, 2^24 strata x 64 draws of 40 steps (the full workload): the
    floating lookback estimate lies within 5 standard errors of the exact
    value from the lattice recursion."""
    gold = json.load(open(os.path.join(GOLD, "oracle_values.json")))
    e = gold["lookback_dp"][0]
    sp = e["spec"]
    g = gbt.make_option(sp["S"], sp["K"], sp["sigma"], sp["r"], sp["T"], sp["N"], sp["payoff"])
    res = gbt.bt_price_stratified(g, 24, 64, seed=0x5EED1701, stream_id=0, precision=precision)
    se = math.sqrt(res["var_unbiased"])
    assert res["paths"] == 2 ** 30
    assert abs(res["value"] - e["value"]) < 5 * se, (res["value"], e["value"], se)


def test_mc_many_strata_matches_oracle(gbt, orc):
    """2^20 strata (16384 work items, the full-size launch structure) of an
    N=22 tree with R_m=4, compared in full with the oracle's draws."""
    g, o = pair(gbt, orc, 100.0, 100.0, 0.2, 0.05, 1.0, 22, "asian_call")
    res = gbt.bt_price_stratified(g, 20, 4, seed=1, stream_id=2, precision="fp64")
    v, vpi, vub = orc.mc_stratified(o, 20, 4, 1, 2)
    assert rel_ok(res["value"], v, "fp64", g.S), (res["value"], v)
    assert rel_ok(res["var_est"], vpi, "fp64", 1e-9), (res["var_est"], vpi)


def test_mc_deterministic(gbt):
    g = gbt.make_option(100.0, 100.0, 0.2, 0.05, 1.0, 40, "lookback_fixed_put")
    a = gbt.bt_price_stratified(g, 12, 64, seed=5, precision="fp32_kahan")
    b = gbt.bt_price_stratified(g, 12, 64, seed=5, precision="fp32_kahan")
    assert a == b  # bit-identical
    # a Monte Carlo estimate's error figure is its standard error
    assert a["err_bound"] == a["std_err"] > 0


@pytest.mark.parametrize("payoff", ["asian_call", "asian_put", "lookback_float"])
def test_variance_estimate_vs_exact_strata(gbt, orc, payoff):
    """N=24, 2^16 prefix strata x 64 draws: the 1/(R_m - 1) variance
    estimate is within 2% of the exact variance of the estimator,
    e^{-2rT} sum_z P(D_z)^2 Var[V | D_z] / R_m (eq. (mc13)), computed by the
    oracle by enumerating all 2^24 paths; the estimate is within 4 standard
    errors of the exact value."""
    g, o = pair(gbt, orc, 100.0, 100.0, 0.2, 0.05, 1.0, 24, payoff)
    ex = orc.exact_strata(o, 16)
    disc2 = math.exp(-2 * o.r * o.T)
    want_var = disc2 * ex["within_sq"] / 64
    res = gbt.bt_price_stratified(g, 16, 64, seed=77, stream_id=1, precision="fp64")
    assert abs(res["var_unbiased"] - want_var) <= 0.02 * want_var, (res["var_unbiased"], want_var)
    assert abs(res["value"] - math.exp(-o.r * o.T) * ex["mean"]) < 4 * math.sqrt(want_var)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
@pytest.mark.parametrize("payoff", ["asian_call", "lookback_float", "lookback_fixed_put", "euro_put"])
def test_few_draws_per_stratum_match_oracle(gbt, orc, payoff, precision):
    """R_m below 64 (several strata per wave pass, including counts that are
    not powers of two and strata counts that are not multiples of the
    pass), against the oracle on the same draws."""
    g, o = pair(gbt, orc, 100.0, 98.0, 0.3, 0.05, 1.0, 16, payoff)
    for (r, Rm) in [(7, 1), (5, 2), (6, 3), (8, 4), (3, 5), (9, 8), (4, 16), (6, 31), (5, 32), (7, 63)]:
        res = gbt.bt_price_stratified(g, r, Rm, seed=123, stream_id=9, precision=precision)
        v, vpi, vub = orc.mc_stratified(o, r, Rm, 123, 9)
        assert res["paths"] == Rm * 2 ** r
        assert rel_ok(res["value"], v, precision, g.S), (r, Rm, res["value"], v)
        assert rel_ok(res["var_est"], vpi, precision, 1e-6), (r, Rm, res["var_est"], vpi)
        if Rm > 1:
            assert rel_ok(res["var_unbiased"], vub, precision, 1e-6), (r, Rm)
        else:
            assert math.isnan(res["var_unbiased"])
        vpl = orc.mc_stratified_plain_var(o, r, Rm, 123, 9)
        assert rel_ok(res["var_plain"], vpl, precision, 1e-6), (r, Rm, res["var_plain"], vpl)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
@pytest.mark.parametrize("payoff", ["asian_put", "lookback_float", "lookback_fixed_put"])
def test_flat_layout_matches_oracle(gbt, orc, payoff, precision):
    """R_m above 64 and not a multiple of 64 (the flat sample layout: strata
    cut by wave-pass boundaries, several strata in one pass, a stratum
    spanning many passes), against the oracle on the same draws."""
    g, o = pair(gbt, orc, 100.0, 103.0, 0.3, 0.05, 1.0, 16, payoff)
    for (r, Rm) in [(7, 65), (6, 100), (8, 129), (2, 1000), (10, 191), (1, 4097)]:
        res = gbt.bt_price_stratified(g, r, Rm, seed=31, stream_id=2, precision=precision)
        v, vpi, vub = orc.mc_stratified(o, r, Rm, 31, 2)
        assert res["paths"] == Rm * 2 ** r
        assert rel_ok(res["value"], v, precision, g.S), (r, Rm, res["value"], v)
        assert rel_ok(res["var_est"], vpi, precision, 1e-6), (r, Rm, res["var_est"], vpi)
        assert rel_ok(res["var_unbiased"], vub, precision, 1e-6), (r, Rm)
        vpl = orc.mc_stratified_plain_var(o, r, Rm, 31, 2)
        assert rel_ok(res["var_plain"], vpl, precision, 1e-6), (r, Rm, res["var_plain"], vpl)


def test_suffix_bits_bit_exact_on_ties(gbt, orc):
    """Thresholds chosen so that a step's 16-bit half ties with the
    threshold's high half: the GPU draws the same fallback and takes the
    same decisions as the oracle."""
    seed, stream, z, m = 0x0DDBA11, 3, 777, 41
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for L in (8, 13, 40):
        for j in (0, 5, L - 1):
            w = orc.philox4x32_10([j // 8, m, z, stream], key)[(j % 8) // 2]
            h = w >> 16 if j % 2 == 0 else w & 0xFFFF
            g = orc.philox4x32_10([0x80000000 + j, m, z, stream], key)[0] >> 16
            for lo in (0, g, min(g + 1, 0xFFFF)):
                thr = (h << 16) | lo
                p = (thr + 0.5) / 2 ** 32
                if not 0.0 < p < 1.0:
                    continue
                assert orc.up_threshold(p) == thr
                want = orc.mc_suffix_bits(seed, stream, z, m, L, thr)
                assert gbt.bt_mc_debug_bits(seed, stream, z, m, L, p) == want, (L, j, lo)
                assert want[j] == (1 if g < lo else 0)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_suffix_lengths_around_block_boundaries(gbt, orc, precision):
    """Suffixes of 1, 7, 8, 9, 16 and 17 steps (one Philox block serves eight
    steps): the walk's offsets and partial blocks match the oracle's draws."""
    for N, r in [(9, 8), (14, 7), (14, 6), (14, 5), (20, 4), (20, 3)]:
        for payoff in ("asian_call", "lookback_float", "lookback_fixed_put", "euro_call"):
            g, o = pair(gbt, orc, 100.0, 101.0, 0.3, 0.04, 1.0, N, payoff)
            res = gbt.bt_price_stratified(g, r, 64, seed=404, stream_id=3, precision=precision)
            v, vpi, vub = orc.mc_stratified(o, r, 64, 404, 3)
            assert rel_ok(res["value"], v, precision, g.S), (N, r, payoff, res["value"], v)
            assert rel_ok(res["var_est"], vpi, precision, 1e-6), (N, r, payoff)


def test_full_size_n64_equals_oracle_on_the_same_draws(gbt, orc):
    """The benchmark's stratified MC at full size (N=64 Asian call, 2^24
    strata x 64 draws of 40 steps, its seed and stream) against the oracle
    evaluating every one of the 2^30 paths with the same Philox draws (the
    strata split over host threads, partial sums added in stratum order):
    1e-12 relative with FP64 paths, 1e-6 with FP32 paths."""
    import concurrent.futures
    from paper_1701_03512_amd import workloads
    mc = workloads.stratified_mc()
    sp = mc["options"][0]
    r, Rm, seed = mc["prefix_steps"], mc["samples_per_stratum"], mc["seed"]
    o = orc.make_option(sp["S"], sp["K"], sp["sigma"], sp["r"], sp["T"], sp["N"], sp["payoff"])
    nchunks = 256
    per = (1 << r) // nchunks
    with concurrent.futures.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        parts = list(ex.map(lambda c: orc.mc_stratified_range(o, r, Rm, seed, 0, c * per, (c + 1) * per),
                            range(nchunks)))
    disc = math.exp(-sp["r"] * sp["T"])
    want = disc * math.fsum(p[0] for p in parts)
    want_var = disc * disc * math.fsum(p[1] for p in parts)
    g = gbt.make_option(sp["S"], sp["K"], sp["sigma"], sp["r"], sp["T"], sp["N"], sp["payoff"])
    for precision in ("fp64", "fp32_kahan"):
        res = gbt.bt_price_stratified(g, r, Rm, seed=seed, stream_id=0, precision=precision)
        assert res["paths"] == 2 ** 30
        assert rel_ok(res["value"], want, precision, g.S), (precision, res["value"], want)
        assert rel_ok(res["var_est"], want_var, precision, 1e-9), (precision, res["var_est"], want_var)
