"""Launch shapes against the oracle: every shape the batch and the one-shot
calls can take must give the value of eq. (f13).  Section 3 splits the sum
over paths into blocks by their leading steps; how the paths are split (the
suffix length k, the prefixes per rectangle, the number of workgroups) must
not change the result beyond rounding.

Runs before the autotuner's tests, so `tune=None` here means the built-in
shapes.  Tolerances as everywhere: FP64 |rel err| <= 1e-12 (floor 1e-15 S),
FP32-Kahan |rel err| <= 1e-6 (floor 1e-9 S)."""
import json
import os

import pytest

import batch_gold

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PAYOFFS = ("asian_call", "asian_put", "lookback_float", "lookback_fixed_put",
           "euro_call", "euro_put")
TOL = {"fp64": (1e-12, 1e-15), "fp32_kahan": (1e-6, 1e-9)}


def check(got, want, S, precision):
    rel, floor = TOL[precision]
    return abs(got - want) <= max(rel * abs(want), floor * S)


def spec_option(bt, sp):
    return bt.make_option(sp["S"], sp["K"], sp["sigma"], sp["r"], sp["T"], sp["N"], sp["payoff"])


@pytest.fixture(scope="module")
def shapes_gold():
    gold = json.load(open(os.path.join(GOLD, "oracle_values.json")))
    rows = gold["shapes"]
    assert sorted({e["spec"]["N"] for e in rows}) == [24, 26, 28, 30]
    return rows


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
@pytest.mark.parametrize("N", [24, 26, 28, 30])
def test_deep_trees_every_split_and_chunk(gbt, shapes_gold, N, precision):
    """The N=32 market's three payoffs at N = 24..30 under the built-in
    shape and under every split the autotuner picks in the 4096-option
    batch (k = 12..15) with 1024- and 2048-prefix rectangles."""
    rows = [e for e in shapes_gold if e["spec"]["N"] == N]
    assert len(rows) == 3
    tunes = [None] + [{"k": k, "chunk": c} for k in (12, 13, 14, 15) for c in (1024, 2048)]
    for e in rows:
        g = spec_option(gbt, e["spec"])
        for tune in tunes:
            r = gbt.bt_price_exact(g, precision, tune=tune)
            assert r["status"] == 0 and r["paths"] == 2 ** N
            if tune:
                assert r["split"] == tune["k"]
            assert check(r["value"], e["value"], g.S, precision), \
                (N, e["spec"]["payoff"], tune, r["value"], e["value"])


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
@pytest.mark.parametrize("payoff", PAYOFFS)
def test_every_split_8_to_16_at_n20(gbt, orc, payoff, precision):
    """k = 8..16 at N = 20 (the autotuner's range), all six payoffs."""
    g = gbt.make_option(95.0, 100.0, 0.3, 0.04, 1.25, 20, payoff)
    o = orc.make_option(95.0, 100.0, 0.3, 0.04, 1.25, 20, payoff)
    want = orc.price_dfs(o, min(16, os.cpu_count() or 1))
    for k in range(8, 17):
        r = gbt.bt_price_exact(g, precision, tune={"k": k})
        assert r["split"] == k
        assert check(r["value"], want, g.S, precision), (k, r["value"], want)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_persistent_grids(gbt, orc, precision):
    """bt_tuning.grid > 0: a fixed number of workgroups loops over the
    rectangles (g, g + grid, ...).  The partial slots do not depend on which
    workgroup fills them, so every grid gives the same bits as one
    workgroup per rectangle, and the oracle's value."""
    from paper_1701_03512_amd import workloads
    specs = workloads.random_options(48, seed=11, n_lo=10, n_hi=22, payoffs=PAYOFFS)
    opts = [spec_option(gbt, s) for s in specs]
    want = [orc.price_dfs(orc.make_option(s["S"], s["K"], s["sigma"], s["r"], s["T"], s["N"],
                                          s["payoff"]), min(16, os.cpu_count() or 1))
            for s in specs]
    # small rectangles, so that the batch has about a thousand of them
    shape = {"k": 10, "chunk": 64}
    plan = gbt.Plan(opts, precision, tune=shape)
    nrect = plan.info()["grid"]
    plan.close()
    assert nrect > 512
    base = gbt.bt_price_batch(opts, precision, tune=shape)
    for grid in (7, 64, 512):
        tune = dict(shape, grid=grid)
        plan = gbt.Plan(opts, precision, tune=tune)
        assert plan.info()["grid"] == grid
        plan.close()
        got = gbt.bt_price_batch(opts, precision, tune=tune)
        for s, g, b, w in zip(specs, got, base, want):
            assert g["status"] == 0
            assert g["value"] == b["value"], (grid, s)
            assert check(g["value"], w, s["S"], precision), (grid, s, g["value"], w)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_full_batch_4096_builtin_shapes(gbt, precision):
    """The 4096-option batch (N 16..30, 5.5e11 paths) in one launch with the
    built-in shapes, every option against the oracle."""
    from paper_1701_03512_amd import workloads
    specs = workloads.random_options(4096)
    opts = [spec_option(gbt, s) for s in specs]
    batch_gold.check_all(precision, opts, gbt.bt_price_batch(opts, precision),
                         "built-in shapes")
