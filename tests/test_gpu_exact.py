"""Parity of the HIP exact enumeration (through the C ABI) with the CPU
oracle.  Tolerances: FP64 |rel err| <= 1e-12 (absolute floor 1e-15 S);
FP32 with Kahan sums |rel err| <= 1e-6 (absolute floor 1e-9 S, for values
near zero where the FP32 rounding of X - Y near the strike does not shrink
with the value).  Integer table contents are compared exactly."""
import json
import os
import random
from dataclasses import replace

import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PAYOFFS = ("asian_call", "asian_put", "lookback_float", "lookback_fixed_put",
           "euro_call", "euro_put")


def close(got, want, S, precision):
    if precision == "fp64":
        return abs(got - want) <= max(1e-12 * abs(want), 1e-15 * S)
    return abs(got - want) <= max(1e-6 * abs(want), 1e-9 * S)


def pair(bt, orc, S, K, sigma, r, T, N, payoff, scheme="crr"):
    g = bt.make_option(S, K, sigma, r, T, N, payoff, scheme)
    o = orc.make_option(S, K, sigma, r, T, N, payoff, scheme)
    assert (g.u, g.p) == (o.u, o.p)
    return g, o


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
@pytest.mark.parametrize("payoff", PAYOFFS)
@pytest.mark.parametrize("N", [1, 2, 3, 5, 8, 12, 17])
def test_small_trees_all_payoffs(gbt, orc, N, payoff, precision):
    g, o = pair(gbt, orc, 100.0, 97.0, 0.3, 0.04, 1.0, N, payoff)
    want = orc.price_naive(o)
    got = gbt.bt_price_exact(g, precision)
    assert got["status"] == 0 and got["paths"] == 2 ** N
    assert close(got["value"], want, g.S, precision), (got["value"], want)


# The server's launch shapes for one tree at a time: depth -> (k, FP64 chunk,
# FP32 chunk), as documented with bt_server_config.
ONE_TREE = {11: (10, 128, 128), 22: (10, 128, 128), 25: (10, 128, 128), 26: (10, 256, 256),
            28: (10, 512, 256), 29: (11, 512, 512), 30: (16, 512, 512), 31: (16, 512, 512)}


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
@pytest.mark.parametrize("N", sorted(ONE_TREE))
def test_one_tree_shapes_each_regime(gbt, orc, N, precision):
    """Each regime of the one-tree launch shapes against the oracle's
    enumeration."""
    import os
    k, c64, c32 = ONE_TREE[N]
    g, o = pair(gbt, orc, 100.0, 105.0, 0.25, 0.04, 1.0, N, "asian_put")
    got = gbt.bt_price_exact(g, precision, tune={"k": k, "chunk": c64 if precision == "fp64" else c32})
    assert got["split"] == k
    want = orc.price_dfs(o, min(16, os.cpu_count() or 1))
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert abs(got["value"] - want) <= tol * abs(want), (N, precision, got, want)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_two_step_tree_by_hand(gbt, precision):
    """The hand-worked N=2 tree (S=100, u=1.1, p=0.5, r=0, K=100)."""
    g = json.load(open(os.path.join(GOLD, "two_step_tree.json")))
    from fractions import Fraction
    import math
    for case in g["cases"]:
        for payoff, v in case["values"].items():
            opt = gbt.Option(case["S"], case["u"], case["p"], case["r"], case["T"], case["K"],
                             case["N"], payoff)
            want = math.exp(-case["r"] * case["T"]) * float(Fraction(v["value"]))
            got = gbt.bt_price_exact(opt, precision)["value"]
            assert close(got, want, case["S"], precision), (payoff, got, want)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_exact_n20_workload(gbt, orc, precision):
    """N=20 Asian call, S=K=100, r=0.05, sigma=0.2, T=1 (CRR)."""
    from paper_1701_03512_amd import workloads
    sp = workloads.exact_small()
    g, o = pair(gbt, orc, sp["S"], sp["K"], sp["sigma"], sp["r"], sp["T"], sp["N"], sp["payoff"])
    want = orc.price_dfs(o)
    got = gbt.bt_price_exact(g, precision)["value"]
    assert close(got, want, g.S, precision), (got, want)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_exact_n32_workload(gbt, precision):
    """N=32 (2^32 paths), three payoffs, against oracle values stored by
    tests/golden/make_oracle_values.py; the launch shape is the default one
    the benchmark uses."""
    gold = json.load(open(os.path.join(GOLD, "oracle_values.json")))
    rows = [e for e in gold["exact"] if e["spec"]["N"] == 32]
    assert len(rows) == 3
    for e in rows:
        sp = e["spec"]
        g = gbt.make_option(sp["S"], sp["K"], sp["sigma"], sp["r"], sp["T"], sp["N"], sp["payoff"])
        got = gbt.bt_price_exact(g, precision)
        assert got["paths"] == 2 ** 32
        assert close(got["value"], e["value"], g.S, precision), (sp["payoff"], got["value"], e["value"])


def test_paper_section5_values(gbt):
    """Seydel parameters, N=32: the paper prints 82.115 (Asian put) and
    93.196 (fixed lookback put)."""
    gold = json.load(open(os.path.join(GOLD, "paper_section5_exact.json")))
    P = gold["params"]
    for payoff, want in gold["values"].items():
        g = gbt.make_option(P["S"], P["K"], P["sigma"], P["r"], P["T"], P["N"], payoff, P["scheme"])
        got = gbt.bt_price_exact(g, "fp64")["value"]
        assert abs(got - want) <= 0.5e-3, (payoff, got)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_split_and_chunk_do_not_change_the_value(gbt, orc, precision):
    g, o = pair(gbt, orc, 90.0, 100.0, 0.35, 0.03, 1.5, 14, "asian_put")
    want = orc.price_naive(o)
    vals = []
    for k in (1, 3, 6, 8, 10, 14):
        for chunk in (4, 8, 64, 256):
            r = gbt.bt_price_exact(g, precision, tune={"k": k, "chunk": chunk})
            assert r["split"] == k
            vals.append(r["value"])
            assert close(r["value"], want, g.S, precision), (k, chunk, r["value"], want)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_tables_bit_exact(gbt, orc, precision):
    """Prefix positions hold every P-step prefix once, in up-count order (ties
    by index: both precisions of a binomial tree share W_a c_a over each
    up-count group); up-counts of prefixes and suffixes equal the oracle's
    path bits."""
    g = gbt.make_option(100.0, 100.0, 0.2, 0.05, 1.0, 13, "lookback_float")
    k = 6
    P = 13 - k
    plan = gbt.Plan([g], precision, tune={"k": k, "chunk": 16})
    plan.tables()
    z, a, b = plan.debug_tables(0, P, k)
    plan.close()
    assert sorted(z) == list(range(2 ** P))
    keys = [(a[q], z[q]) for q in range(2 ** P)]
    assert keys == sorted(keys)
    for q in range(2 ** P):
        assert a[q] == sum(orc.path_of_index(z[q], P))
    for s in range(2 ** k):
        assert b[s] == sum(orc.path_of_index(s, k))


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_batch_equals_single_bitwise(gbt, precision):
    """A mixed batch (one persistent launch) gives each option exactly the
    value it gets alone."""
    rnd = random.Random(7)
    opts = []
    for i in range(24):
        N = rnd.randint(1, 18)
        opts.append(gbt.make_option(rnd.uniform(50, 150), rnd.uniform(60, 140), rnd.uniform(0.1, 0.5),
                                    rnd.uniform(0.0, 0.08), rnd.uniform(0.25, 2.0), N,
                                    PAYOFFS[i % 6]))
    batch = gbt.bt_price_batch(opts, precision)
    for o, b in zip(opts, batch):
        single = gbt.bt_price_exact(o, precision)
        assert b["value"] == single["value"]
        assert b["status"] == 0


def test_batch_matches_oracle(gbt, orc):
    from paper_1701_03512_amd import workloads
    specs = workloads.random_options(40, n_lo=4, n_hi=18,
                                     payoffs=workloads.PAYOFF_NAMES)
    gs, want = [], []
    for sp in specs:
        g, o = pair(gbt, orc, sp["S"], sp["K"], sp["sigma"], sp["r"], sp["T"], sp["N"], sp["payoff"])
        gs.append(g)
        want.append(orc.price_dfs(o, 2))
    for precision in ("fp64", "fp32_kahan"):
        got = gbt.bt_price_batch(gs, precision)
        for g, r, w in zip(gs, got, want):
            assert close(r["value"], w, g.S, precision), (g, r["value"], w)


def test_repeat_bitwise_deterministic(gbt):
    g = gbt.make_option(100.0, 100.0, 0.2, 0.05, 1.0, 24, "lookback_float")
    v = {gbt.bt_price_exact(g, "fp64")["value"] for _ in range(3)}
    assert len(v) == 1


def test_graph_replays_match_eager(gbt):
    import torch
    s = torch.cuda.Stream()
    opts = [gbt.make_option(100.0, 100.0, 0.2, 0.05, 1.0, 22, p)
            for p in ("asian_call", "asian_put", "lookback_float")]
    eager = [r["value"] for r in gbt.bt_price_batch(opts, "fp64")]
    plan = gbt.Plan(opts, "fp64")
    with torch.cuda.stream(s):
        plan.capture(s)
        for rep in range(4):
            plan.launch_graph(s)
            got = [r["value"] for r in plan.results(s)]
            assert got == eager, rep
            # unrelated eager work between replays
            x = torch.randn(1 << 16, device="cuda")
            torch.cuda.synchronize()
            del x
    plan.close()


def test_plan_stages_and_info(gbt, orc):
    g, o = pair(gbt, orc, 100.0, 100.0, 0.2, 0.05, 1.0, 16, "euro_call")
    plan = gbt.Plan([g], "fp64", tune={"k": 10, "chunk": 32})
    info = plan.info()
    assert info["k"] == 10 and info["chunk"] == 32
    # one 1024-suffix tile x (64 prefixes / 32) chunks, four waves sharing the tile
    assert info["items"] == 8
    plan.tables()
    plan.enumerate()
    plan.reduce()
    r = plan.results()[0]
    plan.close()
    assert close(r["value"], orc.euro_backward(o), g.S, "fp64")


def test_deep_tree_range_error(gbt):
    g = gbt.make_option(100.0, 100.0, 0.2, 0.05, 1.0, 41, "asian_call")
    with pytest.raises(gbt.BtError) as e:
        gbt.bt_price_exact(g)
    assert e.value.code == gbt.BT_ERANGE
