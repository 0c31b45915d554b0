"""The autotuner (runs last: it changes the library's tuning table for the
depths it measures)."""
import pytest

import batch_gold

pytestmark = pytest.mark.gpu


def test_autotune_picks_valid_shapes_and_keeps_values(gbt, orc):
    before = {N: gbt.bt_tuning_for(N) for N in (12, 13, 14)}
    vals = {}
    for N in (12, 13, 14):
        g = gbt.make_option(100.0, 100.0, 0.25, 0.03, 1.0, N, "asian_call")
        vals[N] = (g, gbt.bt_price_exact(g)["value"])
    gbt.bt_autotune(12, 14, "fp64")
    for N in (12, 13, 14):
        t = gbt.bt_tuning_for(N)
        assert 1 <= t["k"] <= min(N, 16) and t["chunk"] % 4 == 0 and 4 <= t["chunk"] <= 2048
        g, v0 = vals[N]
        o = orc.make_option(100.0, 100.0, 0.25, 0.03, 1.0, N, "asian_call")
        v1 = gbt.bt_price_exact(g)["value"]
        assert abs(v1 - orc.price_naive(o)) <= 1e-12 * abs(v1)
        assert abs(v1 - v0) <= 1e-13 * abs(v0)
    assert before  # tuning table was readable before autotuning


def test_autotune_on_a_batch_keeps_batch_equal_to_single(gbt, orc):
    """bt_autotune_batch: the tuning it installs applies to every depth of
    the batch; afterwards a batch still equals its options priced alone and
    matches the oracle."""
    from paper_1701_03512_amd import workloads
    specs = workloads.random_options(64, seed=5, n_lo=10, n_hi=18)
    opts = [gbt.make_option(s["S"], s["K"], s["sigma"], s["r"], s["T"], s["N"], s["payoff"])
            for s in specs]
    gbt.bt_autotune_batch(opts, "fp64")
    for N in range(10, 19):
        t = gbt.bt_tuning_for(N)
        assert 1 <= t["k"] <= min(N, 16) and t["chunk"] % 4 == 0 and 4 <= t["chunk"] <= 2048
    batch = gbt.bt_price_batch(opts, "fp64")
    for sp, g, b in list(zip(specs, opts, batch))[:12]:
        assert b["value"] == gbt.bt_price_exact(g, "fp64")["value"]
        o = orc.make_option(sp["S"], sp["K"], sp["sigma"], sp["r"], sp["T"], sp["N"], sp["payoff"])
        want = orc.price_dfs(o, 2)
        assert abs(b["value"] - want) <= max(1e-12 * abs(want), 1e-15 * sp["S"])


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_full_batch_4096_autotuned(gbt, precision):
    """The benchmark's 4096-option batch (N 16..30, 5.5e11 paths) after
    bt_autotune_batch, priced in one launch as the benchmark times it:
    every option against the oracle's stored value (eq. (f13)), and six of
    the N=30 ones equal to their one-option price bit for bit."""
    from paper_1701_03512_amd import workloads
    specs = workloads.random_options(4096)
    opts = [gbt.make_option(s["S"], s["K"], s["sigma"], s["r"], s["T"], s["N"], s["payoff"])
            for s in specs]
    gbt.bt_autotune_batch(opts, precision)
    batch = gbt.bt_price_batch(opts, precision)
    assert len(batch) == 4096
    batch_gold.check_all(precision, opts, batch, "autotuned shapes")
    deep = [i for i, s in enumerate(specs) if s["N"] == 30][:6]
    for i in deep:
        assert batch[i]["value"] == gbt.bt_price_exact(opts[i], precision)["value"], i


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_server_prices_with_builtin_shapes_after_autotune(gbt, precision):
    """The server keeps its one-tree launch shapes whatever bt_autotune has
    installed, so its results do not change when a batch is autotuned."""
    opts = [gbt.make_option(100.0, 95.0, 0.2, 0.05, 1.0, N, "asian_call") for N in (24, 29)]

    def serve_all():
        srv = gbt.Server(mem_budget=1 << 30, precision=precision, exact_max_n=34)
        ts = [srv.submit(o) for o in opts]
        out = []
        for t in ts:
            while True:
                r = srv.poll(t)
                if r is not None:
                    break
            out.append(r[0])
        srv.close()
        return out

    r0 = serve_all()
    gbt.bt_autotune(24, 29, precision)
    t24 = gbt.bt_tuning_for(24, precision)
    assert (t24["k"], t24["chunk"]) != (10, 128)  # the autotuned shape differs from the built-in one
    r1 = serve_all()
    for a, b in zip(r0, r1):
        assert a["status"] == b["status"] == 0
        assert a["value"] == b["value"] and a["split"] == b["split"]
    assert [r["split"] for r in r0] == [10, 11]
    # equal to bt_price_exact with the one-tree shapes passed explicitly
    for o, r, tune in zip(opts, r0, ({"k": 10, "chunk": 128}, {"k": 11, "chunk": 512})):
        assert r["value"] == gbt.bt_price_exact(o, precision, tune=tune)["value"]
