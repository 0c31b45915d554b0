"""The autotuner (runs last: it changes the library's tuning table for the
depths it measures)."""
import pytest

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
