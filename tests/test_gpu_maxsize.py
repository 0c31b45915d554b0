"""The largest trees each exact entry point accepts, checked through
properties the oracle can evaluate at that size: European payoffs against
backward induction, lookbacks against the lattice recursion over (level,
running extreme), the Asian average against its closed form (K = 0) and
Asian put-call parity.  N=40 binomial (2^40 paths), N=40 time-varying,
N=26 trinomial (3^26 paths)."""
import math

import pytest

pytestmark = pytest.mark.gpu


def close(got, want, S, precision):
    if precision == "fp64":
        return abs(got - want) <= max(1e-12 * abs(want), 1e-15 * S)
    return abs(got - want) <= max(1e-6 * abs(want), 1e-9 * S)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_binomial_n40(gbt, orc, precision):
    S, r, T, N = 100.0, 0.05, 1.0, 40
    for payoff, K in (("euro_call", 103.0), ("euro_put", 97.0)):
        g = gbt.make_option(S, K, 0.25, r, T, N, payoff)
        o = orc.make_option(S, K, 0.25, r, T, N, payoff)
        got = gbt.bt_price_exact(g, precision)
        assert got["paths"] == 2 ** 40
        assert close(got["value"], orc.euro_backward(o), S, precision), payoff
    for payoff, K in (("lookback_float", 100.0), ("lookback_fixed_put", 104.0)):
        g = gbt.make_option(S, K, 0.25, r, T, N, payoff)
        o = orc.make_option(S, K, 0.25, r, T, N, payoff)
        want, _ = orc.lookback_dp(o)
        assert close(gbt.bt_price_exact(g, precision)["value"], want, S, precision), payoff
    # Asian: closed-form average (K = 0) and put-call parity at K = 100
    g0 = gbt.make_option(S, 0.0, 0.25, r, T, N, "asian_call")
    gr = g0.p * g0.u + (1 - g0.p) / g0.u
    mean = math.exp(-r * T) * S / N * math.fsum(gr ** t for t in range(1, N + 1))
    assert close(gbt.bt_price_exact(g0, precision)["value"], mean, S, precision)
    c = gbt.bt_price_exact(gbt.make_option(S, 100.0, 0.25, r, T, N, "asian_call"), precision)["value"]
    p = gbt.bt_price_exact(gbt.make_option(S, 100.0, 0.25, r, T, N, "asian_put"), precision)["value"]
    parity = mean - math.exp(-r * T) * 100.0
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert abs((c - p) - parity) <= tol * max(c, p)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_time_varying_n40(gbt, precision):
    from paper_1701_03512_amd import workloads
    S, r, T, N = 100.0, 0.05, 1.0, 40
    uv = [gbt.bt_params(s, r, T, N) for s in workloads.term_structure_sigmas(N, jitter=0.02)]
    u = [a for a, _ in uv]
    p = [b for _, b in uv]
    gr = [pi * ui + (1 - pi) / ui for ui, pi in zip(u, p)]
    disc = math.exp(-r * T)
    fwd = disc * S * math.prod(gr)
    mean = disc * S / N * math.fsum(math.prod(gr[:t + 1]) for t in range(N))
    o = lambda payoff, K: gbt.Option(S, u[0], p[0], r, T, K, N, payoff)
    got = gbt.bt_price_exact_tv(o("euro_call", 0.0), u, p, precision)
    assert got["paths"] == 2 ** 40
    assert close(got["value"], fwd, S, precision)
    assert close(gbt.bt_price_exact_tv(o("asian_call", 0.0), u, p, precision)["value"], mean, S, precision)
    c = gbt.bt_price_exact_tv(o("euro_call", 100.0), u, p, precision)["value"]
    q = gbt.bt_price_exact_tv(o("euro_put", 100.0), u, p, precision)["value"]
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert abs((c - q) - (fwd - disc * 100.0)) <= tol * max(c, q)


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_trinomial_n26(gbt, orc, precision):
    S, r, T, N = 100.0, 0.05, 1.0, 26
    u, pu, pd = gbt.bt_params_trinomial(0.25, r, T, N, 1.224744871391589)
    for payoff, K in (("euro_call", 102.0), ("euro_put", 98.0)):
        g = gbt.Option(S, u, pu, r, T, K, N, payoff)
        o = orc.Option(S, u, pu, r, T, K, N, payoff)
        got = gbt.bt_price_exact_trinomial(g, pd, precision)
        assert got["paths"] == 3 ** 26
        assert close(got["value"], orc.tri_euro_backward(o, pd), S, precision), payoff
    gr = pu * u + (1 - pu - pd) + pd / u
    mean = math.exp(-r * T) * S / N * math.fsum(gr ** t for t in range(1, N + 1))
    g0 = gbt.Option(S, u, pu, r, T, 0.0, N, "asian_call")
    assert close(gbt.bt_price_exact_trinomial(g0, pd, precision)["value"], mean, S, precision)
