"""Pins of the oracle's trinomial-tree form of eq. (f13) (3^N paths,
base-3 digits, first step most significant, 0 = down, 1 = middle, 2 = up):
exact rational brute force, the binomial limit (middle probability 0)
against the pinned binomial oracle, European backward induction on the
recombining lattice, closed forms for the forward and the Asian mean, and
the moment-matched parameters against Boyle's closed-form probabilities."""
import itertools
import math
from fractions import Fraction

import pytest

PAYOFFS = ("asian_call", "asian_put", "lookback_float", "lookback_fixed_put", "euro_call", "euro_put")


def brute_fraction(S, K, u, pu, pd, N, payoff):
    pm = 1 - pu - pd
    tot = Fraction(0)
    for dg in itertools.product((0, 1, 2), repeat=N):
        lev, w, path = 0, Fraction(1), []
        for d in dg:
            lev += d - 1
            w *= (pd, pm, pu)[d]
            path.append(Fraction(S) * (u ** lev))
        mean = sum(path) / N
        f = {"asian_call": max(mean - K, 0), "asian_put": max(K - mean, 0),
             "lookback_float": max(path) - path[-1], "lookback_fixed_put": max(K - min(path), 0),
             "euro_call": max(path[-1] - K, 0), "euro_put": max(K - path[-1], 0)}[payoff]
        tot += w * f
    return tot


def test_digits(orc):
    assert orc.tri_digits(5, 3) == [0, 1, 2]
    assert orc.tri_digits(26, 3) == [2, 2, 2]
    seen = {tuple(orc.tri_digits(x, 4)) for x in range(81)}
    assert len(seen) == 81


def test_moment_matched_parameters(orc):
    """pu u + pm + pd/u = e^{r dt}, pu u^2 + pm + pd/u^2 = e^{(2r + sigma^2) dt},
    and Boyle's closed forms pu = ((V + M^2 - M) u - (M - 1)) / ((u - 1)(u^2 - 1)),
    pd = ((V + M^2 - M) u^2 - (M - 1) u^3) / ((u - 1)(u^2 - 1)),
    M = e^{r dt}, V = M^2 (e^{sigma^2 dt} - 1)."""
    for s, r, T, N, lam in [(0.2, 0.05, 1.0, 20, 1.2247), (0.3, 0.03, 2.0, 10, 1.5)]:
        u, pu, pd = orc.params_trinomial(s, r, T, N, lam)
        h = T / N
        assert u == pytest.approx(math.exp(lam * s * math.sqrt(h)), rel=1e-15)
        pm = 1 - pu - pd
        assert pu * u + pm + pd / u == pytest.approx(math.exp(r * h), rel=1e-14)
        assert pu * u * u + pm + pd / (u * u) == pytest.approx(math.exp((2 * r + s * s) * h), rel=1e-14)
        M = math.exp(r * h)
        V = M * M * (math.exp(s * s * h) - 1)
        assert pu == pytest.approx(((V + M * M - M) * u - (M - 1)) / ((u - 1) * (u * u - 1)), rel=1e-12)
        assert pd == pytest.approx(((V + M * M - M) * u * u - (M - 1) * u ** 3) / ((u - 1) * (u * u - 1)),
                                   rel=1e-12)
    with pytest.raises(ValueError):
        orc.params_trinomial(0.25, 0.0, 1.0, 16, 1.0)  # middle probability not positive


@pytest.mark.parametrize("payoff", PAYOFFS)
def test_tiny_trees_exact_rational(orc, payoff):
    u, pu, pd = Fraction(5, 4), Fraction(3, 10), Fraction(1, 5)
    for N in (1, 2, 3, 4):
        want = float(brute_fraction(100, 100, u, pu, pd, N, payoff))
        o = orc.Option(100.0, 1.25, 0.3, 0.0, 1.0, 100.0, N, payoff)
        for got in (orc.price_tri_naive(o, 0.2), orc.price_tri(o, 0.2, 2)):
            assert got == pytest.approx(want, rel=1e-14, abs=1e-13), (N, got, want)


@pytest.mark.parametrize("payoff", PAYOFFS)
def test_binomial_limit(orc, payoff):
    """Middle probability 0: the trinomial sum is the binomial one."""
    b = orc.make_option(100.0, 97.0, 0.3, 0.04, 1.0, 11, payoff)
    want = orc.price_naive(b)
    t = orc.Option(b.S, b.u, b.p, b.r, b.T, b.K, b.N, payoff)
    assert orc.price_tri(t, 1.0 - b.p, 3) == pytest.approx(want, rel=1e-13, abs=1e-13)


@pytest.mark.parametrize("payoff", ("euro_call", "euro_put"))
def test_european_backward_induction(orc, payoff):
    u, pu, pd = orc.params_trinomial(0.25, 0.05, 1.0, 12, 1.2247)
    o = orc.Option(100.0, u, pu, 0.05, 1.0, 103.0, 12, payoff)
    assert orc.price_tri(o, pd) == pytest.approx(orc.tri_euro_backward(o, pd), rel=1e-12)


def test_forward_and_asian_mean(orc):
    N = 12
    u, pu, pd = orc.params_trinomial(0.2, 0.05, 1.0, N, 1.3)
    g = pu * u + (1 - pu - pd) + pd / u
    disc = math.exp(-0.05)
    fwd = orc.price_tri(orc.Option(100.0, u, pu, 0.05, 1.0, 0.0, N, "euro_call"), pd)
    assert fwd == pytest.approx(disc * 100.0 * g ** N, rel=1e-13)
    assert fwd == pytest.approx(100.0, rel=1e-12)  # moment matching: a martingale
    mean = orc.price_tri(orc.Option(100.0, u, pu, 0.05, 1.0, 0.0, N, "asian_call"), pd)
    assert mean == pytest.approx(disc * 100.0 / N * math.fsum(g ** t for t in range(1, N + 1)), rel=1e-13)


@pytest.mark.parametrize("payoff", PAYOFFS)
def test_naive_and_depth_first_agree(orc, payoff):
    u, pu, pd = orc.params_trinomial(0.3, 0.02, 1.0, 9, 1.2)
    o = orc.Option(100.0, u, pu, 0.02, 1.0, 100.0, 9, payoff)
    assert orc.price_tri(o, pd, 3) == pytest.approx(orc.price_tri_naive(o, pd), rel=1e-14, abs=1e-14)
