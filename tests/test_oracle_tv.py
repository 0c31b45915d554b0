"""Pins of the oracle's time-varying form of eq. (f13) (per-step u_t, p_t,
d_t = 1/u_t, p(x) = prod p_t^{x_t} (1 - p_t)^{1 - x_t}): exact rational
brute force on tiny trees, the constant-parameter special case, closed
forms for the forward and the Asian mean, a risk-neutral martingale check
and the step-permutation invariance of European payoffs."""
import itertools
import math
import random
from fractions import Fraction

import pytest

PAYOFFS = ("asian_call", "asian_put", "lookback_float", "lookback_fixed_put", "euro_call", "euro_put")


def brute_fraction(S, K, u, p, payoff):
    """E[f] over all 2^N paths in exact rational arithmetic (undiscounted)."""
    N = len(u)
    tot = Fraction(0)
    for bits in itertools.product((0, 1), repeat=N):
        St, w, path = Fraction(S), Fraction(1), []
        for t, b in enumerate(bits):
            St = St * u[t] if b else St / u[t]
            w *= p[t] if b else 1 - p[t]
            path.append(St)
        mean = sum(path) / N
        f = {"asian_call": max(mean - K, 0), "asian_put": max(K - mean, 0),
             "lookback_float": max(path) - path[-1], "lookback_fixed_put": max(K - min(path), 0),
             "euro_call": max(path[-1] - K, 0), "euro_put": max(K - path[-1], 0)}[payoff]
        tot += w * f
    return tot


def opt(orc, N, payoff, S=100.0, K=100.0, r=0.0, T=1.0):
    # u and p of the Option are ignored by the time-varying entry points
    return orc.Option(S, 1.1, 0.5, r, T, K, N, payoff)


@pytest.mark.parametrize("payoff", PAYOFFS)
def test_tiny_trees_exact_rational(orc, payoff):
    u = [Fraction(11, 10), Fraction(5, 4), Fraction(6, 5), Fraction(21, 20)]
    p = [Fraction(1, 2), Fraction(2, 5), Fraction(3, 5), Fraction(7, 10)]
    for N in (1, 2, 3, 4):
        want = float(brute_fraction(100, 100, u[:N], p[:N], payoff))
        o = opt(orc, N, payoff)
        uf, pf = [float(x) for x in u[:N]], [float(x) for x in p[:N]]
        for got in (orc.price_tv_naive(o, uf, pf), orc.price_tv(o, uf, pf, 2)):
            assert got == pytest.approx(want, rel=1e-14, abs=1e-13), (N, got, want)


def test_two_step_by_hand(orc):
    """u = (1.1, 1.25), p = (0.5, 0.4), S = K = 100, r = 0: the paths up-up,
    up-down, down-up, down-down end at 137.5, 88, 1250/11, 800/11 with
    weights 0.2, 0.3, 0.2, 0.3; the Asian call pays 23.75 on up-up and
    25/11 on down-up, so its value is 0.2 (23.75 + 25/11) = 229/44."""
    o = opt(orc, 2, "asian_call")
    assert orc.price_tv(o, [1.1, 1.25], [0.5, 0.4], 1) == pytest.approx(229 / 44, rel=1e-15)
    o = opt(orc, 2, "euro_call")
    # up-up pays 37.5, down-up 1250/11 - 100 = 150/11
    assert orc.price_tv(o, [1.1, 1.25], [0.5, 0.4], 1) == pytest.approx(0.2 * 37.5 + 0.2 * 150 / 11,
                                                                        rel=1e-15)


@pytest.mark.parametrize("payoff", PAYOFFS)
def test_constant_steps_reduce_to_the_fixed_tree(orc, payoff):
    o = orc.make_option(100.0, 97.0, 0.3, 0.04, 1.0, 12, payoff)
    want = orc.price_naive(o)
    got = orc.price_tv(o, [o.u] * 12, [o.p] * 12, 4)
    assert got == pytest.approx(want, rel=1e-13, abs=1e-13)


def _random_steps(N, seed):
    g = random.Random(seed)
    return [g.uniform(1.02, 1.2) for _ in range(N)], [g.uniform(0.3, 0.7) for _ in range(N)]


def test_forward_and_asian_mean_closed_forms(orc):
    """K = 0: the European call is E[S_N] = S prod_t g_t and the Asian call
    E[mean S_t] = (S/N) sum_t prod_{i<=t} g_i, g_t = p_t u_t + (1-p_t)/u_t."""
    N = 14
    u, p = _random_steps(N, 3)
    g = [pi * ui + (1 - pi) / ui for ui, pi in zip(u, p)]
    fwd = 100.0 * math.prod(g)
    mean = 100.0 / N * math.fsum(math.prod(g[:t + 1]) for t in range(N))
    assert orc.price_tv(opt(orc, N, "euro_call", K=0.0), u, p) == pytest.approx(fwd, rel=1e-13)
    assert orc.price_tv(opt(orc, N, "asian_call", K=0.0), u, p) == pytest.approx(mean, rel=1e-13)


def test_risk_neutral_martingale(orc):
    """p_t = (e^{r dt} - 1/u_t) / (u_t - 1/u_t) for any u_t: the discounted
    forward equals S."""
    N, r, T = 16, 0.05, 1.0
    u, _ = _random_steps(N, 5)
    dt = T / N
    p = [(math.exp(r * dt) - 1 / x) / (x - 1 / x) for x in u]
    got = orc.price_tv(opt(orc, N, "euro_call", K=0.0, r=r, T=T), u, p)
    assert got == pytest.approx(100.0, rel=1e-13)


@pytest.mark.parametrize("payoff", ("euro_call", "euro_put"))
def test_european_invariant_under_step_permutation(orc, payoff):
    """S_N is a product over the steps, so permuting the (u_t, p_t) pairs
    leaves a European price unchanged (and an Asian one, in general, not)."""
    N = 12
    u, p = _random_steps(N, 9)
    perm = list(range(N))
    random.Random(1).shuffle(perm)
    a = orc.price_tv(opt(orc, N, payoff), u, p)
    b = orc.price_tv(opt(orc, N, payoff), [u[i] for i in perm], [p[i] for i in perm])
    assert a == pytest.approx(b, rel=1e-13)
    sa = orc.price_tv(opt(orc, N, "asian_call"), u, p)
    sb = orc.price_tv(opt(orc, N, "asian_call"), [u[i] for i in perm], [p[i] for i in perm])
    assert abs(sa - sb) > 1e-6


@pytest.mark.parametrize("payoff", PAYOFFS)
def test_naive_and_depth_first_agree(orc, payoff):
    N = 14
    u, p = _random_steps(N, 11)
    o = opt(orc, N, payoff, r=0.03)
    assert orc.price_tv(o, u, p, 3) == pytest.approx(orc.price_tv_naive(o, u, p), rel=1e-14, abs=1e-14)


def test_argument_checks(orc):
    o = opt(orc, 3, "asian_call")
    assert math.isnan(orc.price_tv(o, [1.1, 0.9, 1.1], [0.5, 0.5, 0.5]))   # u_t <= 1
    assert math.isnan(orc.price_tv(o, [1.1, 1.1, 1.1], [0.5, 1.0, 0.5]))   # p_t = 1
    with pytest.raises(ValueError):
        orc.price_tv(o, [1.1, 1.1], [0.5, 0.5])
