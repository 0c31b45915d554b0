"""Helpers for checking the library's per-result error bound (err_bound).

exact_binomial(): eq. (f13) in exact rational arithmetic over all 2^N paths,
taking the option's FP64 inputs (S, u, p, K) as exact binary fractions, so
that |value - exact| <= err_bound can be checked with nothing else rounding
(r = 0 keeps the discount exactly 1).  Small trees only.

oracle_rounding(): a bound on the oracle's own rounding error.  The oracle
forms every price in FP64 (S u^j d^(i-j): about N + 6 roundings, library pow
included), sums N of them, divides and subtracts (Asian payoffs), multiplies
by an FP64 weight (another N + 6) and accumulates in long double; the error
of a path's payoff is then at most (2N + 10) 2^-53 times the size of the
prices it touches, and only paths whose payoff can be nonzero count.  Those
sizes are bounded through the value itself, the strike and the expected
final price: mean <= payoff + K where the call is in the money, mean, min,
S_N <= K where a put is, max <= payoff + S_N for the floating lookback.
"""
from fractions import Fraction
import math

U64 = 2.0 ** -53


def exact_binomial(S, u, p, K, N, payoff):
    S, u, p, K = (Fraction(x) for x in (S, u, p, K))
    price = {l: S * u ** l for l in range(-N, N + 1)}
    q = 1 - p
    total = Fraction(0)
    for x in range(2 ** N):
        ups, lev, s = 0, 0, Fraction(0)
        mx = mn = None
        for t in range(1, N + 1):
            bit = (x >> (N - t)) & 1
            ups += bit
            lev += 1 if bit else -1
            St = price[lev]
            s += St
            mx = St if mx is None or St > mx else mx
            mn = St if mn is None or St < mn else mn
        last = price[lev]
        mean = s / N
        f = {"asian_call": max(mean - K, 0), "asian_put": max(K - mean, 0),
             "lookback_float": mx - last, "lookback_fixed_put": max(K - mn, 0),
             "euro_call": max(last - K, 0), "euro_put": max(K - last, 0)}[payoff]
        total += p ** ups * q ** (N - ups) * f
    return total


def forward_growth(u, p, N, u_t=None, p_t=None, p_down=None):
    """E[S_N] / S: (p u + (1 - p)/u)^N, its time-varying product, or the
    trinomial (p u + pm + pd / u)^N."""
    if u_t is not None:
        g = 1.0
        for a, b in zip(u_t, p_t):
            g *= b * a + (1.0 - b) / a
        return g
    if p_down is not None:
        return (p * u + (1.0 - p - p_down) + p_down / u) ** N
    return (p * u + (1.0 - p) / u) ** N


def oracle_rounding(value, S, K, r, T, N, growth):
    """Bound on |oracle - exact| for a value of this size (see above)."""
    disc = math.exp(-r * T)
    size = abs(value) / disc + 2.0 * K + 2.0 * S * growth
    return 1.001 * ((2 * N + 10) * U64 * disc * size + (N + 10) * U64 * abs(value))
