"""Seeded synthetic workloads: option parameters only.

This module draws contract and market parameters (S, K, sigma, r, T, N,
payoff name) and arrival times.  It holds none of the method's arithmetic (no
tree parameters, no weights, no payoffs): both the GPU library's callers and
the CPU oracle's callers turn these into (u, p) with their own routines.

The paper's workloads are fixed parameter sets (Section 5: a put with K=10,
S=5, sigma=0.30, q=6%, T=1 for the timing runs; an Asian put and a fixed
lookback put with K=100, S=20, q=6%, sigma=3.0, T=1, N=32 for the Monte Carlo
study).  The benchmark configurations below follow the same recipe: CRR
parameters with dt = T/N, u = exp(sigma sqrt(dt)), d = 1/u.
"""
from __future__ import annotations

import numpy as np

PAYOFF_NAMES = ("asian_call", "asian_put", "lookback_float",
                "lookback_fixed_put", "euro_call", "euro_put")

# The three path-dependent payoffs of the N=32 benchmark workload.
BENCH_PAYOFFS = ("asian_call", "asian_put", "lookback_float")

DEFAULT_SEED = 170103512


def spec(S, K, sigma, r, T, N, payoff, scheme="crr"):
    return {"S": float(S), "K": float(K), "sigma": float(sigma), "r": float(r),
            "T": float(T), "N": int(N), "payoff": payoff, "scheme": scheme}


def exact_small():
    """Exact enumeration, N=20: fixed-strike arithmetic-average Asian call
    over S_1..S_N, S=K=100, r=0.05, sigma=0.2, T=1 (CRR)."""
    return spec(100, 100, 0.2, 0.05, 1.0, 20, "asian_call")


def exact_n32():
    """Exact enumeration, N=32 (2^32 paths), same market, three payoffs:
    Asian call, Asian put (K=100), floating lookback max_t S_t - S_N."""
    return [spec(100, 100, 0.2, 0.05, 1.0, 32, p) for p in BENCH_PAYOFFS]


def term_structure_sigmas(N, lo=0.15, hi=0.30, jitter=0.0, seed=DEFAULT_SEED + 11):
    """Per-step volatilities sigma_1..sigma_N for time-varying trees: a
    linear ramp from lo to hi (a rising volatility term structure), plus
    optional seeded uniform jitter of +-jitter.  Each step's (u_t, p_t) is
    then the caller's tree-parameter routine applied to (sigma_t, r, T, N)."""
    ramp = [lo + (hi - lo) * (t / (N - 1) if N > 1 else 0.0) for t in range(N)]
    if jitter:
        g = np.random.default_rng(seed)
        ramp = [s + float(x) for s, x in zip(ramp, g.uniform(-jitter, jitter, size=N))]
    return ramp


def exact_tv_n32():
    """Time-varying exact enumeration, N=32: the N=32 market and payoffs
    with the volatility ramping from 0.15 to 0.30 over the steps."""
    return [dict(s, sigma_t=term_structure_sigmas(32)) for s in exact_n32()]


def exact_tri_n20(lam=1.224744871391589):
    """Trinomial exact enumeration, N=20 (3^20 = 3.49e9 paths, about the
    2^32 of the binomial N=32 workload): the same market and payoffs with
    Boyle's stretch lambda = sqrt(3/2)."""
    return [dict(spec(100, 100, 0.2, 0.05, 1.0, 20, p), lam=lam) for p in BENCH_PAYOFFS]


def paper_mc_study(payoff="asian_put", N=32):
    """Section 5 Monte Carlo study: K=100, S=20, q=6%, sigma=3.0, T=1,
    Seydel's parameters."""
    return spec(20, 100, 3.0, 0.06, 1.0, N, payoff, scheme="seydel")


def paper_timing_put(N):
    """Section 5 timing workload: a put with K=10, S=5, sigma=0.30, q=6%,
    T=1 (valued over all 2^N paths)."""
    return spec(5, 10, 0.30, 0.06, 1.0, N, "euro_put", scheme="seydel")


def random_options(n, seed=DEFAULT_SEED, n_lo=16, n_hi=30,
                   payoffs=BENCH_PAYOFFS):
    """Batch recipe: N ~ UniformInt[n_lo, n_hi], S ~ U(50,150),
    K/S ~ U(0.8,1.2), sigma ~ U(0.1,0.5), T ~ U(0.25,2), r ~ U(0,0.08),
    payoff uniform over `payoffs`."""
    g = np.random.default_rng(seed)
    N = g.integers(n_lo, n_hi + 1, size=n)
    S = g.uniform(50.0, 150.0, size=n)
    KS = g.uniform(0.8, 1.2, size=n)
    sig = g.uniform(0.1, 0.5, size=n)
    T = g.uniform(0.25, 2.0, size=n)
    r = g.uniform(0.0, 0.08, size=n)
    pay = g.integers(0, len(payoffs), size=n)
    return [spec(S[i], KS[i] * S[i], sig[i], r[i], T[i], N[i], payoffs[pay[i]])
            for i in range(n)]


def stratified_mc():
    """Prefix-stratified MC workload: N=64, 2^24 prefix strata of the first 24
    steps, 64 suffix draws of 40 steps per stratum, the N=20 workload's market
    with dt = T/64; Asian call and floating lookback."""
    base = dict(S=100, K=100, sigma=0.2, r=0.05, T=1.0, N=64)
    return {"options": [spec(**base, payoff=p) for p in ("asian_call", "lookback_float")],
            "prefix_steps": 24, "samples_per_stratum": 64,
            "seed": 0x5EED1701}


def mc_variants():
    """The Section 4 estimators on the stratified-MC market (N=64), each at
    2^30 paths: Partitioned MC with proportional allocation over 2^24
    strata (R = 2^30 in total), and Shared-Sample MC with 2^20 prefixes
    evaluated exactly against R = 1024 shared suffix draws of 44 steps."""
    base = stratified_mc()
    return {"options": base["options"], "seed": base["seed"],
            "proportional": {"prefix_steps": 24, "samples": 2 ** 30},
            "shared_sample": {"prefix_steps": 20, "samples": 1024}}


def poisson_arrivals(rate_hz, duration_s, seed=DEFAULT_SEED + 5):
    """Open-loop arrival times (seconds) with exponential gaps of mean
    1/rate_hz, up to duration_s."""
    g = np.random.default_rng(seed)
    n_guess = int(rate_hz * duration_s * 1.2) + 16
    t = np.cumsum(g.exponential(1.0 / rate_hz, size=n_guess))
    while t[-1] < duration_s:
        t = np.concatenate([t, t[-1] + np.cumsum(g.exponential(1.0 / rate_hz, size=n_guess))])
    return t[t < duration_s]


def serving_options(n, seed=DEFAULT_SEED + 7):
    """Serving recipe: as the batch recipe but N ~ UniformInt[16, 64]."""
    return random_options(n, seed=seed, n_lo=16, n_hi=64)
