"""Python access to the plain CPU reference (``bt_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py``; never by the product package.
It shares no code with the GPU library: its own C source, its own enums, its
own parameter routine.  Every function states the passage of the paper it
follows in ``bt_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PAYOFFS = {
    "asian_call": 0,
    "asian_put": 1,
    "lookback_float": 2,
    "lookback_fixed_put": 3,
    "euro_call": 4,
    "euro_put": 5,
}
SCHEMES = {"crr": 0, "seydel": 1}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-o", _LIB + ".tmp", _SRC, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Opt(ctypes.Structure):
    _fields_ = [("S", ctypes.c_double), ("u", ctypes.c_double),
                ("p", ctypes.c_double), ("r", ctypes.c_double),
                ("T", ctypes.c_double), ("K", ctypes.c_double),
                ("N", ctypes.c_int32), ("payoff", ctypes.c_int32)]


class _McSums(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("var_plugin", ctypes.c_double),
                ("var_unbiased", ctypes.c_double), ("second", ctypes.c_double)]


class _McRes(ctypes.Structure):
    _fields_ = [("value", ctypes.c_double), ("var_plugin", ctypes.c_double),
                ("var_unbiased", ctypes.c_double), ("var_plain", ctypes.c_double)]


class _Strata(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_double), ("var_total", ctypes.c_double),
                ("within", ctypes.c_double), ("between", ctypes.c_double),
                ("within_sq", ctypes.c_double), ("shared", ctypes.c_double),
                ("within_y", ctypes.c_double)]


class _Prop(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("var_plugin", ctypes.c_double),
                ("var_unbiased", ctypes.c_double), ("var_paper", ctypes.c_double),
                ("second", ctypes.c_double), ("samples", ctypes.c_uint64)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i32, u32, u64 = ctypes.c_double, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
        sig = {
            "orc_params": (ctypes.c_int, [d, d, d, ctypes.c_int, ctypes.c_int, P(d), P(d)]),
            "orc_path_of_index": (None, [u64, ctypes.c_int, P(ctypes.c_int)]),
            "orc_payoff_of_path": (d, [P(_Opt), P(ctypes.c_int)]),
            "orc_prob_of_path": (d, [P(_Opt), P(ctypes.c_int)]),
            "orc_price_naive": (d, [P(_Opt)]),
            "orc_range_naive": (d, [P(_Opt), u64, u64]),
            "orc_price_dfs": (d, [P(_Opt), ctypes.c_int]),
            "orc_subtree_sum": (d, [P(_Opt), ctypes.c_int, u64]),
            "orc_euro_closed": (d, [P(_Opt)]),
            "orc_euro_backward": (d, [P(_Opt)]),
            "orc_lookback_dp": (d, [P(_Opt), P(d)]),
            "orc_philox4x32_10": (None, [P(u32), P(u32), P(u32)]),
            "orc_up_threshold": (u32, [d]),
            "orc_mc_suffix_bits": (None, [u64, u32, u32, u32, ctypes.c_int, u32, P(ctypes.c_int)]),
            "orc_mc_stratified_range": (ctypes.c_int, [P(_Opt), ctypes.c_int, u32, u64, u32, u64, u64, P(_McSums)]),
            "orc_mc_stratified": (ctypes.c_int, [P(_Opt), ctypes.c_int, u32, u64, u32, P(_McRes)]),
            "orc_exact_strata": (ctypes.c_int, [P(_Opt), ctypes.c_int, P(_Strata)]),
            "orc_mc_proportional": (ctypes.c_int, [P(_Opt), ctypes.c_int, u64, u64, u32, P(_Prop)]),
            "orc_mc_shared": (ctypes.c_int, [P(_Opt), ctypes.c_int, u32, u64, u32, P(_McSums)]),
            "orc_mc_proportional_range": (ctypes.c_int, [P(_Opt), ctypes.c_int, u64, u64, u32,
                                                         u64, u64, P(_Prop)]),
            "orc_mc_shared_draws": (ctypes.c_int, [P(_Opt), ctypes.c_int, u64, u32, u32, u32,
                                                   P(ctypes.c_double)]),
            "orc_price_tv_naive": (d, [P(_Opt), P(d), P(d)]),
            "orc_price_tv": (d, [P(_Opt), P(d), P(d), ctypes.c_int]),
            "orc_params_trinomial": (ctypes.c_int, [d, d, d, ctypes.c_int, d, P(d), P(d), P(d)]),
            "orc_tri_digits": (None, [u64, ctypes.c_int, P(ctypes.c_int)]),
            "orc_price_tri_naive": (d, [P(_Opt), d]),
            "orc_price_tri": (d, [P(_Opt), d, ctypes.c_int]),
            "orc_tri_euro_backward": (d, [P(_Opt), d]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


@dataclass(frozen=True)
class Option:
    """One option on an N-step tree: (S, u, p, r, T, K, N, payoff)."""
    S: float
    u: float
    p: float
    r: float
    T: float
    K: float
    N: int
    payoff: str

    def _c(self) -> _Opt:
        return _Opt(self.S, self.u, self.p, self.r, self.T, self.K, self.N,
                    PAYOFFS[self.payoff])


def params(sigma: float, r: float, T: float, N: int, scheme: str = "crr"):
    """(u, p) from Section 2's assumptions A1-A3 (see bt_oracle.c)."""
    u, p = ctypes.c_double(), ctypes.c_double()
    rc = _L().orc_params(sigma, r, T, N, SCHEMES[scheme], ctypes.byref(u), ctypes.byref(p))
    if rc != 0:
        raise ValueError(f"orc_params failed ({rc})")
    return u.value, p.value


def make_option(S, K, sigma, r, T, N, payoff, scheme="crr") -> Option:
    u, p = params(sigma, r, T, N, scheme)
    return Option(S, u, p, r, T, K, N, payoff)


def path_of_index(x: int, N: int):
    arr = (ctypes.c_int * max(N, 1))()
    _L().orc_path_of_index(x, N, arr)
    return [arr[i] for i in range(N)]


def payoff_of_path(o: Option, bits) -> float:
    arr = (ctypes.c_int * len(bits))(*bits)
    c = o._c()
    return _L().orc_payoff_of_path(ctypes.byref(c), arr)


def prob_of_path(o: Option, bits) -> float:
    arr = (ctypes.c_int * len(bits))(*bits)
    c = o._c()
    return _L().orc_prob_of_path(ctypes.byref(c), arr)


def price_naive(o: Option) -> float:
    """Eq. (f13) one path at a time (discounted)."""
    c = o._c()
    return _L().orc_price_naive(ctypes.byref(c))


def range_naive(o: Option, x_begin: int, x_end: int) -> float:
    """Undiscounted sum of p(x) V(x) over path indices [x_begin, x_end)."""
    c = o._c()
    return _L().orc_range_naive(ctypes.byref(c), x_begin, x_end)


def price_dfs(o: Option, threads: int | None = None) -> float:
    """Eq. (f13) by depth-first enumeration, threads as Section 3 ranks."""
    if threads is None:
        threads = max(1, min(16, os.cpu_count() or 1))
    c = o._c()
    return _L().orc_price_dfs(ctypes.byref(c), threads)


def subtree_sum(o: Option, depth: int, z: int) -> float:
    """Undiscounted sum of p(x) V(x) over paths whose first `depth` steps spell z."""
    c = o._c()
    return _L().orc_subtree_sum(ctypes.byref(c), depth, z)


def euro_closed(o: Option) -> float:
    c = o._c()
    return _L().orc_euro_closed(ctypes.byref(c))


def euro_backward(o: Option) -> float:
    c = o._c()
    return _L().orc_euro_backward(ctypes.byref(c))


def lookback_dp(o: Option):
    """(discounted E[V], undiscounted E[V^2]) by the lattice recursion."""
    c = o._c()
    m2 = ctypes.c_double()
    v = _L().orc_lookback_dp(ctypes.byref(c), ctypes.byref(m2))
    return v, m2.value


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    out = (ctypes.c_uint32 * 4)()
    _L().orc_philox4x32_10(c, k, out)
    return [out[i] for i in range(4)]


def up_threshold(p: float) -> int:
    return _L().orc_up_threshold(p)


def mc_suffix_bits(seed: int, stream: int, z: int, m: int, L: int, thr: int):
    arr = (ctypes.c_int * max(L, 1))()
    _L().orc_mc_suffix_bits(seed, stream, z, m, L, thr, arr)
    return [arr[i] for i in range(L)]


def mc_stratified_range(o: Option, r: int, Rm: int, seed: int, stream: int,
                        z_begin: int, z_end: int):
    """Undiscounted (sum W_z thetahat_z, sum W_z^2 s_z^2/R_m plug-in, unbiased)
    over strata [z_begin, z_end)."""
    c = o._c()
    s = _McSums()
    rc = _L().orc_mc_stratified_range(ctypes.byref(c), r, Rm, seed, stream,
                                      z_begin, z_end, ctypes.byref(s))
    if rc != 0:
        raise ValueError(f"orc_mc_stratified_range failed ({rc})")
    return s.theta, s.var_plugin, s.var_unbiased


def mc_stratified(o: Option, r: int, Rm: int, seed: int, stream: int = 0):
    """Discounted Partitioned MC estimate and its variance estimates."""
    c = o._c()
    res = _McRes()
    rc = _L().orc_mc_stratified(ctypes.byref(c), r, Rm, seed, stream, ctypes.byref(res))
    if rc != 0:
        raise ValueError(f"orc_mc_stratified failed ({rc})")
    return res.value, res.var_plugin, res.var_unbiased


def mc_stratified_plain_var(o: Option, r: int, Rm: int, seed: int, stream: int = 0):
    """Discounted estimate of the variance plain MC would have with the
    same 2^r R_m paths, from the stratified draws: (sum_z P(D_z) mean_m
    V_zm^2 - theta_s^2) / (2^r R_m) (for r = 0, the plug-in variance)."""
    c = o._c()
    res = _McRes()
    rc = _L().orc_mc_stratified(ctypes.byref(c), r, Rm, seed, stream, ctypes.byref(res))
    if rc != 0:
        raise ValueError(f"orc_mc_stratified failed ({rc})")
    return res.var_plain


def mc_stratified_second(o: Option, r: int, Rm: int, seed: int, stream: int,
                         z_begin: int, z_end: int) -> float:
    """Undiscounted sum_z P(D_z) (1/R_m) sum_m V_zm^2 over strata
    [z_begin, z_end): the stratified estimate of E[V^2]."""
    c = o._c()
    s = _McSums()
    rc = _L().orc_mc_stratified_range(ctypes.byref(c), r, Rm, seed, stream,
                                      z_begin, z_end, ctypes.byref(s))
    if rc != 0:
        raise ValueError(f"orc_mc_stratified_range failed ({rc})")
    return s.second


def mc_proportional_second(o: Option, r: int, R: int, seed: int, stream: int = 0) -> float:
    """Undiscounted sum_m P(D_m) (1/R_m) sum_i V_mi^2 under proportional
    allocation (the draws of mc_proportional)."""
    c = o._c()
    s = _Prop()
    rc = _L().orc_mc_proportional(ctypes.byref(c), r, R, seed, stream, ctypes.byref(s))
    if rc != 0:
        raise ValueError(f"orc_mc_proportional failed ({rc})")
    return s.second


def exact_strata(o: Option, r: int):
    """Exact (undiscounted) mean, Var[V], sum P Var[V|D], Var E[V|D],
    sum P^2 Var[V|D] for a stratification on the first r steps."""
    c = o._c()
    s = _Strata()
    rc = _L().orc_exact_strata(ctypes.byref(c), r, ctypes.byref(s))
    if rc != 0:
        raise ValueError(f"orc_exact_strata failed ({rc})")
    return {"mean": s.mean, "var_total": s.var_total, "within": s.within,
            "between": s.between, "within_sq": s.within_sq, "shared": s.shared,
            "within_y": s.within_y}


def mc_proportional(o: Option, r: int, R: int, seed: int, stream: int = 0):
    """Partitioned MC with R_m = max(1, round(R P(D_m))): undiscounted
    (estimate, plug-in variance, 1/(R_m-1) variance, the paper's 1/R^2
    shortcut, total samples)."""
    c = o._c()
    s = _Prop()
    rc = _L().orc_mc_proportional(ctypes.byref(c), r, R, seed, stream, ctypes.byref(s))
    if rc != 0:
        raise ValueError(f"orc_mc_proportional failed ({rc})")
    return s.theta, s.var_plugin, s.var_unbiased, s.var_paper, s.samples


def mc_proportional_range(o: Option, r: int, R: int, seed: int, stream: int,
                          z_begin: int, z_end: int):
    """mc_proportional's sums over strata [z_begin, z_end) only:
    undiscounted (sum P(D_m) thetahat_m, plug-in variance sum, 1/(R_m-1)
    sum, the 1/R^2 sum, samples drawn)."""
    c = o._c()
    s = _Prop()
    rc = _L().orc_mc_proportional_range(ctypes.byref(c), r, R, seed, stream, z_begin, z_end,
                                        ctypes.byref(s))
    if rc != 0:
        raise ValueError(f"orc_mc_proportional_range failed ({rc})")
    return s.theta, s.var_plugin, s.var_unbiased, s.var_paper, s.samples


def mc_shared_draws(o: Option, r: int, seed: int, stream: int, i_begin: int, i_end: int):
    """Shared-Sample: h_i = sum_z P(D_z) V(z, y_i) (undiscounted) for the
    draws i in [i_begin, i_end)."""
    c = o._c()
    n = i_end - i_begin
    arr = (ctypes.c_double * max(n, 1))()
    rc = _L().orc_mc_shared_draws(ctypes.byref(c), r, seed, stream, i_begin, i_end, arr)
    if rc != 0:
        raise ValueError(f"orc_mc_shared_draws failed ({rc})")
    return [arr[i] for i in range(n)]


def mc_shared(o: Option, r: int, R: int, seed: int, stream: int = 0):
    """Shared-Sample MC: undiscounted (estimate, 1/R^2 variance, 1/(R(R-1)))."""
    c = o._c()
    s = _McSums()
    rc = _L().orc_mc_shared(ctypes.byref(c), r, R, seed, stream, ctypes.byref(s))
    if rc != 0:
        raise ValueError(f"orc_mc_shared failed ({rc})")
    return s.theta, s.var_plugin, s.var_unbiased


def _tv_arrays(o: Option, u_t, p_t):
    if len(u_t) != o.N or len(p_t) != o.N:
        raise ValueError("u_t and p_t need one entry per step")
    return (ctypes.c_double * o.N)(*u_t), (ctypes.c_double * o.N)(*p_t)


def price_tv_naive(o: Option, u_t, p_t) -> float:
    """Eq. (f13) with per-step u_t, p_t (index t-1 = step t), one path at a
    time (discounted; o.u and o.p are ignored)."""
    c = o._c()
    u, p = _tv_arrays(o, u_t, p_t)
    return _L().orc_price_tv_naive(ctypes.byref(c), u, p)


def price_tv(o: Option, u_t, p_t, threads: int | None = None) -> float:
    """Eq. (f13) with per-step u_t, p_t, depth-first, threads as ranks."""
    if threads is None:
        threads = max(1, min(16, os.cpu_count() or 1))
    c = o._c()
    u, p = _tv_arrays(o, u_t, p_t)
    return _L().orc_price_tv(ctypes.byref(c), u, p, threads)


def params_trinomial(sigma: float, r: float, T: float, N: int, lam: float):
    """(u, pu, pd): u = exp(lam sigma sqrt(dt)), pu and pd matching the first
    two moments of the lognormal step."""
    u, pu, pd = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    rc = _L().orc_params_trinomial(sigma, r, T, N, lam, ctypes.byref(u), ctypes.byref(pu),
                                   ctypes.byref(pd))
    if rc != 0:
        raise ValueError(f"orc_params_trinomial failed ({rc})")
    return u.value, pu.value, pd.value


def tri_digits(x: int, N: int):
    arr = (ctypes.c_int * max(N, 1))()
    _L().orc_tri_digits(x, N, arr)
    return [arr[i] for i in range(N)]


def price_tri_naive(o: Option, pd: float) -> float:
    """Eq. (f13) over the 3^N trinomial paths, one at a time (o.p = up
    probability, pd = down probability)."""
    c = o._c()
    return _L().orc_price_tri_naive(ctypes.byref(c), pd)


def price_tri(o: Option, pd: float, threads: int | None = None) -> float:
    """Eq. (f13) over the 3^N trinomial paths, depth-first, threads as ranks."""
    if threads is None:
        threads = max(1, min(16, os.cpu_count() or 1))
    c = o._c()
    return _L().orc_price_tri(ctypes.byref(c), pd, threads)


def tri_euro_backward(o: Option, pd: float) -> float:
    c = o._c()
    return _L().orc_tri_euro_backward(ctypes.byref(c), pd)
