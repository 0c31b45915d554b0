"""ctypes binding of libbt (``include/bt.h``): argument marshalling only.

Every step of the computation runs in the library's HIP kernels.  The names
follow the C ABI.  Streams are passed as raw ``hipStream_t`` handles (e.g.
``torch.cuda.current_stream().cuda_stream``); 0 / None is the default stream.
The library is loaded on first use; if it has not been built, or a call
fails, an exception is raised -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
# PAPER_1701_03512_AMD_LIB may name another build of the same library (for
# example a launch-shape experiment); by default the in-tree build is used.
LIB_PATH = os.environ.get("PAPER_1701_03512_AMD_LIB") or os.path.join(_HERE, "libbt.so")

BT_OK, BT_EINVAL, BT_ERANGE, BT_ENOMEM, BT_EDEVICE, BT_EAGAIN, BT_ENOTFOUND, BT_ESHUTDOWN = (
    0, -1, -2, -3, -4, -5, -6, -7)

PAYOFF = {"asian_call": 0, "asian_put": 1, "lookback_float": 2,
          "lookback_fixed_put": 3, "euro_call": 4, "euro_put": 5}
# "fp32" is the Monte Carlo name of the FP32 form (no Kahan sums there)
PRECISION = {"fp64": 0, "fp32_kahan": 1, "fp32": 1}
ESTIMATOR = {"partitioned": 0, "proportional": 1, "shared_sample": 2}
SCHEME = {"crr": 0, "seydel": 1}


class BtError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib().bt_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} ({code})")


class bt_option(ctypes.Structure):
    _fields_ = [("S", ctypes.c_double), ("u", ctypes.c_double), ("p", ctypes.c_double),
                ("r", ctypes.c_double), ("T", ctypes.c_double), ("K", ctypes.c_double),
                ("N", ctypes.c_int32), ("payoff", ctypes.c_int32)]


class bt_result(ctypes.Structure):
    _fields_ = [("value", ctypes.c_double), ("err_bound", ctypes.c_double),
                ("std_err", ctypes.c_double), ("var_est", ctypes.c_double),
                ("var_unbiased", ctypes.c_double), ("var_plain", ctypes.c_double),
                ("paths", ctypes.c_uint64), ("split", ctypes.c_int32),
                ("status", ctypes.c_int32)]


class bt_tuning(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("grid", ctypes.c_int32)]


class bt_server_config(ctypes.Structure):
    _fields_ = [("mem_budget", ctypes.c_size_t), ("max_inflight", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("exact_max_n", ctypes.c_int32), ("mc_target_rel_se", ctypes.c_double),
                ("mc_max_paths", ctypes.c_uint64), ("mc_seed", ctypes.c_uint64)]


class bt_times(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_int64), ("t_admit", ctypes.c_int64),
                ("t_done", ctypes.c_int64)]


# Every exported symbol of include/bt.h: name -> (restype, argtypes).
_P = ctypes.POINTER
_vp, _i32, _u32, _u64, _d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
_int = ctypes.c_int
SIGNATURES = {
    "bt_strerror": (ctypes.c_char_p, [_int]),
    "bt_init": (_int, [_int]),
    "bt_params": (_int, [_d, _d, _d, _i32, _i32, _P(_d), _P(_d)]),
    "bt_price_exact": (_int, [_P(bt_option), _i32, _P(bt_tuning), _P(bt_result), _vp]),
    "bt_price_exact_tv": (_int, [_P(bt_option), _P(ctypes.c_double), _P(ctypes.c_double), _i32,
                                 _P(bt_tuning), _P(bt_result), _vp]),
    "bt_plan_create_tv": (_int, [_P(bt_option), _i32, _P(ctypes.c_double), _P(ctypes.c_double),
                                 _i32, _P(bt_tuning), _P(ctypes.c_void_p)]),
    "bt_price_exact_trinomial": (_int, [_P(bt_option), ctypes.c_double, _i32, _P(bt_tuning),
                                        _P(bt_result), _vp]),
    "bt_plan_create_trinomial": (_int, [_P(bt_option), _i32, ctypes.c_double, _i32,
                                        _P(bt_tuning), _P(ctypes.c_void_p)]),
    "bt_params_trinomial": (_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double, _i32,
                                   ctypes.c_double, _P(ctypes.c_double), _P(ctypes.c_double),
                                   _P(ctypes.c_double)]),
    "bt_price_batch": (_int, [_P(bt_option), _i32, _i32, _P(bt_tuning), _P(bt_result), _vp]),
    "bt_price_batch_noalloc": (_int, [_P(bt_option), _i32, _i32, _P(bt_tuning), _P(bt_result),
                                      _vp]),
    "bt_plan_bytes": (_int, [_P(bt_option), _i32, _i32, _P(bt_tuning), _P(ctypes.c_size_t)]),
    "bt_price_batch_ws": (_int, [_P(bt_option), _i32, _i32, _P(bt_tuning), _P(bt_result), _vp,
                                 ctypes.c_size_t, _vp]),
    "bt_price_exact_ws": (_int, [_P(bt_option), _i32, _P(bt_tuning), _P(bt_result), _vp,
                                 ctypes.c_size_t, _vp]),
    "bt_plan_create": (_int, [_P(bt_option), _i32, _i32, _P(bt_tuning), _P(_vp)]),
    "bt_plan_tables": (_int, [_vp, _vp]),
    "bt_plan_enumerate": (_int, [_vp, _vp]),
    "bt_plan_reduce": (_int, [_vp, _vp]),
    "bt_plan_results": (_int, [_vp, _P(bt_result), _vp]),
    "bt_plan_device_values": (_int, [_vp, _P(_vp)]),
    "bt_plan_capture": (_int, [_vp, _vp]),
    "bt_plan_launch_graph": (_int, [_vp, _vp]),
    "bt_plan_info": (_int, [_vp, _P(_u64), _P(bt_tuning)]),
    "bt_plan_destroy": (_int, [_vp]),
    "bt_plan_debug_tables": (_int, [_vp, _i32, _P(_u64), _P(_i32), _P(_i32), _vp]),
    "bt_price_stratified": (_int, [_P(bt_option), _i32, _i32, _u64, _u32, _i32, _P(bt_result), _vp]),
    "bt_enqueue_stratified": (_int, [_P(bt_option), _i32, _i32, _u64, _u32, _i32, _vp, _vp]),
    "bt_price_mc": (_int, [_P(bt_option), _i32, _i32, _u64, _u64, _u32, _i32, _P(bt_result), _vp]),
    "bt_mc_debug_bits": (_int, [_u64, _u32, _u32, _u32, _i32, _d, _P(_i32), _vp]),
    "bt_autotune": (_int, [_i32, _i32, _i32, _vp]),
    "bt_autotune_batch": (_int, [_P(bt_option), _i32, _i32, _vp]),
    "bt_tuning_for": (_int, [_i32, _i32, _P(bt_tuning)]),
    "bt_server_create": (_int, [_P(bt_server_config), _P(_vp)]),
    "bt_server_submit": (_int, [_vp, _P(bt_option), _P(_u64)]),
    "bt_server_poll": (_int, [_vp, _u64, _P(bt_result), _P(bt_times)]),
    "bt_server_stats": (_int, [_vp, _P(_u64), _P(_u64), _P(_u64), _P(_u64)]),
    "bt_server_destroy": (None, [_vp]),
}

_lib = None


def lib():
    """Load libbt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: torch loads its own copy of the HIP
        # runtime under the same soname; loading torch first makes libbt bind
        # to that copy instead of a second one from /opt/rocm.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1701_03512_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc, where):
    if rc != BT_OK:
        raise BtError(rc, where)


def _stream(s):
    if s is None:
        return None
    if hasattr(s, "cuda_stream"):
        return ctypes.c_void_p(s.cuda_stream)
    return ctypes.c_void_p(int(s))


@dataclass(frozen=True)
class Option:
    S: float
    u: float
    p: float
    r: float
    T: float
    K: float
    N: int
    payoff: str

    def c(self) -> bt_option:
        return bt_option(self.S, self.u, self.p, self.r, self.T, self.K, self.N,
                         PAYOFF[self.payoff])


def _tuning(t):
    if t is None:
        return None
    if isinstance(t, bt_tuning):
        return ctypes.byref(t)
    return ctypes.byref(bt_tuning(t.get("k", 0), t.get("chunk", 0), t.get("waves", 0),
                                  t.get("grid", 0)))


def result_dict(r: bt_result) -> dict:
    return {"value": r.value, "err_bound": r.err_bound, "std_err": r.std_err,
            "var_est": r.var_est, "var_unbiased": r.var_unbiased, "var_plain": r.var_plain,
            "paths": r.paths, "split": r.split, "status": r.status}


def bt_init(device: int = 0):
    _check(lib().bt_init(device), "bt_init")


def bt_params(sigma, r, T, N, scheme="crr"):
    u, p = ctypes.c_double(), ctypes.c_double()
    _check(lib().bt_params(sigma, r, T, N, SCHEME[scheme], ctypes.byref(u), ctypes.byref(p)),
           "bt_params")
    return u.value, p.value


def make_option(S, K, sigma, r, T, N, payoff, scheme="crr") -> Option:
    u, p = bt_params(sigma, r, T, N, scheme)
    return Option(S, u, p, r, T, K, N, payoff)


def bt_price_exact(opt: Option, precision="fp64", tune=None, stream=None) -> dict:
    res = bt_result()
    o = opt.c()
    _check(lib().bt_price_exact(ctypes.byref(o), PRECISION[precision], _tuning(tune),
                                ctypes.byref(res), _stream(stream)), "bt_price_exact")
    return result_dict(res)


def bt_price_exact_tv(opt: Option, u_t, p_t, precision="fp64", tune=None, stream=None) -> dict:
    """Exact value with per-step up factors u_t and probabilities p_t (one
    entry per step; opt.u and opt.p are ignored)."""
    if len(u_t) != opt.N or len(p_t) != opt.N:
        raise ValueError("u_t and p_t need one entry per step")
    res = bt_result()
    o = opt.c()
    u = (ctypes.c_double * opt.N)(*u_t)
    p = (ctypes.c_double * opt.N)(*p_t)
    _check(lib().bt_price_exact_tv(ctypes.byref(o), u, p, PRECISION[precision], _tuning(tune),
                                   ctypes.byref(res), _stream(stream)), "bt_price_exact_tv")
    return result_dict(res)


def bt_params_trinomial(sigma, r, T, N, lam):
    """(u, p_up, p_down) of Boyle's trinomial step with stretch lam."""
    u, pu, pd = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().bt_params_trinomial(sigma, r, T, N, lam, ctypes.byref(u), ctypes.byref(pu),
                                     ctypes.byref(pd)), "bt_params_trinomial")
    return u.value, pu.value, pd.value


def bt_price_exact_trinomial(opt: Option, p_down, precision="fp64", tune=None, stream=None) -> dict:
    """Exact value over the 3^N paths of a trinomial tree (opt.u up factor,
    opt.p up probability, p_down down probability)."""
    res = bt_result()
    o = opt.c()
    _check(lib().bt_price_exact_trinomial(ctypes.byref(o), p_down, PRECISION[precision],
                                          _tuning(tune), ctypes.byref(res), _stream(stream)),
           "bt_price_exact_trinomial")
    return result_dict(res)


def bt_price_batch(opts, precision="fp64", tune=None, stream=None):
    n = len(opts)
    arr = (bt_option * n)(*[o.c() for o in opts])
    outs = (bt_result * n)()
    _check(lib().bt_price_batch(arr, n, PRECISION[precision], _tuning(tune), outs,
                                _stream(stream)), "bt_price_batch")
    return [result_dict(outs[i]) for i in range(n)]


def bt_price_batch_noalloc(opts, precision="fp64", tune=None, stream=None):
    """bt_price_batch in the library's fixed per-device array (no device
    allocation); raises BtError(BT_ENOMEM) if the plan exceeds it."""
    n = len(opts)
    arr = (bt_option * n)(*[o.c() for o in opts])
    outs = (bt_result * n)()
    _check(lib().bt_price_batch_noalloc(arr, n, PRECISION[precision], _tuning(tune), outs,
                                        _stream(stream)), "bt_price_batch_noalloc")
    return [result_dict(outs[i]) for i in range(n)]


def bt_plan_bytes(opts, precision="fp64", tune=None) -> int:
    """Device bytes the plan of bt_price_batch(opts, precision, tune) needs."""
    n = len(opts)
    arr = (bt_option * n)(*[o.c() for o in opts])
    b = ctypes.c_size_t()
    _check(lib().bt_plan_bytes(arr, n, PRECISION[precision], _tuning(tune), ctypes.byref(b)),
           "bt_plan_bytes")
    return b.value


def bt_price_batch_ws(opts, workspace, precision="fp64", tune=None, stream=None):
    """bt_price_batch in caller-owned device memory: `workspace` is a CUDA
    tensor (any dtype, contiguous) of at least bt_plan_bytes bytes; its
    storage is passed as the device pointer."""
    n = len(opts)
    arr = (bt_option * n)(*[o.c() for o in opts])
    outs = (bt_result * n)()
    ptr, nbytes = _workspace(workspace)
    _check(lib().bt_price_batch_ws(arr, n, PRECISION[precision], _tuning(tune), outs, ptr,
                                   nbytes, _stream(stream)), "bt_price_batch_ws")
    return [result_dict(outs[i]) for i in range(n)]


def bt_price_exact_ws(opt: Option, workspace, precision="fp64", tune=None, stream=None) -> dict:
    res = bt_result()
    o = opt.c()
    ptr, nbytes = _workspace(workspace)
    _check(lib().bt_price_exact_ws(ctypes.byref(o), PRECISION[precision], _tuning(tune),
                                   ctypes.byref(res), ptr, nbytes, _stream(stream)),
           "bt_price_exact_ws")
    return result_dict(res)


def _workspace(t):
    if not t.is_contiguous():
        raise ValueError("workspace tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr()), t.numel() * t.element_size()


def bt_price_stratified(opt: Option, prefix_steps, samples_per_stratum, seed, stream_id=0,
                        precision="fp64", stream=None) -> dict:
    res = bt_result()
    o = opt.c()
    _check(lib().bt_price_stratified(ctypes.byref(o), prefix_steps, samples_per_stratum, seed,
                                     stream_id, PRECISION[precision], ctypes.byref(res),
                                     _stream(stream)), "bt_price_stratified")
    return result_dict(res)


def bt_price_mc(opt: Option, estimator, prefix_steps, samples, seed, stream_id=0,
                precision="fp64", stream=None) -> dict:
    res = bt_result()
    o = opt.c()
    _check(lib().bt_price_mc(ctypes.byref(o), ESTIMATOR[estimator], prefix_steps, samples, seed,
                             stream_id, PRECISION[precision], ctypes.byref(res), _stream(stream)),
           "bt_price_mc")
    return result_dict(res)


def bt_enqueue_stratified(opt: Option, prefix_steps, samples_per_stratum, seed, stream_id,
                          precision, d_out_ptr, stream=None):
    o = opt.c()
    _check(lib().bt_enqueue_stratified(ctypes.byref(o), prefix_steps, samples_per_stratum,
                                       seed, stream_id, PRECISION[precision],
                                       ctypes.c_void_p(d_out_ptr), _stream(stream)),
           "bt_enqueue_stratified")


def bt_mc_debug_bits(seed, stream_id, z, m, L, p, stream=None):
    bits = (ctypes.c_int32 * L)()
    _check(lib().bt_mc_debug_bits(seed, stream_id, z, m, L, p, bits, _stream(stream)),
           "bt_mc_debug_bits")
    return [bits[i] for i in range(L)]


def bt_autotune(n_lo, n_hi, precision="fp64", stream=None):
    _check(lib().bt_autotune(n_lo, n_hi, PRECISION[precision], _stream(stream)), "bt_autotune")


def bt_autotune_batch(opts, precision="fp64", stream=None):
    n = len(opts)
    arr = (bt_option * n)(*[o.c() for o in opts])
    _check(lib().bt_autotune_batch(arr, n, PRECISION[precision], _stream(stream)),
           "bt_autotune_batch")


def bt_tuning_for(N, precision="fp64") -> dict:
    t = bt_tuning()
    _check(lib().bt_tuning_for(N, PRECISION[precision], ctypes.byref(t)), "bt_tuning_for")
    return {"k": t.k, "chunk": t.chunk, "waves": t.waves, "grid": t.grid}


class Plan:
    """bt_plan_*: the exact computation of a set of options, stage by stage."""

    def __init__(self, opts, precision="fp64", tune=None, u_t=None, p_t=None, p_down=None):
        """u_t, p_t (one entry per step): options of one depth N sharing the
        time-varying moves (bt_plan_create_tv); p_down: trinomial options
        sharing the down probability (bt_plan_create_trinomial)."""
        self.n = len(opts)
        h = ctypes.c_void_p()
        arr = (bt_option * self.n)(*[o.c() for o in opts])
        if p_down is not None:
            _check(lib().bt_plan_create_trinomial(arr, self.n, p_down, PRECISION[precision],
                                                  _tuning(tune), ctypes.byref(h)),
                   "bt_plan_create_trinomial")
        elif u_t is not None or p_t is not None:
            if len(u_t) != opts[0].N or len(p_t) != opts[0].N:
                raise ValueError("a time-varying plan takes N steps of u_t and p_t")
            u = (ctypes.c_double * opts[0].N)(*u_t)
            p = (ctypes.c_double * opts[0].N)(*p_t)
            _check(lib().bt_plan_create_tv(arr, self.n, u, p, PRECISION[precision],
                                           _tuning(tune), ctypes.byref(h)), "bt_plan_create_tv")
        else:
            _check(lib().bt_plan_create(arr, self.n, PRECISION[precision], _tuning(tune),
                                        ctypes.byref(h)), "bt_plan_create")
        self.h = h

    def tables(self, stream=None):
        _check(lib().bt_plan_tables(self.h, _stream(stream)), "bt_plan_tables")

    def enumerate(self, stream=None):
        _check(lib().bt_plan_enumerate(self.h, _stream(stream)), "bt_plan_enumerate")

    def reduce(self, stream=None):
        _check(lib().bt_plan_reduce(self.h, _stream(stream)), "bt_plan_reduce")

    def results(self, stream=None):
        outs = (bt_result * self.n)()
        _check(lib().bt_plan_results(self.h, outs, _stream(stream)), "bt_plan_results")
        return [result_dict(outs[i]) for i in range(self.n)]

    def device_values(self) -> int:
        p = ctypes.c_void_p()
        _check(lib().bt_plan_device_values(self.h, ctypes.byref(p)), "bt_plan_device_values")
        return p.value

    def capture(self, stream):
        _check(lib().bt_plan_capture(self.h, _stream(stream)), "bt_plan_capture")

    def launch_graph(self, stream):
        _check(lib().bt_plan_launch_graph(self.h, _stream(stream)), "bt_plan_launch_graph")

    def info(self):
        items = ctypes.c_uint64()
        t = bt_tuning()
        _check(lib().bt_plan_info(self.h, ctypes.byref(items), ctypes.byref(t)), "bt_plan_info")
        return {"items": items.value, "k": t.k, "chunk": t.chunk, "waves": t.waves,
                "grid": t.grid}

    def debug_tables(self, i, P, k, stream=None):
        nz, ns = 1 << P, 1 << k
        z = (ctypes.c_uint64 * nz)()
        a = (ctypes.c_int32 * nz)()
        b = (ctypes.c_int32 * ns)()
        _check(lib().bt_plan_debug_tables(self.h, i, z, a, b, _stream(stream)),
               "bt_plan_debug_tables")
        return list(z), list(a), list(b)

    def close(self):
        if self.h:
            lib().bt_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """bt_server_*: continuous-batching pricing loop."""

    def __init__(self, mem_budget=8 << 30, max_inflight=256, streams=4, precision="fp64",
                 exact_max_n=34, mc_target_rel_se=1e-4, mc_max_paths=1 << 24,
                 mc_seed=0x5EED):
        cfg = bt_server_config(mem_budget, max_inflight, streams, PRECISION[precision],
                               exact_max_n, mc_target_rel_se, mc_max_paths, mc_seed)
        h = ctypes.c_void_p()
        _check(lib().bt_server_create(ctypes.byref(cfg), ctypes.byref(h)), "bt_server_create")
        self.h = h

    def submit(self, opt: Option) -> int:
        t = ctypes.c_uint64()
        o = opt.c()
        _check(lib().bt_server_submit(self.h, ctypes.byref(o), ctypes.byref(t)),
               "bt_server_submit")
        return t.value

    def poll(self, ticket):
        """None while pending; (result dict, (t_submit, t_admit, t_done)) when done."""
        res, tm = bt_result(), bt_times()
        rc = lib().bt_server_poll(self.h, ticket, ctypes.byref(res), ctypes.byref(tm))
        if rc == BT_EAGAIN:
            return None
        _check(rc, "bt_server_poll")
        return result_dict(res), (tm.t_submit, tm.t_admit, tm.t_done)

    def stats(self):
        v = [ctypes.c_uint64() for _ in range(4)]
        _check(lib().bt_server_stats(self.h, *[ctypes.byref(x) for x in v]), "bt_server_stats")
        return {"submitted": v[0].value, "admitted": v[1].value, "completed": v[2].value,
                "peak_bytes": v[3].value}

    def close(self):
        if self.h:
            lib().bt_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
