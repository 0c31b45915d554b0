"""CPU checks of the C ABI: the library loads, exports every symbol the
public header declares, and rejects bad arguments before touching a device.
No compute call is made here."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bt.h")


@pytest.fixture(scope="module")
def bt():
    from paper_1701_03512_amd import bt as m
    m.lib()
    return m


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bt_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("bt_price_exact", "bt_price_batch", "bt_price_stratified",
              "bt_server_submit", "bt_server_poll", "bt_params", "bt_strerror"):
        assert n in names


def test_every_declared_symbol_is_exported(bt):
    lib = ctypes.CDLL(bt.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol(bt):
    assert sorted(bt.SIGNATURES) == _declared()


def test_struct_sizes_match_header(bt):
    # bt_option: 6 doubles + 2 int32; bt_result: 6 doubles + u64 + 2 int32
    assert ctypes.sizeof(bt.bt_option) == 56
    assert ctypes.sizeof(bt.bt_result) == 64
    assert bt.bt_result.err_bound.offset == 8 and bt.bt_result.var_plain.offset == 40
    assert ctypes.sizeof(bt.bt_tuning) == 16


def test_params_match_oracle_bitwise(bt, orc):
    for scheme in ("crr", "seydel"):
        for (sig, r, T, N) in [(0.2, 0.05, 1.0, 32), (3.0, 0.06, 1.0, 32), (0.45, 0.0, 2.0, 17)]:
            assert bt.bt_params(sig, r, T, N, scheme) == orc.params(sig, r, T, N, scheme)


def test_params_errors(bt):
    with pytest.raises(bt.BtError) as e:
        bt.bt_params(-0.1, 0.05, 1.0, 10)
    assert e.value.code == bt.BT_EINVAL
    with pytest.raises(bt.BtError):
        bt.bt_params(0.01, 0.5, 1.0, 2)  # p > 1


def test_strerror(bt):
    assert bt.lib().bt_strerror(bt.BT_ERANGE) == b"size out of supported range"


@pytest.mark.parametrize("field,value,code", [
    ("S", -1.0, -1), ("u", 0.9, -1), ("p", 1.0, -1), ("T", 0.0, -1), ("K", -2.0, -1),
    ("N", 0, -1), ("N", 41, -2), ("payoff", "bad", -1)])
def test_exact_argument_checks_before_device(bt, field, value, code):
    base = dict(S=100.0, u=1.05, p=0.5, r=0.0, T=1.0, K=100.0, N=10, payoff=0)
    base[field] = 7 if value == "bad" else value
    o = bt.bt_option(**base)
    res = bt.bt_result()
    rc = bt.lib().bt_price_exact(ctypes.byref(o), 0, None, ctypes.byref(res), None)
    assert rc == code


def test_stratified_argument_checks_before_device(bt):
    o = bt.bt_option(100.0, 1.05, 0.5, 0.0, 1.0, 100.0, 20, 0)
    res = bt.bt_result()
    L = bt.lib()
    assert L.bt_price_stratified(ctypes.byref(o), 20, 4, 1, 0, 0, ctypes.byref(res), None) == bt.BT_EINVAL
    assert L.bt_price_stratified(ctypes.byref(o), 5, 0, 1, 0, 0, ctypes.byref(res), None) == bt.BT_EINVAL
    o.N = 65
    assert L.bt_price_stratified(ctypes.byref(o), 5, 4, 1, 0, 0, ctypes.byref(res), None) == bt.BT_ERANGE


def test_mc_estimator_argument_checks_before_device(bt):
    o = bt.bt_option(100.0, 1.05, 0.5, 0.0, 1.0, 100.0, 30, 0)
    res = bt.bt_result()
    L = bt.lib()
    call = lambda est, r, R, prec=0: L.bt_price_mc(ctypes.byref(o), est, r, R, 1, 0, prec,
                                                    ctypes.byref(res), None)
    assert call(7, 5, 16) == bt.BT_EINVAL                      # unknown estimator
    assert call(2, 5, 0) == bt.BT_EINVAL                       # no samples
    assert call(2, 5, 16, prec=3) == bt.BT_EINVAL              # unknown precision
    assert call(1, 30, 16) == bt.BT_EINVAL                     # r = N
    assert call(1, 5, (1 << 30) + 1) == bt.BT_ERANGE           # R > 2^30
    assert call(2, 27, 16) == bt.BT_ERANGE                     # 2^27 prefixes
    assert call(2, 20, 1 << 20) == bt.BT_ERANGE                # chunks x draws > 2^27
    assert call(0, 5, 1 << 31) == bt.BT_ERANGE                 # per-stratum count


def test_time_varying_argument_checks_before_device(bt):
    L = bt.lib()
    res = bt.bt_result()

    def call(N, u, p, prec=0):
        o = bt.bt_option(100.0, 1.05, 0.5, 0.0, 1.0, 100.0, N, 0)
        U = (ctypes.c_double * len(u))(*u)
        P = (ctypes.c_double * len(p))(*p)
        return L.bt_price_exact_tv(ctypes.byref(o), U, P, prec, None, ctypes.byref(res), None)

    assert call(3, [1.1, 1.0, 1.1], [0.5] * 3) == bt.BT_EINVAL         # u_t <= 1
    assert call(3, [1.1, float("inf"), 1.1], [0.5] * 3) == bt.BT_EINVAL
    assert call(3, [1.1] * 3, [0.5, 0.0, 0.5]) == bt.BT_EINVAL         # p_t outside (0, 1)
    assert call(41, [1.1] * 41, [0.5] * 41) == bt.BT_ERANGE            # N > 40
    assert call(40, [1.05] * 40, [0.001] * 40, prec=1) == bt.BT_ERANGE  # FP32 weight spread


def test_trinomial_params_match_oracle(bt, orc):
    for s, r, T, N, lam in [(0.2, 0.05, 1.0, 20, 1.224744871391589), (0.3, 0.03, 2.0, 10, 1.5)]:
        got = bt.bt_params_trinomial(s, r, T, N, lam)
        want = orc.params_trinomial(s, r, T, N, lam)
        assert got[0] == want[0]
        for g, w in zip(got[1:], want[1:]):
            assert abs(g - w) <= 1e-13 * w
    with pytest.raises(bt.BtError):
        bt.bt_params_trinomial(0.25, 0.0, 1.0, 16, 1.0)


def test_trinomial_argument_checks_before_device(bt):
    L = bt.lib()
    res = bt.bt_result()

    def call(N, pu, pd, prec=0, k=0):
        o = bt.bt_option(100.0, 1.05, pu, 0.0, 1.0, 100.0, N, 0)
        t = bt.bt_tuning(k, 0, 0, 0)
        return L.bt_price_exact_trinomial(ctypes.byref(o), pd, prec, ctypes.byref(t),
                                          ctypes.byref(res), None)

    assert call(10, 0.4, 0.0) == bt.BT_EINVAL       # p_down must be positive
    assert call(10, 0.6, 0.5) == bt.BT_EINVAL       # p_up + p_down > 1
    assert call(27, 0.3, 0.3) == bt.BT_ERANGE       # N > 26
    assert call(26, 0.3, 0.3, k=8) == bt.BT_ERANGE  # 18 prefix digits
    assert call(20, 0.3, 0.3, k=13) == bt.BT_ERANGE  # 13 suffix digits


def test_bad_tuning_rejected(bt):
    o = bt.bt_option(100.0, 1.05, 0.5, 0.0, 1.0, 100.0, 10, 0)
    res = bt.bt_result()
    t = bt.bt_tuning(17, 0, 0, 0)
    assert bt.lib().bt_price_exact(ctypes.byref(o), 0, ctypes.byref(t), ctypes.byref(res), None) == bt.BT_EINVAL
    t = bt.bt_tuning(0, 6, 0, 0)
    assert bt.lib().bt_price_exact(ctypes.byref(o), 0, ctypes.byref(t), ctypes.byref(res), None) == bt.BT_EINVAL


def test_builtin_launch_shapes(bt):
    """The built-in (untuned) shapes, host logic only: k ~ N/2 within
    [10, 16] (all of N up to 10) and chunks of 2^P / 32 (FP64) or 2^P / 64
    (FP32) prefixes, at least 1024 and at most 2048."""
    want = {5: (5, 1024, 1024), 20: (10, 1024, 1024), 24: (12, 1024, 1024), 30: (15, 1024, 1024),
            32: (16, 2048, 1024), 40: (16, 2048, 2048)}
    for N, (k, c64, c32) in want.items():
        t64, t32 = bt.bt_tuning_for(N, "fp64"), bt.bt_tuning_for(N, "fp32_kahan")
        assert (t64["k"], t64["chunk"], t64["grid"]) == (k, c64, 0), (N, t64)
        assert (t32["k"], t32["chunk"], t32["grid"]) == (k, c32, 0), (N, t32)


@pytest.mark.parametrize("precision", [0, 1])
def test_plan_layout_verified_on_host(bt, precision):
    """Without a GPU every exact call must get past argument checks and the
    host-side layout verification (which refuses a plan whose arrays leave
    its allocation, overlap, or do not match the kernels' extents) and fail
    only at the device: BT_EDEVICE, never BT_EINVAL."""
    if os.environ.get("HIP_VISIBLE_DEVICES", None) is None:
        try:
            import torch
            if torch.cuda.is_available():
                pytest.skip("a GPU is visible")
        except ImportError:
            pass
    L = bt.lib()
    res = bt.bt_result()
    for N in (1, 2, 3, 7, 10, 11, 16, 17, 22, 32, 40):
        for k in (0, 1, 8, 16):
            for chunk in (0, 4, 256, 1024):
                o = bt.bt_option(100.0, 1.05, 0.5, 0.01, 1.0, 100.0, N, N % 6)
                t = bt.bt_tuning(k, chunk, 0, 0)
                rc = L.bt_price_exact(ctypes.byref(o), precision, ctypes.byref(t),
                                      ctypes.byref(res), None)
                kk = min(k or 16, N) if N > 10 or k else N
                too_big = N - kk > 26 or (2 ** (N - kk)) / min(chunk or 256, 2 ** (N - kk)) > 2 ** 22
                want = bt.BT_ERANGE if too_big else bt.BT_EDEVICE
                assert rc == want, (N, k, chunk, rc)
    opts = (bt.bt_option * 30)(*[bt.bt_option(100.0, 1.05, 0.5, 0.01, 1.0, 100.0, 1 + i % 24, i % 6)
                                 for i in range(30)])
    outs = (bt.bt_result * 30)()
    assert L.bt_price_batch(opts, 30, precision, None, outs, None) == bt.BT_EDEVICE


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message and a
    nonzero status before touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout.strip() == ""
