"""Write tests/golden/oracle_values.json: reference values that take the
oracle tens of seconds, computed once.  Calls only the oracle and the seeded
workload recipes (no GPU library).  Run from the repository root:
    python tests/golden/make_oracle_values.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1701_03512_amd import workloads  # noqa: E402


def opt(spec):
    return oracle.make_option(spec["S"], spec["K"], spec["sigma"], spec["r"], spec["T"],
                              spec["N"], spec["payoff"], spec["scheme"])


def main():
    oracle.build(force=False)
    out = {"note": "written by tests/golden/make_oracle_values.py from the CPU oracle only",
           "exact": [], "lookback_dp": []}
    t0 = time.time()
    for spec in [workloads.exact_small()] + workloads.exact_n32():
        v = oracle.price_dfs(opt(spec), threads=os.cpu_count())
        out["exact"].append({"spec": spec, "value": v})
        print(spec["N"], spec["payoff"], repr(v), f"{time.time() - t0:.1f}s", flush=True)
    out["exact_tv"] = []
    for spec in workloads.exact_tv_n32():
        steps = [oracle.params(s, spec["r"], spec["T"], spec["N"], spec["scheme"])
                 for s in spec["sigma_t"]]
        o = opt(spec)
        v = oracle.price_tv(o, [u for u, _ in steps], [p for _, p in steps],
                            threads=os.cpu_count())
        out["exact_tv"].append({"spec": spec, "value": v})
        print("tv", spec["N"], spec["payoff"], repr(v), f"{time.time() - t0:.1f}s", flush=True)
    out["exact_tri"] = []
    for spec in workloads.exact_tri_n20():
        u, pu, pd = oracle.params_trinomial(spec["sigma"], spec["r"], spec["T"], spec["N"], spec["lam"])
        o = oracle.Option(spec["S"], u, pu, spec["r"], spec["T"], spec["K"], spec["N"], spec["payoff"])
        v = oracle.price_tri(o, pd, threads=os.cpu_count())
        out["exact_tri"].append({"spec": spec, "value": v})
        print("tri", spec["N"], spec["payoff"], repr(v), f"{time.time() - t0:.1f}s", flush=True)
    mc = workloads.stratified_mc()
    for spec in mc["options"]:
        if spec["payoff"] == "lookback_float":
            v, m2 = oracle.lookback_dp(opt(spec))
            out["lookback_dp"].append({"spec": spec, "value": v, "second_moment": m2})
            print("dp", spec["N"], repr(v), repr(m2))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
