"""Write tests/golden/oracle_values.json: reference values that take the
oracle tens of seconds, computed once.  Calls only the oracle and the seeded
workload recipes (no GPU library).  Run from the repository root:
    python tests/golden/make_oracle_values.py

With --shapes it adds the "shapes" entries to oracle_values.json (the N=32
market's three payoffs at N = 24, 26, 28, 30, the depths whose launch shapes
the tests sweep) and leaves the other entries as they are.

With --batch4096 it writes tests/golden/batch4096_oracle.json instead: the
oracle's depth-first enumeration (eq. (f13)) of every option of the seeded
4096-option batch (N 16..30, 5.5e11 paths; about 15 minutes on 8 host
threads), keyed by the recipe's seed.
"""
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

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


def shapes():
    """The three benchmark payoffs of the N=32 market at depths 24..30."""
    oracle.build(force=False)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")
    out = json.load(open(path))
    out["shapes"] = []
    t0 = time.time()
    for N in (24, 26, 28, 30):
        for spec in workloads.exact_n32():
            spec = dict(spec, N=N)
            v = oracle.price_dfs(opt(spec), threads=os.cpu_count())
            out["shapes"].append({"spec": spec, "value": v})
            print(N, spec["payoff"], repr(v), f"{time.time() - t0:.1f}s", flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


def specs_digest(specs):
    """SHA-256 of the parameter list as canonical JSON."""
    import hashlib
    return hashlib.sha256(json.dumps(specs, sort_keys=True).encode()).hexdigest()


def batch4096():
    """Every option of workloads.random_options(4096) by the oracle's DFS,
    one option per host thread (ctypes releases the interpreter lock)."""
    oracle.build(force=False)
    seed = workloads.DEFAULT_SEED
    specs = workloads.random_options(4096, seed=seed)
    order = sorted(range(len(specs)), key=lambda i: -specs[i]["N"])
    values = [None] * len(specs)
    t0 = time.time()
    done = [0]

    def one(i):
        values[i] = oracle.price_dfs(opt(specs[i]), 1)
        done[0] += 1
        if done[0] % 256 == 0:
            print(f"{done[0]} options, {time.time() - t0:.0f}s", flush=True)

    with ThreadPoolExecutor(max_workers=os.cpu_count()) as ex:
        list(ex.map(one, order))
    out = {"note": "written by tests/golden/make_oracle_values.py --batch4096 from the CPU "
                   "oracle only: orc_price_dfs of workloads.random_options(4096, seed); "
                   "specs_sha256 identifies the recipe's parameter list",
           "seed": seed, "n": len(specs),
           "paths": sum(2 ** s["N"] for s in specs),
           "specs_sha256": specs_digest(specs),
           "values": values}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch4096_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print("wrote", path, f"{time.time() - t0:.0f}s")


if __name__ == "__main__":
    if "--batch4096" in sys.argv[1:]:
        batch4096()
    elif "--shapes" in sys.argv[1:]:
        shapes()
    else:
        main()
