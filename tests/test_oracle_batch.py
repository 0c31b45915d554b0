"""The stored oracle values of the 4096-option batch
(tests/golden/batch4096_oracle.json): they belong to the seeded recipe, and
the oracle's naive enumerator (one path at a time, O(N) per path) gives the
same values as the depth-first enumerator that wrote them, on the shallow
options of each payoff."""
import json
import math
import os

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_stored_batch_matches_recipe_and_naive_enumeration(orc):
    from paper_1701_03512_amd import workloads
    gold = json.load(open(os.path.join(GOLD, "batch4096_oracle.json")))
    specs = workloads.random_options(4096, seed=gold["seed"])
    import hashlib
    digest = hashlib.sha256(json.dumps(specs, sort_keys=True).encode()).hexdigest()
    assert gold["specs_sha256"] == digest and gold["n"] == 4096
    assert gold["paths"] == sum(2 ** s["N"] for s in specs)
    vals = gold["values"]
    assert all(math.isfinite(v) and v >= 0.0 for v in vals)
    checked = {}
    for i, s in enumerate(specs):
        if s["N"] == 16 and checked.get(s["payoff"], 0) < 3:
            o = orc.make_option(s["S"], s["K"], s["sigma"], s["r"], s["T"], s["N"], s["payoff"])
            want = orc.price_naive(o)
            assert abs(vals[i] - want) <= 1e-13 * abs(want) + 1e-15 * s["S"], (i, vals[i], want)
            checked[s["payoff"]] = checked.get(s["payoff"], 0) + 1
    assert sorted(checked) == sorted(workloads.BENCH_PAYOFFS)
