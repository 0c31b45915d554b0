"""The 4096-option batch against the oracle's stored values
(tests/golden/batch4096_oracle.json, written by
tests/golden/make_oracle_values.py --batch4096 from the oracle alone)."""
import json
import os

import bounds

GOLD = os.path.join(os.path.dirname(__file__), "golden")
TOL = {"fp64": (1e-12, 1e-15), "fp32_kahan": (1e-6, 1e-9)}


def check_all(precision, opts, results, label):
    """Every one of the 4096 options against the oracle's stored value, and
    the error bound of each against its actual error (plus the oracle's own
    rounding bound); returns the options that pass only through the absolute
    floor.  The FP32 form's bound must be within the relative tolerance of
    the value on every other option (zero where the value is zero); the
    FP64 bound, which sums input rounding over all paths, is reported."""
    gold = json.load(open(os.path.join(GOLD, "batch4096_oracle.json")))
    from paper_1701_03512_amd import workloads
    specs = workloads.random_options(4096, seed=gold["seed"])
    import hashlib
    assert gold["specs_sha256"] == hashlib.sha256(
        json.dumps(specs, sort_keys=True).encode()).hexdigest()
    rel, floor = TOL[precision]
    floor_only, loose, worst = [], [], 0.0
    for i, (sp, o, r, want) in enumerate(zip(specs, opts, results, gold["values"])):
        assert r["status"] == 0 and r["paths"] == 2 ** sp["N"]
        err = abs(r["value"] - want)
        assert err <= max(rel * abs(want), floor * sp["S"]), (label, i, sp, r["value"], want)
        u, p = o.u, o.p
        ob = bounds.oracle_rounding(want, sp["S"], sp["K"], sp["r"], sp["T"], sp["N"],
                                    bounds.forward_growth(u, p, sp["N"]))
        assert err <= r["err_bound"] + ob, (label, i, sp, err, r["err_bound"], ob)
        if r["err_bound"] > rel * abs(want):
            loose.append(i)
        if err > rel * abs(want):
            floor_only.append((i, err / abs(want) if want else float("inf")))
        else:
            worst = max(worst, err / abs(want) if want else 0.0)
    print(f"{label} {precision}: 4096 options, worst rel err {worst:.3e} outside the floor; "
          f"{len(floor_only)} pass only through the floor {floor} S: {floor_only}; "
          f"{len(loose)} state a bound above {rel} of the value: {loose}", flush=True)
    if precision == "fp32_kahan":
        fo = {i for i, _ in floor_only}
        assert not [i for i in loose if i not in fo], (label, loose)
    return floor_only
