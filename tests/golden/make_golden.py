"""Write tests/golden/config5_marginal.json: oracle (binary128) probabilities of
the large-Torontonian workload's marginal click patterns (800-mode state,
seed 50, click sets drawn by gbs_inputs.config5_pattern).  Calls only the
oracle and the input generators.  Run: python tests/golden/make_golden.py [n ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gbs_inputs as gi  # noqa: E402
import oracle  # noqa: E402


def main(ns):
    cov = gi.state_m800(50)
    out = {"source": "oracle.formS (binary128), state gbs_inputs.state_m800(50)", "cases": []}
    path = os.path.join(HERE, "config5_marginal.json")
    if os.path.exists(path):
        out = json.load(open(path))
    have = {(c["n"], c["seed"]) for c in out["cases"]}
    for n in ns:
        if (n, 50) in have:
            continue
        t = time.time()
        r = oracle.formS(cov, gi.config5_pattern(n, seed=50))
        out["cases"].append({"n": n, "seed": 50, "p_hi": r.p, "p_lo": r.p_lo, "abs_sum": r.abs_sum,
                             "cancel_ratio": r.cancel_ratio, "oracle_seconds": time.time() - t,
                             "oracle_threads": oracle.num_threads()})
        out["cases"].sort(key=lambda c: (c["seed"], c["n"]))
        json.dump(out, open(path, "w"), indent=1)
        print(n, r.p, r.cancel_ratio, time.time() - t, flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [20, 22, 24])
