"""Write tests/golden/instances.json: W_t and C(x*) of every benchmark instance.

Calls only the oracle (exhaustive Gray-code search, complement symmetry) and
the seeded instance generator.  n = 32..35 take minutes on a few host cores.
Run:  python tests/golden/make_golden.py          (rows already in the file are kept)
      python tests/golden/make_golden.py --all    (recompute every row)
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

CASES = [(12, 0), (26, 1), (32, 2), (33, 3), (34, 3), (30, 5), (16, 0), (20, 0), (35, 3)]
PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "instances.json")


def main():
    keep = {}
    if "--all" not in sys.argv and os.path.exists(PATH):
        keep = {(r["n"], r["seed"]): r for r in json.load(open(PATH))["instances"]}
    rows = []
    for n, seed in CASES:
        if (n, seed) in keep:
            rows.append(keep[(n, seed)])
            continue
        w = workloads.complete_graph_tenths(n, seed)
        t = time.time()
        cmax = oracle.cmax_gray(n, w)
        rows.append({"n": n, "seed": seed, "w_total_tenths": oracle.weight_total(w),
                     "cmax_tenths": cmax})
        print(n, seed, cmax, f"{time.time() - t:.1f}s", flush=True)
    out = {"_generator": "tests/golden/make_golden.py (oracle.cmax_gray, workloads.complete_graph_tenths)",
           "instances": rows}
    with open(PATH, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
