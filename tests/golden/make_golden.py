"""Write the stored expected values under tests/golden/ by calling the oracle.

Inputs come from the seeded generator; every expected value comes from
``oracle`` alone.  Run from the repository root:

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2606_24647_amd import datagen as dg  # noqa: E402


def c1():
    rows, seed, bound = 1_000_000, 1, 2466
    t = dg.fact_c1(rows, seed=seed)
    rev = [("col", 1), ("k-col", 100, 2)]
    aggs = [("sum", [("col", 0)]), ("sum", [("col", 1)]), ("sum", [("col", 2)]), ("sum", rev),
            ("count*",)]
    r = oracle.groupby(t, [4, 5], [("range", 3, -(1 << 31), bound)], aggs)
    assert not r.overflow
    groups = []
    for g in range(r.nrows):
        groups.append({"flag": int(r.keys[0][0][g]), "status": int(r.keys[1][0][g]),
                       "sum_qty": int(r.aggs[0][0][g]), "sum_price": int(r.aggs[1][0][g]),
                       "sum_disc": int(r.aggs[2][0][g]), "sum_rev": int(r.aggs[3][0][g]),
                       "count": int(r.aggs[4][0][g])})
    out = {"what": "config-1 filter (shipdate <= 2466) + group by (flag, status): "
                   "SUM(qty), SUM(price), SUM(disc), SUM(price*(100-disc)), COUNT(*)",
           "rows": rows, "seed": seed, "bound": bound, "groups": groups}
    with open(os.path.join(HERE, "c1_filter_groupby.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    c1()
