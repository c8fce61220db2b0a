"""Writes the stored expected values that are not worked by hand.

It calls only the oracle (and the seeded input generators for the inputs);
nothing here comes from the GPU path.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402


def e2():
    values = workloads.hash_values(2, 8)
    offsets = workloads.fixed_offsets(8, 4)
    r = oracle.run(oracle.HASH_EXPAND, offsets, values, emit_outputs=True)
    return {
        "name": "E-2: keep bit 0 of H(x,0) -> expand into (H(x,0)>>1)&3 children H(x,j+1) -> count/sum/min/max",
        "citation": "Sec. 2.1: each input of a node yields zero or more outputs up to a node maximum (here 1, then 3); "
                    "Sec. 4.1: per-parent aggregation. Values written by this script from the oracle.",
        "kind": 2,
        "seed": 2,
        "offsets": offsets.tolist(),
        "elements": values.tolist(),
        "expected": {"count": r.count.tolist(), "sum": [int(x) for x in r.sum],
                     "min": r.min.tolist(), "max": r.max.tolist()},
        "outputs": r.out.tolist(),
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "e2_hash_expand.json"), "w") as f:
        json.dump(e2(), f, indent=1)
        f.write("\n")
    print("wrote e2_hash_expand.json")
