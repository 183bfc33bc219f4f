"""Writes c2_oracle.npz: the FP64 oracle's outputs on pairs 0..15 of the
image-histogram family (28x28 grids, m = n = 784, squared grid distance
normalised by its maximum, eta = 0.1, K = 250): cost and potentials per pair.
Only oracle/ and the seeded input generators are called.
Run: python tests/golden/make_c2_fixtures.py
"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

S, ETA, K, PAIRS = 28, 0.1, 250, 16
OUT = os.path.join(HERE, "c2_oracle.npz")


def one(q):
    import oracle
    import workloads as W

    p = W.blob_pair(q, s=S)
    o = oracle.pins(oracle.cost_grid(S), p["a"], p["b"], want_plan=False, eta=ETA, K=K)
    assert o["status"] == 0, q
    return q, o


def main():
    import oracle

    oracle.build()
    out = dict(s=S, eta=ETA, K=K)
    costs = []
    with ProcessPoolExecutor(max_workers=4) as ex:
        for q, o in ex.map(one, range(PAIRS)):
            costs.append(o["cost"])
            out["alpha_%d" % q] = o["alpha"]
            out["beta_%d" % q] = o["beta"]
            print(q, "cost %.17g newton %d" % (o["cost"], o["newton"]), flush=True)
    out["cost"] = np.array(costs)
    np.savez_compressed(OUT, **out)


if __name__ == "__main__":
    main()
