"""Writes c5_oracle_128.npz: the FP64 oracle's outputs on the first two 128x128
requests of the served workload's stream (instance 0 of the request generator;
one Gaussian-mixture and one white-noise pair; eta = 1e-3, K = 10), the
largest size of the request mix (m = n = 16384).  Each solve takes the plain
oracle about an hour on one core and about 5 GB of memory (the
dense 16384 x 16384 cost), so the two run in two processes.  Stored per
request: its index in the stream, side, cost and potentials.  Only oracle/ and
the seeded input generators are called.
Run: python tests/golden/make_c5_large_fixtures.py
"""
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

ETA, K, STREAM, SIDE = 1e-3, 10, 2000, 128
OUT = os.path.join(HERE, "c5_oracle_128.npz")


def sample():
    import workloads as W

    reqs = W.serve_requests(STREAM, 1.0)
    return [(q, reqs[q]) for q, r in enumerate(reqs) if r["s"] == SIDE][:2]


def one(item):
    import oracle

    q, r = item
    t0 = time.time()
    o = oracle.pins(oracle.cost_grid(r["s"]), r["a"], r["b"], want_plan=False, eta=ETA, K=K)
    assert o["status"] == 0, q
    return q, r["s"], o, time.time() - t0


def main():
    import oracle

    oracle.build()
    items = sample()
    out = dict(eta=ETA, K=K, stream=STREAM)
    idx, sides, costs = [], [], []
    with ProcessPoolExecutor(max_workers=2) as ex:
        for q, s, o, dt in ex.map(one, items):
            idx.append(q)
            sides.append(s)
            costs.append(o["cost"])
            out["alpha_%d" % q] = o["alpha"]
            out["beta_%d" % q] = o["beta"]
            print(q, s, "cost %.17g newton %d cg %d sinkhorn %d  %.0f s" % (o["cost"], o["newton"], o["cg"],
                                                                            o["sinkhorn"], dt), flush=True)
    out["index"] = np.array(idx)
    out["side"] = np.array(sides)
    out["cost"] = np.array(costs)
    np.savez_compressed(OUT, **out)


if __name__ == "__main__":
    main()
