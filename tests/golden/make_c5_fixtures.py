"""Writes c5_oracle.npz: the FP64 oracle's outputs on sampled requests of the
served workload (Poisson stream of grid requests, instance 0 of the request
generator: 60% 32x32, 30% 64x64, 10% 128x128 grids, Gaussian-mixture or
white-noise histograms; eta = 1e-3, K = 10): the first six 32x32 requests and
the first two 64x64 requests of the stream (128x128 requests are beyond the
oracle's reach in minutes).  Stored per request: its index in the stream, side,
cost and potentials.  The request problems do not depend on the arrival rate.
Only oracle/ and the seeded input generators are called.
Run: python tests/golden/make_c5_fixtures.py
"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

ETA, K, STREAM = 1e-3, 10, 2000
OUT = os.path.join(HERE, "c5_oracle.npz")


def sample():
    import workloads as W

    reqs = W.serve_requests(STREAM, 1.0)
    s32 = [q for q, r in enumerate(reqs) if r["s"] == 32][:6]
    s64 = [q for q, r in enumerate(reqs) if r["s"] == 64][:2]
    return [(q, reqs[q]) for q in s32 + s64]


def one(item):
    import oracle

    q, r = item
    o = oracle.pins(oracle.cost_grid(r["s"]), r["a"], r["b"], want_plan=False, eta=ETA, K=K)
    assert o["status"] == 0, q
    return q, r["s"], o


def main():
    import oracle

    oracle.build()
    items = sample()
    out = dict(eta=ETA, K=K, stream=STREAM)
    idx, sides, costs = [], [], []
    with ProcessPoolExecutor(max_workers=4) as ex:
        for q, s, o in ex.map(one, items):
            idx.append(q)
            sides.append(s)
            costs.append(o["cost"])
            out["alpha_%d" % q] = o["alpha"]
            out["beta_%d" % q] = o["beta"]
            print(q, s, "cost %.17g newton %d" % (o["cost"], o["newton"]), flush=True)
    out["index"] = np.array(idx)
    out["side"] = np.array(sides)
    out["cost"] = np.array(costs)
    np.savez_compressed(OUT, **out)


if __name__ == "__main__":
    main()
