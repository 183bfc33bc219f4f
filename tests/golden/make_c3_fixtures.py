"""Writes c3_oracle.npz: the FP64 oracle's outputs on the 64 x 64 grid
configuration (m = n = 4096, squared grid distance / (2*63^2), eta = 1e-3,
K = 10), one pair per histogram class (white noise, 5-component Gaussian
mixture, Cauchy bumps; pair 0 of each).

Stored per class: cost <C, X^K>, marginal residual, gauge-fixed potentials
alpha and beta (4096 each), and the oracle's iteration counts.  Only oracle/
and the seeded input generators are called; each class takes a few minutes
single-threaded, so the classes run in parallel processes.
Run: python tests/golden/make_c3_fixtures.py
"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

S, ETA, K = 64, 1e-3, 10
CLASSES = ("white", "gmm", "cauchy")
OUT = os.path.join(HERE, "c3_oracle.npz")


def one(cls):
    import oracle
    import workloads as W

    pr = W.grid_pair(cls, 0, s=S)
    C = oracle.cost_grid(S)
    r = oracle.pins(C, pr["a"], pr["b"], eta=ETA, K=K, want_plan=False)
    assert r["status"] == 0, (cls, r["status"])
    return cls, r


def main():
    import oracle

    oracle.build()
    out = dict(s=S, eta=ETA, K=K)
    with ProcessPoolExecutor(max_workers=len(CLASSES)) as ex:
        for cls, r in ex.map(one, CLASSES):
            out[cls + "_alpha"] = r["alpha"]
            out[cls + "_beta"] = r["beta"]
            out[cls + "_scalars"] = np.array([r["cost"], r["resid"], r["dual"], r["entropy"]])
            out[cls + "_counts"] = np.array([r["sinkhorn"], r["newton"], r["cg"], r["fallbacks"], r["flags"]])
            print(cls, "cost %.17g resid %.3g newton %d cg %d fallbacks %d" % (r["cost"], r["resid"], r["newton"],
                                                                              r["cg"], r["fallbacks"]), flush=True)
    np.savez_compressed(OUT, **out)


if __name__ == "__main__":
    main()
