"""Writes c2_lp.json: the transport LP optimum (scipy's HiGHS through
oracle/lp.py) of pairs 0..3 of the 28x28 image-histogram family (squared grid
distance / (2*27^2)), the reference for the cost error of the 64-pair
configuration at a given number of outer iterations.  Only oracle/ and the
seeded input generators are called; each LP takes about a minute, so the pairs
run in parallel processes.
Run: python tests/golden/make_c2_lp.py
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

S, PAIRS = 28, 4
OUT = os.path.join(HERE, "c2_lp.json")


def one(i):
    import oracle
    from oracle import lp
    import workloads as W

    pr = W.blob_pair(i, s=S)
    ot, _ = lp.lp_highs(oracle.cost_grid(S), pr["a"], pr["b"])
    return i, ot


def main():
    import oracle

    oracle.build()
    out = dict(s=S, what="LP optimum by HiGHS (oracle/lp.py), cost normalised by 2 (s-1)^2", lp={})
    with ProcessPoolExecutor(max_workers=PAIRS) as ex:
        for i, ot in ex.map(one, range(PAIRS)):
            out["lp"][str(i)] = ot
            print("pair %d LP %.17g" % (i, ot), flush=True)
    json.dump(out, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main()
