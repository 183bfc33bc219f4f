"""Writes oracle_fixtures.json: the FP64 oracle's outputs on three small seeded
instances (a point cloud, a random assignment, an image-histogram grid).

The paper prints no worked example with reproducible numbers (its tables
summarise random instances with unpublished seeds), so the oracle is pinned by
closed forms, brute force and invariants (test_oracle_pins.py); these fixtures
freeze what the pinned oracle computes, so that a later change of its
arithmetic shows up as a changed fixture.  Only oracle/ and the seeded input
generators are called.  Run: python tests/golden/make_oracle_fixtures.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def cases():
    """(name, C, a, b, eta, K) of every fixture; shared with the test."""
    p = W.points_instance(0, m=12, n=9)
    yield "points_12x9", W.sqeuclid_dense(p["x"], p["y"]), p["a"], p["b"], 0.05, 8
    q = W.assignment_instance(0, 10)
    yield "assignment_10", q["C"], q["a"], q["b"], 1e-2, 20
    h = W.blob_pair(0, s=5)
    yield "blobs_5x5", W.grid_dense(5), h["a"], h["b"], 0.1, 30


def main():
    out = {}
    for name, C, a, b, eta, K in cases():
        r = oracle.pins(C, a, b, eta=eta, K=K, want_plan=False)
        assert r["status"] == 0, name
        out[name] = dict(eta=eta, K=K, cost=r["cost"], resid=r["resid"], alpha=list(r["alpha"]),
                         beta=list(r["beta"]))
    with open(os.path.join(HERE, "oracle_fixtures.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
