"""Serving (pins_server_*): requests from several host threads, admitted as
workers free up onto concurrent batches.  Each result must be bitwise the one
its problem gets alone, and match the oracle."""
import threading
import time

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2502_03749_amd as P  # noqa: E402


def test_served_results_equal_alone():
    print("case serving mix", flush=True)
    eta, K = 0.1, 12
    prm = P.params(eta=eta, max_outer=K)
    reqs = []
    for i in range(16):
        s = (12, 16, 20)[i % 3]
        pr = W.blob_pair(100 + i, s=s)
        reqs.append((s, pr["a"], pr["b"]))
    srv = P.Server(prm, workers=2, max_batch=6)
    tickets = [None] * len(reqs)

    def producer(lo):
        for q in range(lo, len(reqs), 2):
            s, a, b = reqs[q]
            tickets[q] = srv.submit(P.COST_GRID, a, b, grid_s=s)
            time.sleep(0.002 * (q % 4))  # arrivals spread over the first batches

    th = [threading.Thread(target=producer, args=(k,)) for k in (0, 1)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    served = [srv.wait(t) for t in tickets]
    srv.close()
    ctx = P.Context(0)
    try:
        for q, (s, a, b) in enumerate(reqs):
            r = served[q]
            assert r["rc"] == 0 and r["resid"] <= 1e-10 and r["latency_ms"] > 0.0
            alone = ctx.solve(P.COST_GRID, a, b, prm, grid_s=s)
            assert np.array_equal(alone["alpha"], r["alpha"]) and np.array_equal(alone["beta"], r["beta"]), q
            assert alone["cost"] == r["cost"]
        for q in (0, 7):
            s, a, b = reqs[q]
            o = oracle.pins(oracle.cost_grid(s), a, b, want_plan=False, eta=eta, K=K)
            assert abs(served[q]["cost"] - o["cost"]) / o["cost"] <= 1e-9
    finally:
        ctx.close()


def test_server_rejects_invalid_requests():
    print("case serving invalid", flush=True)
    srv = P.Server(P.params(eta=0.1, max_outer=3), workers=1, max_batch=4)
    try:
        with pytest.raises(P.PinsError):
            srv.submit(P.COST_GRID, np.full(9, 1 / 9), np.full(9, 1 / 9), grid_s=2)  # 9 != 2*2
        bad = np.full(16, 1 / 16)
        bad[0] = -bad[0]
        with pytest.raises(P.PinsError):
            srv.submit(P.COST_GRID, bad, np.full(16, 1 / 16), grid_s=4)  # negative mass: rejected at submit
        ok = srv.submit(P.COST_GRID, np.full(16, 1 / 16), np.full(16, 1 / 16), grid_s=4)
        assert srv.wait(ok)["rc"] in (0, 1)
    finally:
        srv.close()
