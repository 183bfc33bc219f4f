"""The batch autotuner (pins_tune_batch_device) and the exponential probe through the C ABI.

The lane count it searches is a launch-schedule choice only: the batch solved
with any count must give bitwise the single-lane results, and the tuner's own
outputs must be those results.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2502_03749_amd as P  # noqa: E402

from test_gpu_parity import _rand  # noqa: E402

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def _batch():
    t = lambda v: torch.as_tensor(np.ascontiguousarray(v), dtype=torch.float64, device=DEV)
    probs, outs = [], []
    for q, (m, n) in enumerate([(40, 30), (7, 90), (64, 64), (25, 25), (90, 11), (33, 47), (5, 5), (70, 20)]):
        C, a, b = _rand(m, n, 300 + q)
        probs.append(dict(kind=P.COST_DENSE, m=m, n=n, C=t(C), a=t(a), b=t(b), cost_scale=1.0))
        outs.append(dict(alpha=torch.empty(m, dtype=torch.float64, device=DEV),
                         beta=torch.empty(n, dtype=torch.float64, device=DEV)))
    return probs, outs


def _host(outs):
    return [(o["alpha"].cpu().numpy().copy(), o["beta"].cpu().numpy().copy()) for o in outs]


def test_tuner_picks_a_lane_count_and_keeps_results(ctx):
    print("case tuner 8 uneven dense instances", flush=True)
    probs, outs = _batch()
    prm = P.params(eta=0.03, max_outer=6)
    st = torch.cuda.current_stream().cuda_stream
    rc, ref = ctx.solve_batch_device(probs, P.params(eta=0.03, max_outer=6, streams=1), outs, stream=st)
    torch.cuda.synchronize()
    assert rc == 0
    want = _host(outs)
    best, ms = ctx.tune_batch_device(probs, prm, outs, max_lanes=4, reps=1, stream=st)
    torch.cuda.synchronize()
    assert 1 <= best <= 4 and len(ms) == 4
    assert all(v > 0 for v in ms) and ms[best - 1] == min(ms)
    for (a1, b1), (a2, b2) in zip(want, _host(outs)):
        assert np.array_equal(a1, a2) and np.array_equal(b1, b2)
    # the chosen count gives the same results as one lane
    rc, got = ctx.solve_batch_device(probs, P.params(eta=0.03, max_outer=6, streams=best), outs, stream=st)
    torch.cuda.synchronize()
    assert rc == 0
    for (a1, b1), (a2, b2) in zip(want, _host(outs)):
        assert np.array_equal(a1, a2) and np.array_equal(b1, b2)
    for r1, r2 in zip(ref, got):
        assert r1["cost"] == r2["cost"] and r1["resid"] == r2["resid"]


def test_tuner_tries_no_more_lanes_than_instances(ctx):
    print("case tuner 2 instances", flush=True)
    probs, outs = _batch()
    best, ms = ctx.tune_batch_device(probs[:2], P.params(eta=0.03, max_outer=2), outs[:2], max_lanes=4, reps=1)
    torch.cuda.synchronize()
    assert best in (1, 2) and ms[0] > 0 and ms[1] > 0 and ms[2] == 0.0 and ms[3] == 0.0


def test_tuner_rejects_bad_arguments(ctx):
    print("case tuner bad arguments", flush=True)
    probs, outs = _batch()
    prm = P.params(eta=0.03, max_outer=2)
    for kw in (dict(max_lanes=0), dict(max_lanes=5), dict(reps=0)):
        with pytest.raises(P.PinsError) as e:
            ctx.tune_batch_device(probs[:2], prm, outs[:2], **kw)
        assert e.value.code == P._binding.PINS_EINVAL


def test_exp_probe_rate_is_plausible():
    """The exponential probe runs and gives a rate between 1 and 64 float exponentials per
    compute-unit cycle (256 CUs at 2.4 GHz); 64 (4 SIMDs x 16 lanes) is the full VALU rate."""
    print("case exp probe", flush=True)
    rate, ms = P.probe_exp_rate(0, blocks=2048, iters=1024)
    assert ms > 0.0
    per_cu_cycle = rate / (256 * 2.4e9)
    assert 1.0 <= per_cu_cycle <= 64.0, per_cu_cycle


@pytest.mark.parametrize("lanes", [1, 3])
def test_graph_replay_equals_kernel_by_kernel(ctx, lanes):
    """params.graphs: outer iterations on the quick path (one warm-up iteration,
    one-block CGs) replay one captured HIP graph (shift, warm-up iteration,
    Newton pass, Sparsify, CG, first Armijo trial) instead of launching kernel
    by kernel.  The graph is replayed in most of the K = 60 outer iterations,
    with the solver's readbacks and eager launches in between; every
    instance's result must be bitwise the kernel-by-kernel one.  12 pairs of
    28x28 histograms (grid cost), eta = 0.1, on a non-default caller stream,
    one lane and three lanes."""
    import workloads as W

    s, n, K = 28, 784, 60
    print("case graphs lanes %d" % lanes, flush=True)
    t = lambda v: torch.as_tensor(np.ascontiguousarray(v), dtype=torch.float64, device=DEV)
    pairs = [W.blob_pair(i, s=s) for i in range(12)]
    probs = [dict(kind=P.COST_GRID, m=n, n=n, grid_s=s, a=t(p["a"]), b=t(p["b"])) for p in pairs]
    st = torch.cuda.Stream()
    res = {}
    for g in (0, 1):
        outs = [dict(alpha=torch.empty(n, dtype=torch.float64, device=DEV),
                     beta=torch.empty(n, dtype=torch.float64, device=DEV)) for _ in pairs]
        torch.cuda.synchronize()
        rc, rs = ctx.solve_batch_device(probs, P.params(eta=0.1, max_outer=K, streams=lanes, graphs=g), outs,
                                        stream=st.cuda_stream)
        st.synchronize()
        assert rc == 0
        res[g] = (rs, outs)
    for q in range(len(pairs)):
        r0, r1 = res[0][0][q], res[1][0][q]
        assert r0["cost"] == r1["cost"] and r0["newton_iters"] == r1["newton_iters"], q
        assert r0["cg_iters"] == r1["cg_iters"] and r0["sinkhorn_iters"] == r1["sinkhorn_iters"], q
        assert torch.equal(res[0][1][q]["alpha"], res[1][1][q]["alpha"]), q
        assert torch.equal(res[0][1][q]["beta"], res[1][1][q]["beta"]), q
