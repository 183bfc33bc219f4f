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


def test_tuner_picks_a_schedule_and_tiles_and_keeps_results(ctx):
    """The tuner tries lanes 1..4, graph replay and 8 / 32 / 64 rows per tile for each
    size class present; the lane count and the graphs leave every result bitwise
    unchanged, and a solve with the chosen parameters reproduces the tuner's
    last outputs exactly (results depend on the tile rows only through each
    instance's own size class)."""
    print("case tuner 8 uneven dense instances", flush=True)
    probs, outs = _batch()
    prm = P.params(eta=0.03, max_outer=6)
    st = torch.cuda.Stream()
    rc, ref = ctx.solve_batch_device(probs, P.params(eta=0.03, max_outer=6, streams=1), outs, stream=st.cuda_stream)
    st.synchronize()
    assert rc == 0
    want = _host(outs)
    best, trials = ctx.tune_batch_device(probs, prm, outs, max_lanes=4, reps=1, stream=st.cuda_stream)
    st.synchronize()
    assert 1 <= best.streams <= 4 and best.graphs in (0, 1)
    # the batch's m span three size classes: 4 lane counts, graphs, 3 tile choices per class
    classes = {0 if p["m"] < 64 else 1 if p["m"] < 256 else 2 for p in probs}
    assert len(trials) == 4 + 1 + 3 * len(classes)
    assert all(t["ms"] > 0 for t in trials)
    chosen = [t for t in trials if t["streams"] == best.streams and t["graphs"] == best.graphs and
              t["tile_rows"] == list(best.tile_rows)]
    assert chosen and chosen[0]["ms"] == min(t["ms"] for t in trials)
    # lanes and graphs alone: bitwise the one-lane results
    for t in trials[:5]:
        o2 = [dict(alpha=torch.empty_like(o["alpha"]), beta=torch.empty_like(o["beta"])) for o in outs]
        rc, got = ctx.solve_batch_device(probs, P.params(eta=0.03, max_outer=6, streams=t["streams"],
                                                         graphs=t["graphs"]), o2, stream=st.cuda_stream)
        st.synchronize()
        for (a1, b1), (a2, b2) in zip(want, _host(o2)):
            assert np.array_equal(a1, a2) and np.array_equal(b1, b2)
    # the chosen configuration reproduces itself, and each instance alone equals its batched result
    o3 = [dict(alpha=torch.empty_like(o["alpha"]), beta=torch.empty_like(o["beta"])) for o in outs]
    rc, got = ctx.solve_batch_device(probs, best, o3, stream=st.cuda_stream)
    st.synchronize()
    assert rc == 0
    alone = P.params(eta=0.03, max_outer=6, tile_rows=list(best.tile_rows))
    for q in range(len(probs)):
        o1 = dict(alpha=torch.empty_like(outs[q]["alpha"]), beta=torch.empty_like(outs[q]["beta"]))
        _, r1 = ctx.solve_device(probs[q], alone, o1, stream=st.cuda_stream)
        st.synchronize()
        assert torch.equal(o1["alpha"], o3[q]["alpha"]) and r1["cost"] == got[q]["cost"], q


@pytest.mark.parametrize("lanes", [6, 8, 12])
def test_many_lanes_equal_one_lane(ctx, lanes):
    """Up to PINS_MAX_LANES (8) lanes, here more than the process's hardware
    queues, so that lane streams share them; a request above the cap runs on 8
    lanes.  Every instance bitwise its one-lane result (8 uneven dense
    instances: with 6 lanes two groups hold two instances, with 8 or more each
    lane one)."""
    print("case lanes %d" % lanes, flush=True)
    probs, outs = _batch()
    st = torch.cuda.Stream()
    rc, _ = ctx.solve_batch_device(probs, P.params(eta=0.03, max_outer=6, streams=1), outs, stream=st.cuda_stream)
    st.synchronize()
    assert rc == 0
    want = _host(outs)
    o2 = [dict(alpha=torch.empty_like(o["alpha"]), beta=torch.empty_like(o["beta"])) for o in outs]
    rc, got = ctx.solve_batch_device(probs, P.params(eta=0.03, max_outer=6, streams=lanes), o2, stream=st.cuda_stream)
    st.synchronize()
    assert rc == 0
    assert max(r["group"] for r in got) == min(lanes, 8) - 1
    for (a1, b1), (a2, b2) in zip(want, _host(o2)):
        assert np.array_equal(a1, a2) and np.array_equal(b1, b2)


@pytest.mark.parametrize("rows", [1, 3, 8, 32, 40, 64])
def test_tile_rows_parity(ctx, rows):
    """Dense passes with 1 to 64 rows per tile (every size class; 150 rows, so
    the last row block is ragged, and 40 rows leave a partial 16-row pass in
    the Sparsify fill and the output kernel): parity with the oracle at the
    FP64 bar."""
    import oracle
    from test_gpu_parity import check_parity, gpu_solve

    print("case tile rows %d" % rows, flush=True)
    C, a, b = _rand(150, 97, 31337)
    prm = P.params(eta=0.03, max_outer=8, tile_rows=[rows] * 4)
    g = gpu_solve(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b), prm)
    g["_C"] = C
    o = oracle.pins(C, a, b, eta=0.03, K=8)
    check_parity(g, o, a, b)


def test_tuner_tries_no_more_lanes_than_instances(ctx):
    print("case tuner 2 instances", flush=True)
    probs, outs = _batch()
    best, trials = ctx.tune_batch_device(probs[:2], P.params(eta=0.03, max_outer=2), outs[:2], max_lanes=4, reps=1)
    torch.cuda.synchronize()
    assert best.streams in (1, 2) and max(t["streams"] for t in trials) == 2


def test_tuner_rejects_bad_arguments(ctx):
    print("case tuner bad arguments", flush=True)
    probs, outs = _batch()
    prm = P.params(eta=0.03, max_outer=2)
    for kw in (dict(max_lanes=0), dict(max_lanes=9), dict(reps=0)):
        with pytest.raises(P.PinsError) as e:
            ctx.tune_batch_device(probs[:2], prm, outs[:2], **kw)
        assert e.value.code == P._binding.PINS_EINVAL
    with pytest.raises(P.PinsError) as e:
        ctx.solve_batch_device(probs[:2], P.params(eta=0.03, max_outer=2, tile_rows=[65, 0, 0, 0]), outs[:2])
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
