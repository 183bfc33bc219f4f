"""The entry point that allocates nothing (pins_solve_device_noalloc) against
pins_solve_device, through the C ABI: two calls in a row on the library's
fixed device scratch, the second with a smaller problem, each bitwise equal to
the allocating entry point's result (same kernels, same arithmetic), and the
size limit rejected before anything runs.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2502_03749_amd as P  # noqa: E402

DEV = torch.device("cuda:0")


def _t(v):
    return torch.as_tensor(np.ascontiguousarray(v), dtype=torch.float64, device=DEV)


def _problem(kind, m, n, seed):
    if kind == P.COST_DENSE:
        inst = W.points_instance(seed, m=m, n=n)
        C = W.sqeuclid_dense(inst["x"], inst["y"])
        return dict(kind=P.COST_DENSE, m=m, n=n, C=_t(C), a=_t(inst["a"]), b=_t(inst["b"]), cost_scale=1.0)
    s = int(round(m ** 0.5))
    a = W.blob_histogram(seed, 0, s=s)
    b = W.blob_histogram(seed, 1, s=s)
    return dict(kind=P.COST_GRID, m=s * s, n=s * s, grid_s=s, a=_t(a), b=_t(b))


def _outs(m, n):
    return dict(alpha=torch.empty(m, dtype=torch.float64, device=DEV),
                beta=torch.empty(n, dtype=torch.float64, device=DEV),
                X=torch.empty(m, n, dtype=torch.float64, device=DEV))


def _run(ctx, fn, prob, prm, stream):
    out = _outs(prob["m"], prob["n"])
    rc, r = getattr(ctx, fn)(prob, prm, out, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    return rc, r, {k: v.cpu().numpy() for k, v in out.items()}


def _same(ra, oa, rb, ob):
    assert ra[0] == rb[0]
    for k in ("alpha", "beta", "X"):
        assert np.array_equal(oa[k], ob[k]), k
    for k in ("cost", "resid", "dual", "entropy", "newton_iters", "cg_iters", "sinkhorn_iters", "nnz_last",
              "fallbacks"):
        assert ra[1][k] == rb[1][k], k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_allocating_entry_point(precision):
    prm = P.params(eta=1e-2, max_outer=12, precision=P.FP64 if precision == "fp64" else P.MIXED)
    ctx = P.Context(0)
    st = torch.cuda.Stream()  # a non-default caller stream
    try:
        # two calls in a row on the fixed scratch, the second smaller (and of
        # another cost kind); the first call's contents are still in the array
        cases = [(P.COST_DENSE, 96, 80, 3), (P.COST_GRID, 36, 36, 5)]
        for kind, m, n, seed in cases:
            prob = _problem(kind, m, n, seed)
            print("noalloc case: kind=%d m=%d n=%d precision=%s" % (kind, m, n, precision), flush=True)
            r_fix = _run(ctx, "solve_device_noalloc", prob, prm, st)
            r_ref = _run(ctx, "solve_device", prob, prm, st)
            assert r_fix[0] >= 0 and r_fix[1]["resid"] <= 1e-9
            _same(r_fix[:2], r_fix[2], r_ref[:2], r_ref[2])
        # once more the first problem: the second call's leftovers change nothing
        prob = _problem(*cases[0])
        r_fix = _run(ctx, "solve_device_noalloc", prob, prm, st)
        r_ref = _run(ctx, "solve_device", prob, prm, st)
        _same(r_fix[:2], r_fix[2], r_ref[:2], r_ref[2])
    finally:
        ctx.close()


def test_noalloc_rejects_sizes_beyond_the_scratch_and_profiling():
    ctx = P.Context(0)
    try:
        prm = P.params(eta=1e-3, max_outer=2)
        s = 128  # a 128 x 128 grid needs several hundred MB of workspace
        assert P.workspace_bytes([dict(kind=P.COST_GRID, m=s * s, n=s * s, grid_s=s)], prm) > P.NOALLOC_SCRATCH_BYTES
        u = torch.full((s * s,), 1.0 / (s * s), dtype=torch.float64, device=DEV)
        prob = dict(kind=P.COST_GRID, m=s * s, n=s * s, grid_s=s, a=u, b=u)
        with pytest.raises(P.PinsError) as e:
            ctx.solve_device_noalloc(prob, prm, dict(alpha=torch.empty_like(u), beta=torch.empty_like(u)))
        assert e.value.code == -2 and "scratch" in str(e.value)
        small = _problem(P.COST_DENSE, 20, 16, 1)
        with pytest.raises(P.PinsError) as e:
            ctx.solve_device_noalloc(small, P.params(eta=1e-2, max_outer=2, profile=1), _outs(20, 16))
        assert e.value.code == -1
    finally:
        ctx.close()
