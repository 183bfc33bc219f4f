"""Checkpoint / resume of the EPPA outer loop through pins_solve_resume.

After k completed outer iterations of Alg. 2 the next subproblem, eq.
(eppa-sub), is fixed by k, the dual iterate (F, G) and the accumulated shifts
(A, B).  A solve split into several calls, each resuming from the state the
previous one saved, must therefore give bitwise the unbroken solve's outputs,
and the unbroken solve must match the oracle.  Invalid states are rejected
before anything runs.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2502_03749_amd as P  # noqa: E402

from test_gpu_parity import _rand  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def _split(ctx, prob, prm, stops):
    """Run the solve as consecutive calls ending at each of `stops`; return the last result and
    the per-call results."""
    state, calls = None, []
    for s in stops:
        r = ctx.solve_resume(prm=prm, state=state, stop=s, **prob)
        assert r["rc"] >= 0, r
        assert r["outer_iters"] == s and r["state"]["outer_done"] == s
        state = r["state"]
        calls.append(r)
    return calls[-1], calls


def _same(r1, r2):
    for k in ("alpha", "beta"):
        assert np.array_equal(r1[k], r2[k]), k
    if r1["X"] is not None:
        assert np.array_equal(r1["X"], r2["X"])
    for k in ("cost", "resid", "dual", "gap", "entropy", "eps", "flags", "status", "nnz_last"):
        assert r1[k] == r2[k], (k, r1[k], r2[k])


CASES = {
    # dense FP64, sparsified Hessian products throughout
    "dense_fp64": dict(mk=lambda: dict(kind=P.COST_DENSE, C=_rand(60, 45, 77)[0], a=_rand(60, 45, 77)[1],
                                       b=_rand(60, 45, 77)[2], cost_scale=1.0),
                       prm=dict(eta=0.03, max_outer=12), stops=[4, 9, 12]),
    # hybrid products: the split falls on both sides of the switch to sparsified products
    "dense_hybrid": dict(mk=lambda: dict(kind=P.COST_DENSE, C=_rand(70, 90, 78)[0], a=_rand(70, 90, 78)[1],
                                         b=_rand(70, 90, 78)[2], cost_scale=1.0),
                         prm=dict(eta=0.02, max_outer=10, hvp=2, hvp_switch=5), stops=[3, 5, 6, 10]),
    # streamed grid cost, mixed precision (FP32 warm-up sweeps)
    "grid_mixed": dict(mk=lambda: dict(kind=P.COST_GRID, grid_s=8,
                                       a=np.random.default_rng(5).dirichlet(np.ones(64)) * 0.999 + 0.001 / 64,
                                       b=np.random.default_rng(6).dirichlet(np.ones(64)) * 0.999 + 0.001 / 64),
                       prm=dict(eta=0.01, max_outer=8, precision=P.MIXED), stops=[1, 2, 7, 8]),
}


@pytest.mark.parametrize("case", list(CASES))
def test_split_solve_equals_unbroken_solve(ctx, case):
    print("case resume %s" % case, flush=True)
    c = CASES[case]
    prob = c["mk"]()
    prob["want_plan"] = True
    prm = P.params(**c["prm"])
    whole = ctx.solve(prm=prm, **prob)
    assert whole["rc"] == 0, whole
    # one call over every iteration is pins_solve
    one = ctx.solve_resume(prm=prm, **prob)
    _same(one, whole)
    assert one["state"]["outer_done"] == prm.max_outer
    last, calls = _split(ctx, prob, prm, c["stops"])
    _same(last, whole)
    assert last["outer_iters"] == whole["outer_iters"]
    # the work is the unbroken solve's, divided between the calls
    for k in ("sinkhorn_iters", "newton_iters", "cg_iters", "fallbacks"):
        assert sum(r[k] for r in calls) == whole[k], k
    # an intermediate call's outputs are the plan after its iterations, at eps = eta / stop
    mid = calls[0]
    assert mid["eps"] == prm.eta / c["stops"][0]
    assert np.isfinite(mid["cost"]) and mid["resid"] >= 0.0


def test_resumed_solve_matches_oracle(ctx):
    print("case resume oracle", flush=True)
    C, a, b = _rand(37, 53, 91)
    eta, K = 0.03, 8
    prm = P.params(eta=eta, max_outer=K)
    last, _ = _split(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b, cost_scale=1.0, want_plan=True), prm, [3, 8])
    o = oracle.pins(C, a, b, eta=eta, K=K)
    assert last["rc"] == 0
    assert abs(last["cost"] - o["cost"]) / abs(o["cost"]) <= 1e-9
    assert last["resid"] <= 1e-10
    assert np.abs(last["X"] - o["X"]).sum() <= 1e-9
    assert np.abs(last["alpha"] - o["alpha"]).max() <= 1e-8
    assert np.abs(last["beta"] - o["beta"]).max() <= 1e-8


def test_resume_rejects_invalid_states(ctx):
    print("case resume invalid", flush=True)
    C, a, b = _rand(20, 15, 92)
    prob = dict(kind=P.COST_DENSE, C=C, a=a, b=b, cost_scale=1.0)
    prm = P.params(eta=0.05, max_outer=6)
    st = ctx.solve_resume(prm=prm, stop=2, **prob)["state"]

    def rejected(code, **kw):
        args = dict(prm=prm, state=st, stop=6)
        args.update(kw)
        with pytest.raises(P.PinsError) as e:
            ctx.solve_resume(**args, **prob)
        assert e.value.code == code, e.value

    rejected(P._binding.PINS_EINVAL, stop=7)                         # beyond K
    rejected(P._binding.PINS_EINVAL, stop=2)                         # nothing left to run
    rejected(P._binding.PINS_EINVAL, state=dict(st, outer_done=0))   # not a completed iteration
    bad = dict(st, F=st["F"].copy())
    bad["F"][3] = np.nan
    rejected(P._binding.PINS_EINVAL, state=bad)                      # non-finite state
    rejected(P._binding.PINS_EINVAL, state=dict(st, G=st["G"][:-1], B=st["B"][:-1]))  # sizes
    rejected(P._binding.PINS_EUNSUPPORTED, prm=P.params(eta=0.05, max_outer=6, shift_mode=P.SHIFT_MATERIALIZED))
    # the context still works and the valid resume completes
    r = ctx.solve_resume(prm=prm, state=st, stop=6, **prob)
    assert r["rc"] == 0 and r["state"]["outer_done"] == 6
