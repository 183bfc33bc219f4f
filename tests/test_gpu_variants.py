"""The paper's comparison variants, run by the same HIP kernels through the C ABI
(Section 5.1, methods (1)-(4)): each is a parameter setting of Alg. 2.

* Sinkhorn (no EPPA): K = 1, Sinkhorn iterations to a tight marginal error, no
  Newton steps (the entropic plan at eps = eta);
* Newton (no EPPA): K = 1, the default warm-up and sparse Newton;
* Sinkhorn + EPPA: K outer iterations, every subproblem solved by Sinkhorn;
* PINS: the defaults.

Each variant is compared with the oracle run with the same parameters, and the
finite-K equivalence (the plan of K outer iterations at eta is the entropic
plan at eta / K) is checked across variants on the GPU.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2502_03749_amd as P  # noqa: E402

from test_gpu_parity import _rand, check_parity, gpu_solve  # noqa: E402

VARIANTS = {
    "sinkhorn": dict(gpu=dict(max_outer=1, max_sinkhorn=200000, max_newton=0, warm_tol=1e-12, final_tol=1e-10),
                     orc=dict(K=1, T1=200000, T2=0, warm_tol=1e-12, final_tol=1e-10)),
    "newton": dict(gpu=dict(max_outer=1), orc=dict(K=1)),
    "sinkhorn_eppa": dict(gpu=dict(max_outer=8, max_sinkhorn=200000, max_newton=0, warm_tol=1e-12, final_tol=1e-10),
                          orc=dict(K=8, T1=200000, T2=0, warm_tol=1e-12, final_tol=1e-10)),
    "pins": dict(gpu=dict(max_outer=8), orc=dict(K=8)),
}


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_variant_parity(ctx, variant):
    print("case variant %s" % variant, flush=True)
    C, a, b = _rand(40, 30, 2024)
    eta = 0.05
    v = VARIANTS[variant]
    g = gpu_solve(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b), P.params(eta=eta, **v["gpu"]))
    g["_C"] = C
    o = oracle.pins(C, a, b, eta=eta, **v["orc"])
    assert o["status"] == 0
    check_parity(g, o, a, b)


def test_variants_reach_the_same_finite_K_plan(ctx):
    """Sinkhorn at eta/K, Sinkhorn + EPPA and PINS at (eta, K): one plan."""
    print("case variant equivalence", flush=True)
    C, a, b = _rand(40, 30, 2025)
    eta, K = 0.05, 8
    prob = dict(kind=P.COST_DENSE, C=C, a=a, b=b)
    sk = gpu_solve(ctx, prob, P.params(eta=eta / K, max_outer=1, max_sinkhorn=200000, max_newton=0, warm_tol=1e-12,
                                       final_tol=1e-10))
    se = gpu_solve(ctx, prob, P.params(eta=eta, max_outer=K, max_sinkhorn=200000, max_newton=0, warm_tol=1e-12,
                                       final_tol=1e-10))
    pn = gpu_solve(ctx, prob, P.params(eta=eta, max_outer=K))
    for r in (sk, se, pn):
        assert r["rc"] == 0 and r["resid"] <= 1e-10
    assert np.abs(sk["X"] - pn["X"]).sum() <= 1e-9
    assert np.abs(se["X"] - pn["X"]).sum() <= 1e-9
    assert abs(sk["cost"] - pn["cost"]) / pn["cost"] <= 1e-9


@pytest.mark.parametrize("kind", ["dense", "grid", "points"])
def test_matrix_free_hessian_products_parity(ctx, kind):
    """params.hvp = 1: the Newton CG multiplies by the full Hessian, X~ recomputed
    tile by tile (the paper's streaming variant; no Sparsify).  Same converged
    output as the oracle (whose CG uses the sparsified Hessian)."""
    print("case matrix-free %s" % kind, flush=True)
    import workloads as W

    if kind == "dense":
        C, a, b = _rand(45, 38, 2031)
        prob = dict(kind=P.COST_DENSE, C=C, a=a, b=b)
        eta, K = 0.05, 8
    elif kind == "grid":
        pr = W.blob_pair(11, s=12)
        C, a, b = oracle.cost_grid(12), pr["a"], pr["b"]
        prob = dict(kind=P.COST_GRID, grid_s=12, a=a, b=b)
        eta, K = 0.1, 10
    else:
        inst = W.points_instance(3, m=60, n=50, d=8)
        C, a, b = oracle.cost_points(inst["x"], inst["y"]), inst["a"], inst["b"]
        prob = dict(kind=P.COST_POINTS, x=inst["x"], y=inst["y"], a=a, b=b)
        eta, K = 0.02, 6
    g = gpu_solve(ctx, prob, P.params(eta=eta, max_outer=K, hvp=1))
    g["_C"] = C
    o = oracle.pins(C, a, b, eta=eta, K=K)
    check_parity(g, o, a, b)
    assert g["newton_iters"] > 0 and g["cg_iters"] > 0


def test_hybrid_hessian_schedule_parity(ctx):
    """params.hvp = 2: matrix-free products in the first outer iterations, the
    sparsified Hessian after; converged output as the oracle's."""
    print("case hybrid hessian", flush=True)
    import workloads as W

    pr = W.blob_pair(13, s=14)
    C, a, b = oracle.cost_grid(14), pr["a"], pr["b"]
    eta, K = 0.1, 12
    for prec in (P.FP64, P.MIXED):
        g = gpu_solve(ctx, dict(kind=P.COST_GRID, grid_s=14, a=a, b=b),
                      P.params(eta=eta, max_outer=K, hvp=2, hvp_switch=4, precision=prec))
        g["_C"] = C
        o = oracle.pins(C, a, b, eta=eta, K=K)
        if prec == P.FP64:
            check_parity(g, o, a, b)
        else:
            assert g["rc"] == 0 and g["resid"] <= 1e-10 and abs(g["cost"] - o["cost"]) / o["cost"] <= 1e-6
        assert g["kern_work"]["pcg_wide"] > 0 and g["kern_work"]["pcg"] > 0


def test_device_texp_matches_host_reference():
    """The FP64 dense passes' exp evaluated on the device (pins_probe_texp, the
    kernels' own code and table) against numpy's exp: within 1 ulp (plus one
    for the reference's own rounding) over [-746, 710], subnormal results
    included; 0 below the range, inf above it, NaN kept."""
    import numpy as np
    import torch

    import paper_2502_03749_amd as P

    g = np.random.default_rng(11)
    x = np.concatenate([g.uniform(-746.0, 710.0, 2_000_000), g.uniform(-745.2, -708.0, 200_000),
                        g.uniform(-1.0, 1.0, 200_000), [0.0, -0.0, 709.78, -745.13, -746.5, 710.5, np.inf,
                                                        -np.inf, np.nan]])
    xt = torch.as_tensor(x, dtype=torch.float64, device="cuda:0")
    yt = torch.empty_like(xt)
    P.probe_texp(xt, yt, stream=torch.cuda.current_stream().cuda_stream)
    y = yt.cpu().numpy()
    ref = np.exp(x)
    fin = np.isfinite(ref) & np.isfinite(x)
    ulp = np.spacing(np.abs(ref[fin]))
    ulp[ref[fin] == 0.0] = np.nextafter(0.0, 1.0)
    err = np.abs(y[fin] - ref[fin]) / ulp
    assert err.max() <= 2.0, (err.max(), x[fin][err.argmax()])
    assert y[-5] == 0.0 and np.isinf(y[-4]) and np.isinf(y[-3]) and y[-2] == 0.0 and np.isnan(y[-1])
