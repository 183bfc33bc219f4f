"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bar (FP64 path): relative cost difference <= 1e-9, GPU marginal residual
<= 1e-10, plan L1 distance <= 1e-9, gauge-fixed potentials within 1e-8
(costs are normalised to [0, 1]).  Mixed path: relative cost difference
<= 1e-6.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2502_03749_amd as P  # noqa: E402

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def _t(v):
    return torch.as_tensor(np.ascontiguousarray(v), dtype=torch.float64, device=DEV)


def gpu_solve(ctx, prob, prm, want_plan=True):
    """Device-API solve of a host problem dict (kind, a, b, C | x,y | grid_s)."""
    m, n = len(prob["a"]), len(prob["b"])
    default_scale = 1.0 if prob["kind"] == P.COST_DENSE else 0.0  # dense C is used as given
    dp = dict(kind=prob["kind"], m=m, n=n, a=_t(prob["a"]), b=_t(prob["b"]),
              cost_scale=prob.get("cost_scale", default_scale))
    if "C" in prob:
        dp["C"] = _t(prob["C"])
    if "x" in prob:
        dp["x"], dp["y"], dp["d"] = _t(prob["x"]), _t(prob["y"]), prob["x"].shape[1]
    if "grid_s" in prob:
        dp["grid_s"] = prob["grid_s"]
    out = dict(alpha=torch.empty(m, dtype=torch.float64, device=DEV),
               beta=torch.empty(n, dtype=torch.float64, device=DEV),
               X=torch.empty(m, n, dtype=torch.float64, device=DEV) if want_plan else None)
    rc, r = ctx.solve_device(dp, prm, out, stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    r["rc"] = rc
    r["alpha"] = out["alpha"].cpu().numpy()
    r["beta"] = out["beta"].cpu().numpy()
    r["X"] = out["X"].cpu().numpy() if want_plan else None
    return r


def check_parity(g, o, a, b, cost_tol=1e-9, plan_tol=1e-9, resid_tol=1e-10):
    rel = abs(g["cost"] - o["cost"]) / max(abs(o["cost"]), 1e-300)
    assert g["rc"] == 0, g
    assert rel <= cost_tol, (g["cost"], o["cost"], rel)
    assert g["resid"] <= resid_tol, g["resid"]
    if g["X"] is not None and o["X"] is not None:
        l1 = np.abs(g["X"] - o["X"]).sum()
        assert l1 <= plan_tol, l1
        # the plan is the exponential of the potentials (standard form)
        Xp = np.exp((g["alpha"][:, None] + g["beta"][None, :] - g["_C"]) / g["eps"])
        assert np.abs(Xp - g["X"]).sum() <= 1e-10
    # gauge <a,alpha> = <b,beta>; gauge-fixed potentials agree (costs are O(1))
    assert abs(a @ g["alpha"] - b @ g["beta"]) <= 1e-12
    assert np.abs(g["alpha"] - o["alpha"]).max() <= 1e-8
    assert np.abs(g["beta"] - o["beta"]).max() <= 1e-8
    # where the oracle never needed the Sinkhorn fallback (no ascent step from
    # the sparse Newton direction), neither may the HIP path
    if o["fallbacks"] == 0:
        assert g["fallbacks"] == 0, g["fallbacks"]
    return rel


def _rand(m, n, seed):
    g = np.random.default_rng(seed)
    C = g.uniform(0, 1, (m, n))
    a = g.uniform(0.2, 1.0, m)
    b = g.uniform(0.2, 1.0, n)
    return C, a / a.sum(), b / b.sum()


@pytest.mark.parametrize("m,n,eta,K", [(1, 1, 0.1, 2), (1, 5, 0.1, 3), (6, 1, 0.1, 3), (2, 2, 0.4, 3),
                                       (7, 5, 0.05, 6), (37, 53, 0.03, 8), (100, 100, 0.01, 10),
                                       (300, 17, 0.02, 5), (17, 600, 0.02, 5)])
def test_dense_parity(ctx, m, n, eta, K):
    print("case dense m=%d n=%d eta=%g K=%d" % (m, n, eta, K), flush=True)
    C, a, b = _rand(m, n, 1000 + m * 7 + n)
    prm = P.params(eta=eta, max_outer=K)
    g = gpu_solve(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b), prm)
    g["_C"] = C
    o = oracle.pins(C, a, b, eta=eta, K=K)
    check_parity(g, o, a, b)


def test_points_plane_instance_reaches_lp(ctx):
    """100x100 plane instance, K = 2000: parity with the oracle and <= 1e-8 vs the LP."""
    from oracle import lp

    inst = W.points_instance(0)
    C = oracle.cost_points(inst["x"], inst["y"])
    K = 2000
    print("case points 100x100 K=%d" % K, flush=True)
    prm = P.params(eta=1e-2, max_outer=K)
    g = gpu_solve(ctx, dict(kind=P.COST_POINTS, x=inst["x"], y=inst["y"], a=inst["a"], b=inst["b"]), prm)
    g["_C"] = C
    o = oracle.pins(C, inst["a"], inst["b"], eta=1e-2, K=K)
    check_parity(g, o, inst["a"], inst["b"])
    ot, _ = lp.lp_highs(C, inst["a"], inst["b"])
    assert abs(g["cost"] - ot) / ot <= 1e-8


@pytest.mark.parametrize("s,K", [(5, 6), (12, 10)])
def test_grid_streamed_parity(ctx, s, K):
    print("case grid s=%d K=%d" % (s, K), flush=True)
    pr = W.blob_pair(3, s=s)
    C = oracle.cost_grid(s)
    prm = P.params(eta=0.1, max_outer=K)
    g = gpu_solve(ctx, dict(kind=P.COST_GRID, grid_s=s, a=pr["a"], b=pr["b"]), prm)
    g["_C"] = C
    o = oracle.pins(C, pr["a"], pr["b"], eta=0.1, K=K)
    check_parity(g, o, pr["a"], pr["b"])


@pytest.mark.parametrize("kind", ["dense", "grid"])
def test_materialised_shift_parity(ctx, kind):
    print("case materialised %s" % kind, flush=True)
    if kind == "dense":
        C, a, b = _rand(40, 29, 77)
        prob = dict(kind=P.COST_DENSE, C=C, a=a, b=b)
        eta = 0.02
    else:
        pr = W.blob_pair(5, s=9)
        C, a, b = oracle.cost_grid(9), pr["a"], pr["b"]
        prob = dict(kind=P.COST_GRID, grid_s=9, a=a, b=b)
        eta = 0.1
    K = 12
    prm = P.params(eta=eta, max_outer=K, shift_mode=P.SHIFT_MATERIALIZED)
    g = gpu_solve(ctx, prob, prm)
    g["_C"] = C
    o = oracle.pins(C, a, b, eta=eta, K=K)
    check_parity(g, o, a, b)


@pytest.mark.parametrize("kind", ["dense", "grid"])
def test_mixed_precision_parity(ctx, kind):
    print("case mixed %s" % kind, flush=True)
    if kind == "dense":
        C, a, b = _rand(64, 48, 91)
        prob = dict(kind=P.COST_DENSE, C=C, a=a, b=b)
        eta = 0.02
    else:
        pr = W.blob_pair(7, s=14)
        C, a, b = oracle.cost_grid(14), pr["a"], pr["b"]
        prob = dict(kind=P.COST_GRID, grid_s=14, a=a, b=b)
        eta = 0.1
    K = 15
    prm = P.params(eta=eta, max_outer=K, precision=P.MIXED)
    g = gpu_solve(ctx, prob, prm)
    g["_C"] = C
    o = oracle.pins(C, a, b, eta=eta, K=K)
    rel = abs(g["cost"] - o["cost"]) / o["cost"]
    assert g["rc"] == 0 and rel <= 1e-6 and g["resid"] <= 1e-10


def test_batch_equals_alone(ctx):
    """Uneven batch: every instance's result is bitwise the one it gets alone."""
    print("case batch", flush=True)
    shapes = [(7, 5), (64, 33), (130, 257), (1, 9), (300, 300)]
    probs, outs, hosts = [], [], []
    prm = P.params(eta=0.03, max_outer=6)
    for q, (m, n) in enumerate(shapes):
        C, a, b = _rand(m, n, 500 + q)
        hosts.append((C, a, b))
        probs.append(dict(kind=P.COST_DENSE, m=m, n=n, C=_t(C), a=_t(a), b=_t(b), cost_scale=1.0))
        outs.append(dict(alpha=torch.empty(m, dtype=torch.float64, device=DEV),
                         beta=torch.empty(n, dtype=torch.float64, device=DEV)))
    rc, rs = ctx.solve_batch_device(probs, prm, outs, stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert rc == 0
    for q, (C, a, b) in enumerate(hosts):
        g = gpu_solve(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b), prm, want_plan=False)
        assert rs[q]["cost"] == g["cost"], q
        assert np.array_equal(outs[q]["alpha"].cpu().numpy(), g["alpha"]), q
        assert np.array_equal(outs[q]["beta"].cpu().numpy(), g["beta"]), q
        assert rs[q]["newton_iters"] == g["newton_iters"] and rs[q]["cg_iters"] == g["cg_iters"]


def test_multi_lane_batch_equals_alone(ctx):
    """A batch split over three concurrent lanes (own streams and host threads)
    gives every instance bitwise the result it gets alone."""
    print("case multi-lane batch", flush=True)
    shapes = [(40, 30), (64, 64), (7, 90), (120, 33), (50, 50), (9, 9), (200, 150)]
    probs, outs, hosts = [], [], []
    prm = P.params(eta=0.03, max_outer=5, streams=3)
    for q, (m, n) in enumerate(shapes):
        C, a, b = _rand(m, n, 900 + q)
        hosts.append((C, a, b))
        probs.append(dict(kind=P.COST_DENSE, m=m, n=n, C=_t(C), a=_t(a), b=_t(b), cost_scale=1.0))
        outs.append(dict(alpha=torch.empty(m, dtype=torch.float64, device=DEV),
                         beta=torch.empty(n, dtype=torch.float64, device=DEV)))
    rc, rs = ctx.solve_batch_device(probs, prm, outs, stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert rc == 0
    assert len({r["group"] for r in rs}) == 3
    for q, (C, a, b) in enumerate(hosts):
        g = gpu_solve(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b), P.params(eta=0.03, max_outer=5), want_plan=False)
        assert rs[q]["cost"] == g["cost"], q
        assert np.array_equal(outs[q]["alpha"].cpu().numpy(), g["alpha"]), q


def test_deterministic(ctx):
    print("case determinism", flush=True)
    C, a, b = _rand(90, 70, 3)
    prm = P.params(eta=0.02, max_outer=8)
    g1 = gpu_solve(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b), prm)
    g2 = gpu_solve(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b), prm)
    assert g1["cost"] == g2["cost"]
    assert np.array_equal(g1["X"], g2["X"]) and np.array_equal(g1["alpha"], g2["alpha"])


def test_host_api_matches_device_api(ctx):
    print("case host api", flush=True)
    C, a, b = _rand(33, 44, 8)
    prm = P.params(eta=0.03, max_outer=5)
    h = ctx.solve(P.COST_DENSE, a, b, prm, C=C, want_plan=True, cost_scale=1.0)
    g = gpu_solve(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b), prm)
    assert h["cost"] == g["cost"]
    assert np.array_equal(h["X"], g["X"]) and np.array_equal(h["alpha"], g["alpha"])


def test_invalid_inputs_rejected(ctx):
    print("case invalid", flush=True)
    C, a, b = _rand(5, 4, 1)
    prm = P.params(eta=0.1, max_outer=2)
    bad_a = a.copy()
    bad_a[0] += 1e-6
    with pytest.raises(P.PinsError) as e:
        ctx.solve(P.COST_DENSE, bad_a, b, prm, C=C)
    assert e.value.code == -1
    neg = a.copy()
    neg[1] = -neg[1]
    with pytest.raises(P.PinsError):
        ctx.solve(P.COST_DENSE, neg, b, prm, C=C)
    with pytest.raises(P.PinsError):
        ctx.solve(P.COST_DENSE, a, b, P.params(eta=0.0), C=C)
    Cn = C.copy()
    Cn[2, 3] = np.nan
    with pytest.raises(P.PinsError) as e:
        ctx.solve(P.COST_DENSE, a, b, prm, C=Cn)
    assert e.value.code == -1
    # the context stays usable
    r = ctx.solve(P.COST_DENSE, a, b, prm, C=C)
    assert r["rc"] == 0


def test_caps_report_not_converged(ctx):
    print("case caps", flush=True)
    C, a, b = _rand(30, 30, 12)
    r = ctx.solve(P.COST_DENSE, a, b, P.params(eta=0.01, max_outer=3, max_newton=0, max_sinkhorn=1), C=C)
    assert r["rc"] == 1 and (r["flags"] & 1)
    assert np.isfinite(r["alpha"]).all() and np.isfinite(r["cost"])


@pytest.mark.parametrize("case", ["square", "tall"])
def test_large_instances_parity(ctx, case):
    """Dense instances above the one-block CG's limit (m + n > 4096): the wide
    CG over many blocks, with 16-bit indices (m, n <= 65536)."""
    print("case large %s" % case, flush=True)
    m, n = (4100, 4000) if case == "square" else (6000, 2300)
    C, a, b = _rand(m, n, 4242 + m)
    eta, K = 0.05, 1
    prm = P.params(eta=eta, max_outer=K)
    g = gpu_solve(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b), prm)
    g["_C"] = C
    o = oracle.pins(C, a, b, eta=eta, K=K)
    check_parity(g, o, a, b)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_int32_index_storage_parity(ctx, precision):
    """m > 65535 makes the wide CG's copy of S store 32-bit byte offsets
    (16-bit indices otherwise), with double (FP64) or float (mixed) values;
    parity in both precisions."""
    print("case tall 70000x3 %s" % precision, flush=True)
    m, n = 70000, 3
    C, a, b = _rand(m, n, 515)
    eta, K = 0.05, 3
    prm = P.params(eta=eta, max_outer=K, precision=P.FP64 if precision == "fp64" else P.MIXED)
    g = gpu_solve(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b), prm)
    g["_C"] = C
    o = oracle.pins(C, a, b, eta=eta, K=K)
    if precision == "fp64":
        check_parity(g, o, a, b)
    else:
        rel = abs(g["cost"] - o["cost"]) / o["cost"]
        assert g["rc"] == 0 and rel <= 1e-6 and g["resid"] <= 1e-10


@pytest.mark.parametrize("precision,hvp_switch", [("mixed", 15), ("fp64", 15), ("mixed", 0)])
def test_full_size_batch_sampled_parity(ctx, precision, hvp_switch):
    """The benchmarked configuration itself: 64 pairs of 28x28 histograms, grid
    cost, eta = 0.1, K = 250, one batched call over four lanes with the default
    tiles, with the timed Hessian schedule (matrix-free products for the first
    15 outer iterations, sparsified after) and with sparsified products
    throughout.  Every instance converges (status OK, marginal residual <= 1e-10,
    gauge); pairs 0..15 match the oracle's stored outputs at the same K
    (tests/golden/c2_oracle.npz) and pair 37 the oracle run here: relative cost
    mixed <= 1e-6, FP64 <= 1e-9; potentials mixed <= 1e-6, FP64 <= 1e-8."""
    s, K, eta = 28, 250, 0.1
    n = s * s
    print("case full-size batch 64 x %dx%d %s switch %d" % (n, n, precision, hvp_switch), flush=True)
    pairs = [W.blob_pair(i, s=s) for i in range(64)]
    probs = [dict(kind=P.COST_GRID, m=n, n=n, grid_s=s, a=_t(p["a"]), b=_t(p["b"])) for p in pairs]
    outs = [dict(alpha=torch.empty(n, dtype=torch.float64, device=DEV),
                 beta=torch.empty(n, dtype=torch.float64, device=DEV)) for _ in pairs]
    hess = dict(hvp=2, hvp_switch=hvp_switch) if hvp_switch > 0 else dict(hvp=0)
    prm = P.params(eta=eta, max_outer=K, precision=P.MIXED if precision == "mixed" else P.FP64, streams=4, **hess)
    rc, rs = ctx.solve_batch_device(probs, prm, outs, stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert rc == 0
    for q, r in enumerate(rs):
        assert r["status"] == 0 and r["resid"] <= 1e-10, (q, r["status"], r["resid"])
        al, be = outs[q]["alpha"].cpu().numpy(), outs[q]["beta"].cpu().numpy()
        assert abs(pairs[q]["a"] @ al - pairs[q]["b"] @ be) <= 1e-12
    import os

    bar = 1e-6 if precision == "mixed" else 1e-9
    pbar = 1e-6 if precision == "mixed" else 1e-8
    f = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_oracle.npz"))
    assert int(f["s"]) == s and float(f["eta"]) == eta and int(f["K"]) == K
    ref = {q: (f["cost"][q], f["alpha_%d" % q], f["beta_%d" % q]) for q in range(len(f["cost"]))}
    o = oracle.pins(oracle.cost_grid(s), pairs[37]["a"], pairs[37]["b"], want_plan=False, eta=eta, K=K)
    ref[37] = (o["cost"], o["alpha"], o["beta"])
    for q, (c, al, be) in ref.items():
        rel = abs(rs[q]["cost"] - c) / c
        assert rel <= bar, (q, rel)
        # gauge-fixed potentials, elementwise
        assert np.abs(outs[q]["alpha"].cpu().numpy() - al).max() <= pbar, q
        assert np.abs(outs[q]["beta"].cpu().numpy() - be).max() <= pbar, q


@pytest.mark.parametrize("m,n", [(150, 97), (2000, 30)])
def test_dense_cost_scaled_by_its_maximum(ctx, m, n):
    """cost_scale <= 0 on the device path: the library divides C by its own
    maximum (a reduction over whole rows; 150 rows leave blocks of the grid
    idle, 2000 rows give each block several).  Parity with the oracle run on
    C / max C."""
    print("case dense 1/max scale %dx%d" % (m, n), flush=True)
    C, a, b = _rand(m, n, 4000 + m)
    C = 3.7 * C
    Cs = C / C.max()
    g = gpu_solve(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b, cost_scale=0.0), P.params(eta=0.05, max_outer=4))
    g["_C"] = Cs
    o = oracle.pins(Cs, a, b, eta=0.05, K=4)
    check_parity(g, o, a, b)


@pytest.mark.parametrize("m,n,d", [(77, 50, 2), (45, 130, 8), (100, 64, 32), (33, 17, 3)])
def test_points_cost_on_matrix_cores_parity(ctx, m, n, d):
    """Point-cloud cost built with the FP64 matrix cores (ragged 32x32 tiles,
    d not a multiple of 4): parity with the oracle's direct sum of squares."""
    print("case points m=%d n=%d d=%d" % (m, n, d), flush=True)
    g = np.random.default_rng(900 + d)
    x, y = g.uniform(0, 1, (m, d)), g.uniform(0, 1, (n, d))
    a, b = g.uniform(0.2, 1, m), g.uniform(0.2, 1, n)
    a, b = a / a.sum(), b / b.sum()
    C = oracle.cost_points(x, y)
    eta, K = 0.02, 6
    prm = P.params(eta=eta, max_outer=K)
    gr = gpu_solve(ctx, dict(kind=P.COST_POINTS, x=x, y=y, a=a, b=b), prm)
    gr["_C"] = C
    o = oracle.pins(C, a, b, eta=eta, K=K)
    check_parity(gr, o, a, b)


def test_uneven_batch_of_point_clouds(ctx):
    """256 uneven point-cloud instances (m, n log-uniform in [64, 2048], d cycling
    over 2, 8, 32, Dirichlet marginals, eta = 1e-2, K = 20, mixed precision) in one
    call: every instance converges (status OK, residual <= 1e-10, gauge); the
    three smallest match the oracle (<= 1e-6); two instances solved alone give
    bitwise the batched potentials."""
    print("case uneven batch 256 point clouds", flush=True)
    insts = [W.batch_instance(i) for i in range(256)]
    probs = [dict(kind=P.COST_POINTS, m=x["x"].shape[0], n=x["y"].shape[0], d=x["d"], x=_t(x["x"]), y=_t(x["y"]),
                  a=_t(x["a"]), b=_t(x["b"])) for x in insts]
    outs = [dict(alpha=torch.empty(p["m"], dtype=torch.float64, device=DEV),
                 beta=torch.empty(p["n"], dtype=torch.float64, device=DEV)) for p in probs]
    eta, K = 1e-2, 20
    prm = P.params(eta=eta, max_outer=K, precision=P.MIXED)
    st = torch.cuda.current_stream().cuda_stream
    rc, rs = ctx.solve_batch_device(probs, prm, outs, stream=st)
    torch.cuda.synchronize()
    assert rc == 0
    for q, r in enumerate(rs):
        assert r["status"] == 0 and r["resid"] <= 1e-10, (q, r["status"], r["resid"])
        al, be = outs[q]["alpha"].cpu().numpy(), outs[q]["beta"].cpu().numpy()
        assert abs(insts[q]["a"] @ al - insts[q]["b"] @ be) <= 1e-12
    small = sorted(range(256), key=lambda q: insts[q]["x"].shape[0] * insts[q]["y"].shape[0])[:3]
    for q in small:
        C = oracle.cost_points(insts[q]["x"], insts[q]["y"])
        o = oracle.pins(C, insts[q]["a"], insts[q]["b"], want_plan=False, eta=eta, K=K)
        assert abs(rs[q]["cost"] - o["cost"]) / o["cost"] <= 1e-6, q
    for q in (small[0], 101):
        out1 = dict(alpha=torch.empty(probs[q]["m"], dtype=torch.float64, device=DEV),
                    beta=torch.empty(probs[q]["n"], dtype=torch.float64, device=DEV))
        _, r1 = ctx.solve_device(probs[q], prm, out1, stream=st)
        torch.cuda.synchronize()
        assert torch.equal(out1["alpha"], outs[q]["alpha"]) and torch.equal(out1["beta"], outs[q]["beta"]), q
        assert r1["cost"] == rs[q]["cost"]


@pytest.mark.parametrize("cls", ["white", "gmm", "cauchy"])
def test_large_grid_properties(ctx, cls):
    """64x64 grids (m = n = 4096, cost streamed), eta = 1e-3, K = 10, mixed
    precision, one pair per histogram class.  The oracle is far too slow at this
    size, so the checks are properties that hold at any size: status and
    marginal residual; the gauge; the returned plan equals
    exp((alpha_i + beta_j - C_ij)/eps) on sampled entries (C from the grid
    formula on the host); cost = <C, X> recomputed on the host; and the gap
    identity cost - <a,alpha> - <b,beta> = eps*H(X) + <alpha, Xe - a> + <beta, X^T e - b>."""
    s, eta, K = 64, 1e-3, 10
    n = s * s
    print("case grid64 %s" % cls, flush=True)
    pr = W.grid_pair(cls, 0, s=s)
    a, b = pr["a"], pr["b"]
    prm = P.params(eta=eta, max_outer=K, precision=P.MIXED)
    g = gpu_solve(ctx, dict(kind=P.COST_GRID, grid_s=s, a=a, b=b), prm)
    assert g["rc"] == 0 and g["resid"] <= 1e-10
    al, be, X, eps = g["alpha"], g["beta"], g["X"], g["eps"]
    assert abs(eps - eta / K) <= 1e-15
    assert abs(a @ al - b @ be) <= 1e-12
    coords = np.array([(p // s, p % s) for p in range(n)], dtype=np.float64)
    scale = 1.0 / (2.0 * (s - 1) ** 2)
    d0 = coords[:, 0][:, None] - coords[:, 0][None, :]
    d1 = coords[:, 1][:, None] - coords[:, 1][None, :]
    C = (d0 * d0 + d1 * d1) * scale
    # the plan form over all 16.8 M entries (evaluated with torch in float64 on the device)
    Ct, Xt = _t(C), _t(X)
    Xp = torch.exp((_t(al)[:, None] + _t(be)[None, :] - Ct) / eps)
    assert bool(torch.all(torch.abs(Xp - Xt) <= 1e-12 + 1e-11 * Xt))
    del Ct, Xt, Xp
    cost = float((C * X).sum())
    assert abs(cost - g["cost"]) <= 1e-12 * cost
    r, c = X.sum(1), X.sum(0)
    assert np.abs(r - a).sum() + np.abs(c - b).sum() <= 1e-10
    pos = X > 0
    H = -float((X[pos] * np.log(X[pos])).sum())
    gap = cost - (a @ al + b @ be)
    rhs = eps * H + al @ (r - a) + be @ (c - b)
    assert abs(gap - rhs) <= 1e-9 * abs(cost)


def test_gpu_matches_stored_oracle_fixtures(ctx):
    """The HIP path (FP64) against the stored oracle outputs of
    tests/golden/oracle_fixtures.json: the cost at the FP64 parity bar, the
    residual, and the gauge-fixed potentials to 1e-8, except for the
    random-assignment fixture.  Near an assignment (that case at eps = eta / K
    = 5e-4) the plan is almost a permutation sigma, and moving alpha_i up and
    beta_sigma(i) down by the same amount changes only its tiny
    off-permutation entries, so the dual's Hessian (the plan's entries over
    eta) barely sees that direction and the method fixes it only loosely: the
    oracle itself, run with other valid inner settings (CG tolerance 1e-9 or
    1e-3, warm-up cap 5), moves the potentials by up to 2e-3 while alpha_i +
    beta_sigma(i) and the cost stay within 2e-16.  There the check is on what
    the plan determines: alpha_i + beta_sigma(i) to 1e-8 and the dual value
    <a, alpha> + <b, beta> to 1e-9 relative."""
    import json
    import os
    import sys

    gdir = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, gdir)
    import make_oracle_fixtures as G

    ref = json.load(open(os.path.join(gdir, "oracle_fixtures.json")))
    for name, C, a, b, eta, K in G.cases():
        print("case fixture %s" % name, flush=True)
        g = gpu_solve(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b), P.params(eta=eta, max_outer=K),
                      want_plan=False)
        f = ref[name]
        assert g["rc"] == 0 and g["resid"] <= 1e-10, (name, g["resid"])
        assert abs(g["cost"] - f["cost"]) <= 1e-9 * abs(f["cost"]), name
        fa, fb = np.array(f["alpha"]), np.array(f["beta"])
        if name.startswith("assignment"):
            sig = np.argmax(fa[:, None] + fb[None, :] - C, axis=1)  # the plan's dominant entry per row
            assert len(set(sig.tolist())) == len(sig), name  # a permutation
            assert np.abs((g["alpha"] + g["beta"][sig]) - (fa + fb[sig])).max() <= 1e-8, name
            dual, fdual = a @ g["alpha"] + b @ g["beta"], a @ fa + b @ fb
            assert abs(dual - fdual) <= 1e-9 * abs(fdual), name
        else:
            assert np.abs(g["alpha"] - fa).max() <= 1e-8, name
            assert np.abs(g["beta"] - fb).max() <= 1e-8, name


def test_c3_grids_match_stored_oracle(ctx):
    """64x64 grids (m = n = 4096, streamed cost), eta = 1e-3, K = 10, one pair
    per histogram class, against the oracle's outputs stored in
    tests/golden/c3_oracle.npz (written by make_c3_fixtures.py from oracle/
    only): FP64 path cost <= 1e-9 relative and potentials <= 1e-8; mixed path
    cost <= 1e-6 relative and potentials <= 1e-6."""
    import os

    f = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_oracle.npz"))
    s, eta, K = int(f["s"]), float(f["eta"]), int(f["K"])
    for cls in ("white", "gmm", "cauchy"):
        pr = W.grid_pair(cls, 0, s=s)
        cost_o = f[cls + "_scalars"][0]
        for prec, cbar, pbar in ((P.FP64, 1e-9, 1e-8), (P.MIXED, 1e-6, 1e-6)):
            print("case c3 fixture %s precision %d" % (cls, prec), flush=True)
            g = gpu_solve(ctx, dict(kind=P.COST_GRID, grid_s=s, a=pr["a"], b=pr["b"]),
                          P.params(eta=eta, max_outer=K, precision=prec), want_plan=False)
            assert g["rc"] == 0 and g["resid"] <= 1e-10, (cls, prec, g["resid"])
            assert abs(g["cost"] - cost_o) <= cbar * cost_o, (cls, prec, g["cost"], cost_o)
            assert np.abs(g["alpha"] - f[cls + "_alpha"]).max() <= pbar, (cls, prec)
            assert np.abs(g["beta"] - f[cls + "_beta"]).max() <= pbar, (cls, prec)


@pytest.mark.parametrize("budget", [64.0, 4.0])
@pytest.mark.parametrize("case", ["dense", "grid"])
@pytest.mark.parametrize("t2", [1, 2, 3])
def test_one_newton_step_parity(ctx, case, t2, budget):
    """Sparsify, CG and the line search pinned one Newton step at a time: K = 1,
    exactly three warm-up iterations (warm_tol = 0), exactly t2 Newton steps
    (marginal tolerance 0, so that no convergence decision sits at a tolerance
    boundary), and both sides' CG run to a relative residual of 1e-13, so that
    both solve the same sparsified Newton system (the GPU on its Schur
    complement, the oracle on the full system) to far below the tolerances.  The
    kept count of the last Sparsify, the fallback count, the Newton step count
    and the gauge-fixed potentials (<= 1e-9) must then match the oracle's; both
    report status 1 (the Newton cap).  Budget 64 keeps nearly every entry (all of
    them on the 8x8 grid), budget 4 a sparse level (about 35 of 4096 entries on
    the grid, 170 of 1710 on the dense instance)."""
    if case == "dense":
        C, a, b = _rand(45, 38, 314)
        prob = dict(kind=P.COST_DENSE, C=C, a=a, b=b)
        eta = 0.05
    else:
        pr = W.blob_pair(11, s=8)
        C, a, b = oracle.cost_grid(8), pr["a"], pr["b"]
        prob = dict(kind=P.COST_GRID, grid_s=8, a=a, b=b)
        eta = 0.1
    print("case one-newton %s t2=%d budget %g" % (case, t2, budget), flush=True)
    kw = dict(eta=eta, warm_tol=0.0, cg_rtol=1e-13, inner_tol=0.0, final_tol=0.0, budget=budget)
    prm = P.params(max_outer=1, max_sinkhorn=3, max_newton=t2, cg_max_iter=4000, **kw)
    g = gpu_solve(ctx, prob, prm, want_plan=False)
    o = oracle.pins(C, a, b, want_plan=False, K=1, T1=3, T2=t2, cg_max=4000, **kw)
    assert g["rc"] == o["status"] == 1, (g["rc"], o["status"])
    assert g["sinkhorn_iters"] == o["sinkhorn"] == 3
    assert g["newton_iters"] == o["newton"], (g["newton_iters"], o["newton"])
    assert g["nnz_last"] == o["nnz_last"], (g["nnz_last"], o["nnz_last"])
    assert g["fallbacks"] == o["fallbacks"], (g["fallbacks"], o["fallbacks"])
    assert abs(g["cost"] - o["cost"]) <= 1e-9 * o["cost"]
    assert np.abs(g["alpha"] - o["alpha"]).max() <= 1e-9
    assert np.abs(g["beta"] - o["beta"]).max() <= 1e-9


def test_sparsify_at_the_papers_retained_fraction(ctx):
    """The numerical appendix's own Sparsify setting: at most (3n - 1)/(2n^2) of
    the n x n coupling block kept, i.e. a budget of (3n - 1)/2 entries, which in
    units of m + n - 1 is (3n - 1)/(2(2n - 1)) (about 0.75).  On a 40 x 40 dense
    instance at eta = 0.05, K = 8 the kept sets are then so small that every
    subproblem ends at the Newton cap on both sides (391 Newton steps against 19
    with the default budget of 64 spanning trees, the reason for that default).
    The GPU must still follow the oracle step for step: the same status, Newton
    and fallback counts, the same kept count in the last Newton step (within the
    budget), and cost and potentials at parity."""
    print("case sparsify paper fraction", flush=True)
    n = 40
    C, a, b = _rand(n, n, 11)
    eta, K = 0.05, 8
    budget = (3 * n - 1) / (2 * (2 * n - 1))
    g = gpu_solve(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b), P.params(eta=eta, max_outer=K, budget=budget))
    o = oracle.pins(C, a, b, eta=eta, K=K, budget=budget)
    assert g["rc"] == o["status"] == 1, (g["rc"], o["status"])
    assert g["newton_iters"] == o["newton"], (g["newton_iters"], o["newton"])
    assert g["fallbacks"] == o["fallbacks"], (g["fallbacks"], o["fallbacks"])
    assert g["nnz_last"] == o["nnz_last"] <= (3 * n - 1) // 2, (g["nnz_last"], o["nnz_last"])
    assert abs(g["cost"] - o["cost"]) <= 1e-9 * o["cost"], (g["cost"], o["cost"])
    # the last subproblem is far from its tolerance too (residual about 4e-4), the same on both sides
    assert abs(g["resid"] - o["resid"]) <= 1e-8 * o["resid"], (g["resid"], o["resid"])
    assert np.abs(g["alpha"] - o["alpha"]).max() <= 1e-8
    assert np.abs(g["beta"] - o["beta"]).max() <= 1e-8


def test_sparsify_no_level_within_budget(ctx):
    """One Sparsify level (rho = 1e-3) and a budget of three spanning trees
    (3 (m + n - 1) entries): whenever the level keeps more, no entry is kept and
    the Newton system is its diagonal, on both sides.  On this instance the first
    three subproblems keep nothing (and hit the Newton cap), the later ones fit.
    Parity with the oracle, and the same kept count in the last Newton step."""
    print("case sparsify no level", flush=True)
    C, a, b = _rand(60, 50, 2718)
    eta, K = 0.05, 6
    kw = dict(rho_levels=1, budget=3.0, rho=1e-3)
    g = gpu_solve(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b), P.params(eta=eta, max_outer=K, **kw))
    g["_C"] = C
    o = oracle.pins(C, a, b, eta=eta, K=K, **kw)
    assert o["flags"] & 2 and g["flags"] & 2  # earlier subproblems hit the cap on both sides
    check_parity(g, o, a, b)
    assert g["nnz_last"] == o["nnz_last"], (g["nnz_last"], o["nnz_last"])


def test_cg_storage_forms_against_oracle(ctx):
    """The one-block CG's two storage forms of S against the oracle: the
    jagged-diagonal form (rows cut into pieces of up to 16 quads, one lane per
    piece), and the row-contiguous form it falls back to when a half has more
    pieces than the CG's LDS array of piece sums holds (2048 for m + n <= 1024,
    4096 up to 2048, else 6144).  A 100x100 instance at eta = 0.01 keeps a sparse
    set (jagged-diagonal); a 600x600 instance at eta = 0.5 with a budget of 512
    spanning trees keeps all 360 000 entries: per half 600 rows of 150 quads,
    ten pieces each, 6000 > 4096 (row-contiguous).  Each form must have done the
    instance's CG work."""
    for m, eta, K, budget, cls in ((100, 0.01, 10, 64.0, "pcg"), (600, 0.5, 3, 512.0, "pcg_rows")):
        print("case cg storage %s m=n=%d" % (cls, m), flush=True)
        C, a, b = _rand(m, m, 4242 + m)
        g = gpu_solve(ctx, dict(kind=P.COST_DENSE, C=C, a=a, b=b), P.params(eta=eta, max_outer=K, budget=budget))
        g["_C"] = C
        o = oracle.pins(C, a, b, eta=eta, K=K, budget=budget)
        check_parity(g, o, a, b)
        other = "pcg_rows" if cls == "pcg" else "pcg"
        assert g["kern_work"][cls] > 0 and g["kern_work"][other] == 0, g["kern_work"]
        if cls == "pcg_rows":
            assert g["nnz_last"] == m * m


def test_mixed_cg_kinds_batch_equals_alone(ctx):
    """The CG an instance takes (one block for m + n <= 4096, else the wide CG
    with 16-bit or 32-bit indices) is its own: a batch that mixes all three
    kinds gives every instance bitwise the result it gets alone.  Grids 32x32
    (one block) with a 64x64 grid (wide), and dense instances 30x20 (one block),
    4100x40 (wide, 16-bit) and 70000x3 (wide, 32-bit), each batch on a
    non-default caller stream."""
    st = torch.cuda.Stream()
    grids = [(32, 1), (64, 2), (32, 3)]
    gp = [W.grid_pair("gmm", i, s=s) for s, i in grids]
    gprobs = [dict(kind=P.COST_GRID, m=s * s, n=s * s, grid_s=s, a=_t(p["a"]), b=_t(p["b"]))
              for (s, _), p in zip(grids, gp)]
    dense = [(30, 20), (4100, 40), (70000, 3)]
    dprobs = []
    for q, (m, n) in enumerate(dense):
        C, a, b = _rand(m, n, 7000 + q)
        dprobs.append(dict(kind=P.COST_DENSE, m=m, n=n, C=_t(C), a=_t(a), b=_t(b), cost_scale=1.0))
    for name, probs, prm in (("grids", gprobs, P.params(eta=1e-2, max_outer=3)),
                             ("dense", dprobs, P.params(eta=0.05, max_outer=3))):
        print("case mixed cg kinds %s" % name, flush=True)
        outs = [dict(alpha=torch.empty(p["m"], dtype=torch.float64, device=DEV),
                     beta=torch.empty(p["n"], dtype=torch.float64, device=DEV)) for p in probs]
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            rc, rs = ctx.solve_batch_device(probs, prm, outs, stream=st.cuda_stream)
        st.synchronize()
        assert rc >= 0
        for q, pr in enumerate(probs):
            o1 = dict(alpha=torch.empty(pr["m"], dtype=torch.float64, device=DEV),
                      beta=torch.empty(pr["n"], dtype=torch.float64, device=DEV))
            _, r1 = ctx.solve_device(pr, prm, o1, stream=st.cuda_stream)
            st.synchronize()
            assert r1["cost"] == rs[q]["cost"], (name, q)
            assert torch.equal(o1["alpha"], outs[q]["alpha"]) and torch.equal(o1["beta"], outs[q]["beta"]), (name, q)
            assert r1["cg_iters"] == rs[q]["cg_iters"] and r1["newton_iters"] == rs[q]["newton_iters"], (name, q)


def test_device_marginals_checked_on_the_solve_stream(ctx):
    """Device marginals are validated by the set-up kernel on the solve's own
    stream: marginals written by a kernel on a non-default caller stream just
    before the call are seen (valid ones accepted), and invalid ones (an entry
    <= 0, a sum off by 1e-6) are rejected with PINS_EINVAL, nothing written."""
    print("case device marginals", flush=True)
    C, a, b = _rand(40, 30, 99)
    st = torch.cuda.Stream()
    prm = P.params(eta=0.05, max_outer=3)
    with torch.cuda.stream(st):
        Ct = _t(C)
        ad = torch.zeros(40, dtype=torch.float64, device=DEV)
        bd = torch.zeros(30, dtype=torch.float64, device=DEV)
        torch.cuda.synchronize()
        # written on the caller stream right before the solve on that stream
        ad.copy_(_t(a), non_blocking=True)
        bd.copy_(_t(b), non_blocking=True)
        out = dict(alpha=torch.full((40,), 7.0, dtype=torch.float64, device=DEV),
                   beta=torch.full((30,), 7.0, dtype=torch.float64, device=DEV))
        rc, r = ctx.solve_device(dict(kind=P.COST_DENSE, m=40, n=30, C=Ct, a=ad, b=bd, cost_scale=1.0), prm, out,
                                 stream=st.cuda_stream)
    st.synchronize()
    assert rc == 0 and r["resid"] <= 1e-10
    for bad in ("neg", "sum"):
        av = a.copy()
        if bad == "neg":
            av[3] = -av[3]
        else:
            av[0] += 1e-6
        out = dict(alpha=torch.full((40,), 7.0, dtype=torch.float64, device=DEV),
                   beta=torch.full((30,), 7.0, dtype=torch.float64, device=DEV))
        with pytest.raises(P.PinsError) as e:
            ctx.solve_device(dict(kind=P.COST_DENSE, m=40, n=30, C=Ct, a=_t(av), b=bd, cost_scale=1.0), prm, out,
                             stream=st.cuda_stream)
        assert e.value.code == -1 and "a must" in str(e.value)
        st.synchronize()
        assert bool(torch.all(out["alpha"] == 7.0)) and bool(torch.all(out["beta"] == 7.0))



def test_headline_pairs_reach_the_lp_at_the_calibrated_k(ctx):
    """The 28x28 image-histogram pairs at eta = 0.1 (mixed precision, the
    headline's arithmetic): after 2000 outer iterations the cost of each of
    pairs 0..3 is within 1e-6 of the LP optimum (HiGHS through oracle/lp.py,
    stored in tests/golden/c2_lp.json by make_c2_lp.py; measured at most 7e-9);
    after 250 it is not (1.7e-3 to 2.9e-3), so the bench reports the batch at
    both."""
    import json
    import os

    lp = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_lp.json")))["lp"]
    for i in (0, 1, 2, 3):
        print("case c2 pair %d vs lp" % i, flush=True)
        pr = W.blob_pair(i, s=28)
        prob = dict(kind=P.COST_GRID, grid_s=28, a=pr["a"], b=pr["b"])
        ot = lp[str(i)]
        g = gpu_solve(ctx, prob, P.params(eta=0.1, max_outer=2000, precision=P.MIXED), want_plan=False)
        assert g["rc"] == 0 and abs(g["cost"] - ot) / ot <= 1e-6, (i, g["cost"], ot)
        g = gpu_solve(ctx, prob, P.params(eta=0.1, max_outer=250, precision=P.MIXED), want_plan=False)
        assert g["rc"] == 0 and abs(g["cost"] - ot) / ot > 1e-4, (i, g["cost"], ot)
