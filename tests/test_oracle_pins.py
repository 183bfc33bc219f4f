"""Pins of the FP64 oracle against facts it does not compute itself.

P1  permutation brute force (Birkhoff vertices)        -> LP value
P2  basic-solution enumeration                         -> LP value, arbitrary marginals
P3  1-D monotone (north-west corner) coupling          -> LP value
P4  scipy HiGHS on the 100x100 plane instance           -> LP value at calibrated K
P5  2x2 closed form of the entropic plan at eta/K       -> whole finite-K output
P6  separable cost                                       -> plan a b^T
P7  finite-K output = entropic plan at eps = eta/K (matrix-scaling Sinkhorn written here)
P8  KKT: marginals, dual feasibility, gap identity, gap -> 0
P9  descent of <C, X^k> over outer iterations (Thm. 1)
P10 sparsity of the limit plan (Thm. 2: at most 2n-1 coupling entries)
P11 metamorphic relations
P12 gauge and the potential form of the plan
plus exactness of the single half-sweeps and the cost constructions.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import lp


def _rand_problem(m, n, seed, kind="unif"):
    g = np.random.default_rng(seed)
    C = g.uniform(0, 1, (m, n))
    a = g.uniform(0.2, 1.0, m)
    b = g.uniform(0.2, 1.0, n)
    return C, a / a.sum(), b / b.sum()


# --------------------------------------------------------------------------- cost

def test_cost_points_matches_generator(oracle_mod):
    inst = W.points_instance(3, m=17, n=11, d=3)
    C1 = oracle_mod.cost_points(inst["x"], inst["y"])
    C2 = W.sqeuclid_dense(inst["x"], inst["y"])
    assert np.allclose(C1, C2, rtol=1e-14, atol=1e-15)
    assert C1.max() == pytest.approx(1.0, abs=1e-15)
    # explicit scale: no normalisation
    C3 = oracle_mod.cost_points(inst["x"], inst["y"], scale=1.0)
    assert np.allclose(C3, W.sqeuclid_dense(inst["x"], inst["y"], normalise=False), rtol=1e-14)


def test_cost_grid_matches_generator(oracle_mod):
    for s in (2, 5, 28):
        C = oracle_mod.cost_grid(s)
        assert np.allclose(C, W.grid_dense(s), rtol=0, atol=1e-15)
        assert C.max() == pytest.approx(1.0)  # max squared distance is 2(s-1)^2
        i = s * (s - 1) + 2 if s > 2 else 1
        j = 1
        dr, dc = i // s - j // s, i % s - j % s
        assert C[i, j] == pytest.approx((dr * dr + dc * dc) / (2.0 * (s - 1) ** 2))


# --------------------------------------------------------------------------- half sweeps

def test_row_update_matches_row_marginals(oracle_mod):
    """After the f-update of Alg. 2 the row sums of Xt(f, g) equal a exactly (block ascent)."""
    C, a, b = _rand_problem(7, 5, 1)
    eta = 0.07
    g = np.random.default_rng(2)
    f0, g0 = g.normal(size=7) * 0.1, g.normal(size=5) * 0.1
    f1, err = oracle_mod.sinkhorn_row(C, a, eta, f0, g0)
    X0 = np.exp((f0[:, None] + g0[None, :] - C - eta) / eta)
    assert err == pytest.approx(np.abs(X0.sum(1) - a).sum(), rel=1e-12)
    X1 = np.exp((f1[:, None] + g0[None, :] - C - eta) / eta)
    assert np.allclose(X1.sum(1), a, rtol=1e-13)
    g1 = oracle_mod.sinkhorn_col(C, b, eta, f1, g0)
    X2 = np.exp((f1[:, None] + g1[None, :] - C - eta) / eta)
    assert np.allclose(X2.sum(0), b, rtol=1e-13)
    Xr = oracle_mod.recover(C, eta, f1, g1)
    assert np.allclose(Xr, X2, rtol=1e-14)


# --------------------------------------------------------------------------- LP pins

@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_P1_bruteforce_permutations(oracle_mod, n):
    for inst in range(2):
        d = W.assignment_instance(inst, n)
        ot = lp.lp_bruteforce_perm(d["C"])
        r = oracle_mod.pins(d["C"], d["a"], d["b"], eta=1e-2, K=60)
        assert r["status"] == 0
        assert abs(r["cost"] - ot) / ot <= 1e-10
        # weak duality and feasibility: dual <= OT* <= cost (+ residual slack)
        assert r["dual"] <= ot + 1e-12
        assert r["cost"] >= ot - r["resid"] * d["C"].max() - 1e-15


def test_P2_vertex_enumeration_arbitrary_marginals(oracle_mod):
    for seed in range(3):
        C, a, b = _rand_problem(3, 4, 10 + seed)
        ot = lp.lp_vertex_enum(C, a, b)
        ot_h, _ = lp.lp_highs(C, a, b)
        assert ot == pytest.approx(ot_h, rel=1e-9)
        r = oracle_mod.pins(C, a, b, eta=1e-2, K=200)
        assert r["status"] == 0
        assert abs(r["cost"] - ot) / ot <= 1e-9


def test_P3_monotone_coupling_1d(oracle_mod):
    g = np.random.default_rng(7)
    for m, n, eta, K, tol in ((12, 9, 1e-3, 100, 1e-12), (40, 30, 1e-2, 3000, 5e-6)):
        x = g.uniform(0, 1, m)
        y = g.uniform(0, 1, n)
        a = g.uniform(0.5, 1, m)
        b = g.uniform(0.5, 1, n)
        a /= a.sum()
        b /= b.sum()
        C = (x[:, None] - y[None, :]) ** 2
        ot = lp.lp_monotone_1d(x, y, a, b)
        ot_h, _ = lp.lp_highs(C, a, b)
        assert ot == pytest.approx(ot_h, rel=1e-8)
        s = C.max()
        r = oracle_mod.pins(C / s, a, b, eta=eta, K=K, want_plan=False)
        assert r["status"] == 0
        assert abs(r["cost"] * s - ot) / ot <= tol


def test_P4_highs_plane_instance_calibrated_K(oracle_mod):
    """Plain 100x100 plane instance: K = 2000 at eta = 1e-2 reaches <= 1e-8 vs the LP."""
    inst = W.points_instance(0)
    C = oracle_mod.cost_points(inst["x"], inst["y"])
    ot, _ = lp.lp_highs(C, inst["a"], inst["b"])
    r = oracle_mod.pins(C, inst["a"], inst["b"], eta=1e-2, K=2000, want_plan=False)
    assert r["status"] == 0
    assert abs(r["cost"] - ot) / ot <= 1e-8
    assert r["resid"] <= 1e-12


# --------------------------------------------------------------------------- finite-K output

@pytest.mark.parametrize("K", [1, 3, 8])
def test_P5_closed_form_2x2(oracle_mod, K):
    C = np.array([[0.1, 0.7], [0.4, 0.05]])
    a = np.array([0.3, 0.7])
    b = np.array([0.55, 0.45])
    eta = 0.4
    r = oracle_mod.pins(C, a, b, eta=eta, K=K)
    Xcf = lp.entropic_2x2(C, a, b, eta / K)
    assert np.abs(r["X"] - Xcf).max() <= 1e-13
    assert r["eps"] == pytest.approx(eta / K)


def test_P6_separable_cost(oracle_mod):
    g = np.random.default_rng(3)
    u, v = g.uniform(0, 1, 6), g.uniform(0, 1, 9)
    a = g.uniform(0.1, 1, 6)
    b = g.uniform(0.1, 1, 9)
    a /= a.sum()
    b /= b.sum()
    C = u[:, None] + v[None, :]
    for K in (1, 5):
        r = oracle_mod.pins(C, a, b, eta=0.05, K=K)
        assert np.abs(r["X"] - np.outer(a, b)).max() <= 1e-14
        assert r["cost"] == pytest.approx(u @ a + v @ b, rel=1e-13)


def _scaling_sinkhorn(C, a, b, eps, iters=20000):
    """Textbook matrix-scaling Sinkhorn (u = a/(Kv), v = b/(K^T u)), written here."""
    Kmat = np.exp(-C / eps)
    v = np.ones(len(b))
    for _ in range(iters):
        u = a / (Kmat @ v)
        v = b / (Kmat.T @ u)
    return u[:, None] * Kmat * v[None, :]


def test_P7_entropic_plan_at_eta_over_K(oracle_mod):
    C, a, b = _rand_problem(9, 6, 5)
    eta, K = 0.1, 6
    r = oracle_mod.pins(C, a, b, eta=eta, K=K)
    Xs = _scaling_sinkhorn(C, a, b, eta / K)
    assert np.abs(r["X"] - Xs).sum() <= 1e-12
    # and the oracle's own Alg. 1 at the same eps
    s = oracle_mod.sinkhorn(C, a, b, eta / K, tol=1e-15)
    assert np.abs(r["X"] - s["X"]).sum() <= 1e-12


def test_P7_independent_of_inner_path(oracle_mod):
    """Changing warm-up length, tolerances, CG accuracy or Sparsify leaves X^K unchanged."""
    inst = W.points_instance(1, m=30, n=25)
    C = oracle_mod.cost_points(inst["x"], inst["y"])
    base = oracle_mod.pins(C, inst["a"], inst["b"], eta=1e-2, K=40)
    for kw in (dict(T1=3, warm_tol=0.0), dict(warm_tol=1e-8), dict(cg_rtol=1e-3), dict(rho=1e-4, budget=2.0),
               dict(inner_tol=1e-6)):
        r = oracle_mod.pins(C, inst["a"], inst["b"], eta=1e-2, K=40, **kw)
        assert r["status"] == 0, kw
        assert np.abs(r["X"] - base["X"]).sum() <= 1e-10, kw
        assert abs(r["cost"] - base["cost"]) <= 1e-12, kw


# --------------------------------------------------------------------------- certificates

def test_P8_kkt_and_gap(oracle_mod):
    inst = W.points_instance(2, m=40, n=35)
    C = oracle_mod.cost_points(inst["x"], inst["y"])
    a, b = inst["a"], inst["b"]
    prev_gap = math.inf
    for K in (5, 20, 80):
        r = oracle_mod.pins(C, a, b, eta=1e-2, K=K)
        X, al, be, eps = r["X"], r["alpha"], r["beta"], r["eps"]
        assert r["status"] == 0
        assert np.abs(X.sum(1) - a).sum() + np.abs(X.sum(0) - b).sum() <= 1e-12
        assert r["resid"] <= 1e-12
        # dual feasibility: X_ij <= 1  <=>  alpha_i + beta_j <= C_ij
        assert (al[:, None] + be[None, :] - C).max() <= 1e-14
        # gap identity: <C,X> - <a,al> - <b,be> = eps*H(X) + <al, Xe-a> + <be, X^Te-b>
        H = -(X[X > 0] * np.log(X[X > 0])).sum()
        lhs = (C * X).sum() - a @ al - b @ be
        rhs = eps * H + al @ (X.sum(1) - a) + be @ (X.sum(0) - b)
        assert lhs == pytest.approx(rhs, rel=1e-10, abs=1e-15)
        assert r["gap"] == pytest.approx(lhs, rel=1e-10, abs=1e-15)
        assert r["gap"] < prev_gap
        prev_gap = r["gap"]


def test_P9_outer_descent(oracle_mod):
    inst = W.points_instance(4, m=50, n=45)
    C = oracle_mod.cost_points(inst["x"], inst["y"])
    r = oracle_mod.pins(C, inst["a"], inst["b"], eta=1e-2, K=60, trace=True, want_plan=False)
    cost = r["trace"][:, 5]
    eps = 1e-2 / np.arange(1, 61)
    bound = math.sqrt(2 * 50) * eps
    assert np.all(np.diff(cost) <= bound[1:])
    # tight inner solves: monotone non-increase
    assert np.all(np.diff(cost) <= 1e-12)


def test_P10_sparsity_of_limit(oracle_mod):
    """Near the LP vertex the significant entries number at most 2n-1 (Thm. 2, m = n)."""
    d = W.assignment_instance(5, 30)
    r = oracle_mod.pins(d["C"], d["a"], d["b"], eta=1e-2, K=300)
    X = r["X"]
    thr = 1e-3 * np.minimum(d["a"][:, None], d["b"][None, :])
    assert (X >= thr).sum() <= 2 * 30 - 1
    n = 30
    nnzH = 2 * n + 2 * (X >= thr).sum()
    assert nnzH / (2 * n) ** 2 <= (3 * n - 1) / (2 * n * n) + 1e-15
    assert r["nnz_last"] <= 64 * (2 * n - 1)


# --------------------------------------------------------------------------- metamorphic

def test_P11_metamorphic(oracle_mod):
    C, a, b = _rand_problem(12, 9, 21)
    eta, K = 0.03, 15
    base = oracle_mod.pins(C, a, b, eta=eta, K=K)
    X = base["X"]
    g = np.random.default_rng(0)
    pr, pc = g.permutation(12), g.permutation(9)
    r = oracle_mod.pins(C[pr][:, pc], a[pr], b[pc], eta=eta, K=K)
    assert np.abs(r["X"] - X[pr][:, pc]).sum() <= 1e-10
    r = oracle_mod.pins(C.T, b, a, eta=eta, K=K)
    assert np.abs(r["X"] - X.T).sum() <= 1e-10
    u, v = g.uniform(-1, 1, 12), g.uniform(-1, 1, 9)
    r = oracle_mod.pins(C + u[:, None] + v[None, :], a, b, eta=eta, K=K)
    assert np.abs(r["X"] - X).sum() <= 1e-10
    assert r["cost"] == pytest.approx(base["cost"] + u @ a + v @ b, abs=1e-11)
    r = oracle_mod.pins(3.0 * C, a, b, eta=3.0 * eta, K=K)
    assert np.abs(r["X"] - X).sum() <= 1e-10


def test_P12_gauge_and_potential_form(oracle_mod):
    C, a, b = _rand_problem(8, 11, 31)
    r = oracle_mod.pins(C, a, b, eta=0.05, K=9)
    al, be, eps = r["alpha"], r["beta"], r["eps"]
    assert a @ al == pytest.approx(b @ be, abs=1e-15)
    Xp = np.exp((al[:, None] + be[None, :] - C) / eps)
    assert np.abs(Xp - r["X"]).sum() <= 1e-12
    assert r["dual"] == pytest.approx(a @ al + b @ be, abs=1e-15)


def test_degenerate_sizes(oracle_mod):
    # one source: the only feasible plan is b^T
    b = np.array([0.2, 0.5, 0.3])
    r = oracle_mod.pins(np.array([[0.3, 0.1, 0.9]]), np.array([1.0]), b, eta=0.1, K=3)
    assert np.allclose(r["X"], b[None, :], atol=1e-15)
    r = oracle_mod.pins(np.array([[0.7]]), np.array([1.0]), np.array([1.0]), eta=0.1, K=2)
    assert r["X"][0, 0] == pytest.approx(1.0, abs=1e-15)
    assert r["cost"] == pytest.approx(0.7)


def test_oracle_reproduces_its_fixtures(oracle_mod):
    """tests/golden/oracle_fixtures.json (written by make_oracle_fixtures.py from
    the pinned oracle): the oracle still computes the same outputs."""
    import json
    import os
    import sys

    gdir = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, gdir)
    import make_oracle_fixtures as G

    ref = json.load(open(os.path.join(gdir, "oracle_fixtures.json")))
    for name, C, a, b, eta, K in G.cases():
        r = oracle_mod.pins(C, a, b, eta=eta, K=K, want_plan=False)
        f = ref[name]
        assert r["status"] == 0 and f["eta"] == eta and f["K"] == K, name
        assert abs(r["cost"] - f["cost"]) <= 1e-12 * abs(f["cost"]), name
        assert np.abs(r["alpha"] - np.array(f["alpha"])).max() <= 1e-11, name
        assert np.abs(r["beta"] - np.array(f["beta"])).max() <= 1e-11, name
