"""Planted mistakes: each mutant of the oracle source must fail at least one pin.

The mutation is applied to a temporary copy of ``oracle/pins_oracle.c`` on the
CPU; the real oracle is never modified.  This shows that the pins are tight
enough to catch a dropped term, a wrong sign, a wrong index or a transposed
operand anywhere on the path that decides the result.
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle import lp

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "pins_oracle.c")

MUTANTS = {
    "shift_sign": ("L[q] = (f[i] + g[j] - Ck[q] - eta) / eta;", "L[q] = (f[i] + g[j] + Ck[q] - eta) / eta;"),
    "alpha_drop_eta": ("alpha[i] = (U[i] + eta * loga[i]) / K - eta;", "alpha[i] = (U[i] + eta * loga[i]) / K;"),
    "row_wrong_marginal": ("f[i] = f[i] + eta * (log(a[i]) - l);", "f[i] = f[i] + eta * (log(a[0]) - l);"),
    "recover_drop_eta": ("X[(long)i * n + j] = exp((f[i] + g[j] - Ck[(long)i * n + j] - eta) / eta);",
                         "X[(long)i * n + j] = exp((f[i] + g[j] - Ck[(long)i * n + j]) / eta);"),
    "col_transposed": ("for (i = 0; i < m; ++i) z[i] = (f[i] + g[j] - Ck[(long)i * n + j] - eta) / eta;",
                       "for (i = 0; i < m; ++i) z[i] = (f[i] + g[j] - Ck[((long)j * m + i) % ((long)m * n)] - eta) / eta;"),
    "grid_index": ("dc = (double)(i % s - j % s);", "dc = (double)(i % s - j / s);"),
    "hessian_coupling": ("y[H->m + j] += H->v[k] * u[i];", "y[H->m + j] += H->v[k] * u[H->m + j];"),
    "armijo_sign": ("inc = al * (da + db) - eta * sm;", "inc = al * (da + db) + eta * sm;"),
    "gauge_sign": ("tg = 0.5 * (sb - sa);\n        for (i = 0; i < m; ++i) alpha[i] += tg;\n        for (j = 0; j < n; ++j) beta[j] -= tg;\n        for (i = 0; i < m; ++i) r[i] = 0.0;",
                   "tg = 0.5 * (sa - sb);\n        for (i = 0; i < m; ++i) alpha[i] += tg;\n        for (j = 0; j < n; ++j) beta[j] -= tg;\n        for (i = 0; i < m; ++i) r[i] = 0.0;"),
    "dual_sum_V": ("for (j = 0; j < n; ++j) V[j] += g[j];", "for (j = 0; j < n; ++j) V[j] += f[j % m];"),
    "sparsify_keep_small": ("if (Xt[(long)i * n + j] >= rl * mn_ab) {", "if (Xt[(long)i * n + j] <= rl * mn_ab) {"),
}


def _pin_suite(O):
    """Quick subset of the pins; returns the list of failed pin names."""
    failed = []

    def check(name, cond):
        if not cond:
            failed.append(name)

    C = np.array([[0.1, 0.7], [0.4, 0.05]])
    a2, b2 = np.array([0.3, 0.7]), np.array([0.55, 0.45])
    r = O.pins(C, a2, b2, eta=0.4, K=3)
    check("P5", np.isfinite(r["X"]).all() and np.abs(r["X"] - lp.entropic_2x2(C, a2, b2, 0.4 / 3)).max() <= 1e-13)

    d = W.assignment_instance(0, 5)
    ot = lp.lp_bruteforce_perm(d["C"])
    r = O.pins(d["C"], d["a"], d["b"], eta=1e-2, K=60)
    check("P1", r["status"] == 0 and abs(r["cost"] - ot) / ot <= 1e-10)

    g = np.random.default_rng(31)
    Cr = g.uniform(0, 1, (8, 11))
    a = g.uniform(0.2, 1, 8)
    b = g.uniform(0.2, 1, 11)
    a /= a.sum()
    b /= b.sum()
    r = O.pins(Cr, a, b, eta=0.05, K=9)
    ok = r["status"] == 0 and np.isfinite(r["X"]).all()
    if ok:
        Xp = np.exp((r["alpha"][:, None] + r["beta"][None, :] - Cr) / r["eps"])
        ok = abs(a @ r["alpha"] - b @ r["beta"]) <= 1e-15 and np.abs(Xp - r["X"]).sum() <= 1e-12
        ok = ok and np.abs(r["X"].sum(1) - a).sum() + np.abs(r["X"].sum(0) - b).sum() <= 1e-12
        ok = ok and r["newton"] <= 9 * 12 and r["fallbacks"] == 0
    check("P8/P12", ok)

    Cs = g.uniform(0, 1, (7, 5))
    a7 = g.uniform(0.2, 1, 7)
    b5 = g.uniform(0.2, 1, 5)
    a7 /= a7.sum()
    b5 /= b5.sum()
    f0, g0 = g.normal(size=7) * 0.1, g.normal(size=5) * 0.1
    f1, _ = O.sinkhorn_row(Cs, a7, 0.07, f0, g0)
    g1 = O.sinkhorn_col(Cs, b5, 0.07, f1, g0)
    X1 = np.exp((f1[:, None] + g1[None, :] - Cs - 0.07) / 0.07)
    Xf = np.exp((f1[:, None] + g0[None, :] - Cs - 0.07) / 0.07)
    check("half-sweeps", np.allclose(Xf.sum(1), a7, rtol=1e-13) and np.allclose(X1.sum(0), b5, rtol=1e-13)
          and np.allclose(O.recover(Cs, 0.07, f1, g1), X1, rtol=1e-14))

    check("grid", np.allclose(O.cost_grid(5), W.grid_dense(5), atol=1e-15))
    return failed


def test_pin_suite_passes_on_oracle(oracle_mod):
    assert _pin_suite(oracle_mod) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(oracle_mod, monkeypatch, tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor must be unique"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    so = oracle_mod.compile_to(str(mpath), str(tmp_path / "libmutant.so"))
    monkeypatch.setattr(oracle_mod, "_lib", oracle_mod.load(so))
    with np.errstate(all="ignore"):
        failed = _pin_suite(oracle_mod)
    assert failed, "mutant %s passed every pin" % name
