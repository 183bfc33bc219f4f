"""Independent references for the oracle -- TEST INFRASTRUCTURE ONLY.

None of these use the PINS iteration; each pins the oracle to something it
does not compute itself:

* ``lp_bruteforce_perm``  -- m = n <= 8, uniform marginals: LP optima sit at
  vertices of the Birkhoff polytope, i.e. permutation matrices (proof of
  Thm. 2, vertex structure), so OT* = min over permutations of mean C_{i,s(i)}.
* ``lp_vertex_enum``      -- tiny m, n, arbitrary marginals: enumerate bases
  of m+n-1 cells (a vertex has at most m+n-1 nonzeros), keep the feasible
  ones, take the cheapest (textbook LP theory).
* ``lp_monotone_1d``      -- points on a line with convex cost (x-y)^2: the
  sorted north-west-corner coupling is optimal (textbook).
* ``lp_highs``            -- scipy's HiGHS LP solver on eq. (ot).
* ``entropic_2x2``        -- closed form of the 2x2 entropic plan at eps.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def lp_bruteforce_perm(C):
    C = np.asarray(C, np.float64)
    n = C.shape[0]
    assert C.shape == (n, n) and n <= 8
    best = math.inf
    for s in itertools.permutations(range(n)):
        v = sum(C[i, s[i]] for i in range(n)) / n
        if v < best:
            best = v
    return best


def lp_vertex_enum(C, a, b):
    """Cheapest basic feasible solution of eq. (ot) by enumeration (m*n <= ~16)."""
    C = np.asarray(C, np.float64)
    m, n = C.shape
    cells = [(i, j) for i in range(m) for j in range(n)]
    # equality constraints: rows (m) and columns (n), one redundant -> drop last column constraint
    A = np.zeros((m + n - 1, m * n))
    rhs = np.concatenate([a, b[:-1]])
    for i in range(m):
        for j in range(n):
            A[i, i * n + j] = 1.0
            if j < n - 1:
                A[m + j, i * n + j] = 1.0
    best = math.inf
    for basis in itertools.combinations(range(m * n), m + n - 1):
        B = A[:, basis]
        if abs(np.linalg.det(B)) < 1e-12:
            continue
        xb = np.linalg.solve(B, rhs)
        if xb.min() < -1e-12:
            continue
        v = float(sum(C[cells[q]] * xb[k] for k, q in enumerate(basis)))
        best = min(best, v)
    return best


def lp_monotone_1d(x, y, a, b):
    """OT* for squared distance on the real line via the sorted north-west-corner coupling."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    ix = np.argsort(x, kind="stable")
    iy = np.argsort(y, kind="stable")
    ra = np.asarray(a, np.float64)[ix].copy()
    rb = np.asarray(b, np.float64)[iy].copy()
    i = j = 0
    cost = 0.0
    while i < len(ra) and j < len(rb):
        t = min(ra[i], rb[j])
        cost += t * (x[ix[i]] - y[iy[j]]) ** 2
        ra[i] -= t
        rb[j] -= t
        if ra[i] <= rb[j]:
            i += 1
        else:
            j += 1
    return cost


def lp_highs(C, a, b):
    """OT* by scipy.optimize.linprog(method='highs') on eq. (ot)."""
    from scipy.optimize import linprog
    from scipy.sparse import coo_matrix, vstack

    C = np.asarray(C, np.float64)
    m, n = C.shape
    rows = np.repeat(np.arange(m), n)
    cols = np.arange(m * n)
    Ar = coo_matrix((np.ones(m * n), (rows, cols)), shape=(m, m * n))
    rows = np.tile(np.arange(n), m)
    Ac = coo_matrix((np.ones(m * n), (rows, cols)), shape=(n, m * n))
    A = vstack([Ar, Ac]).tocsr()
    beq = np.concatenate([a, b])
    res = linprog(C.ravel(), A_eq=A, b_eq=beq, bounds=(0, None), method="highs",
                  options=dict(primal_feasibility_tolerance=1e-10, dual_feasibility_tolerance=1e-10))
    if res.status != 0:
        raise RuntimeError(res.message)
    return float(res.fun), res.x.reshape(m, n)


def entropic_2x2(C, a, b, eps):
    """Entropic-OT plan of a 2x2 problem at eps in closed form.

    The plan is X = [[t, a1-t], [b1-t, 1-a1-b1+t]]; stationarity of
    <C,X> + eps*sum X log X along the one feasible direction gives
    t(1-a1-b1+t) = q (a1-t)(b1-t) with q = exp(-(C11+C22-C12-C21)/eps),
    i.e. (1-q) t^2 + (1-a1-b1+q(a1+b1)) t - q a1 b1 = 0.
    """
    C = np.asarray(C, np.float64)
    a1, b1 = float(a[0]), float(b[0])
    q = math.exp(-(C[0, 0] + C[1, 1] - C[0, 1] - C[1, 0]) / eps)
    lo, hi = max(0.0, a1 + b1 - 1.0), min(a1, b1)
    A2 = 1.0 - q
    B2 = 1.0 - a1 - b1 + q * (a1 + b1)
    C2 = -q * a1 * b1
    if abs(A2) < 1e-300:
        t = -C2 / B2
    else:
        disc = math.sqrt(max(B2 * B2 - 4 * A2 * C2, 0.0))
        # numerically stable pair of roots
        if B2 >= 0:
            r1 = (-B2 - disc) / (2 * A2)
            r2 = (2 * C2) / (-B2 - disc) if (-B2 - disc) != 0 else r1
        else:
            r1 = (2 * C2) / (-B2 + disc) if (-B2 + disc) != 0 else 0.0
            r2 = (-B2 + disc) / (2 * A2)
        cands = [r for r in (r1, r2) if lo - 1e-15 <= r <= hi + 1e-15]
        t = min(max(cands[0], lo), hi) if cands else min(max(r1, lo), hi)
    return np.array([[t, a1 - t], [b1 - t, 1.0 - a1 - b1 + t]])
