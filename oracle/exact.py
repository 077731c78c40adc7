"""Exact references for tiny QPs, used to pin the oracle.

TEST INFRASTRUCTURE ONLY: see the package docstring.

Brute-force active-set enumeration (the textbook fact behind active-set
methods, Sec. 1): the minimiser of a strictly convex QP over a polytope is
the minimiser of F on the affine set cut out by its active constraints.
Enumerating every choice of (variable at lb / at ub / free) x (constraint
row active / inactive), solving the equality-constrained KKT system and
keeping the best feasible point therefore yields x* and F* exactly (up to
the rounding of the small linear solves).  Cost 3^n 2^p solves: n <= 8.
"""
from __future__ import annotations

import itertools

import numpy as np


def _eq_qp(Q, q, G, g, lb, ub, state, active):
    """Minimise F with x_i fixed per `state` and rows `active` of G as equalities."""
    n = Q.shape[0]
    fixed = np.array([s != 0 for s in state], bool)
    xF = np.where(np.array(state) < 0, lb, ub)[fixed]
    free = ~fixed
    m = int(free.sum())
    A = G[list(active)] if active else np.zeros((0, n))
    bA = g[list(active)] if active else np.zeros(0)
    na = A.shape[0]
    if m == 0:
        x = np.where(np.array(state) < 0, lb, ub).astype(float)
        if na and np.max(np.abs(A @ x + bA)) > 1e-9:
            return None
        return x, np.zeros(na)
    Qff = Q[np.ix_(free, free)]
    Qfx = Q[np.ix_(free, fixed)]
    Af = A[:, free]
    Ax = A[:, fixed]
    K = np.zeros((m + na, m + na))
    K[:m, :m] = Qff
    K[:m, m:] = Af.T
    K[m:, :m] = Af
    rhs = np.concatenate([-(q[free] + Qfx @ xF), -(bA + Ax @ xF)])
    if np.linalg.cond(K) > 1e12:
        return None
    sol = np.linalg.solve(K, rhs)
    x = np.empty(n)
    x[fixed] = xF
    x[free] = sol[:m]
    return x, sol[m:]


def brute_force_qp(Q, q, G, g, lb, ub, tol: float = 1e-9, eq=None):
    """Exact (x*, F*, lambda*) of min F s.t. Gx+g <= 0, lb <= x <= ub (n <= 8).

    eq (optional) marks rows that are equalities (G_i x + g_i = 0): they are
    active in every face.  lambda* is recovered from the stationarity
    equations on the active rows (least squares; unique under LICQ)."""
    n, p = Q.shape[0], G.shape[0]
    if n > 8 or p > 8:
        raise ValueError("brute force is for n, p <= 8")
    eqm = np.zeros(p, bool) if eq is None else np.asarray(eq, bool)
    best = None
    for state in itertools.product((-1, 0, 1), repeat=n):
        for act in itertools.product((0, 1), repeat=p):
            if any(eqm[j] and not act[j] for j in range(p)):
                continue
            active = tuple(j for j in range(p) if act[j])
            r = _eq_qp(Q, q, G, g, lb, ub, state, active)
            if r is None:
                continue
            x, _ = r
            if np.any(x < lb - tol) or np.any(x > ub + tol):
                continue
            if p and np.any((G @ x + g)[~eqm] > tol):
                continue
            if p and np.any(np.abs(G @ x + g)[eqm] > tol):
                continue
            f = 0.5 * x @ Q @ x + q @ x
            if best is None or f < best[1] - 1e-13:
                best = (x, f)
    if best is None:
        raise ValueError("infeasible QP")
    x, f = best
    # multipliers of the active rows from stationarity on the free coordinates
    lam = np.zeros(p)
    act = np.where((G @ x + g > -1e-8) | eqm)[0] if p else np.zeros(0, int)
    free = (x > lb + 1e-8) & (x < ub - 1e-8)
    if len(act):
        grad = Q @ x + q
        A = G[np.ix_(act, np.where(free)[0])].T if free.any() else np.zeros((0, len(act)))
        if A.shape[0]:
            sol, *_ = np.linalg.lstsq(A, -grad[free], rcond=None)
            lam[act] = sol
    return x, float(f), lam


def box_qp_exact(Q, c, lb, ub, tol: float = 1e-10):
    """Exact minimiser of 1/2 u^T Q u + c^T u over the box (n <= 10), by face enumeration."""
    n = Q.shape[0]
    zeros_G = np.zeros((0, n))
    best = None
    for state in itertools.product((-1, 0, 1), repeat=n):
        r = _eq_qp(Q, c, zeros_G, np.zeros(0), lb, ub, state, ())
        if r is None:
            continue
        x, _ = r
        if np.any(x < lb - tol) or np.any(x > ub + tol):
            continue
        f = 0.5 * x @ Q @ x + c @ x
        if best is None or f < best[1]:
            best = (x, f)
    return best[0], float(best[1])
