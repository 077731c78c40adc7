"""Textbook primal-dual interior-point method for a dense convex QP.

TEST INFRASTRUCTURE ONLY: see the package docstring.  It shares nothing
with the dual first-order method; it is here to cross-check optimal values
(Sec. 1 names interior-point solvers as the standard for small dense QPs).

    min 1/2 x^T Q x + q^T x   s.t.  C x <= d,  E x + e = 0
with C = [G; I; -I], d = [-g; ub; -lb] and optional equality rows (E, e).
Infeasible-start path following with Mehrotra's predictor-corrector on the
normal equations (a saddle-point system when equality rows are present).
"""
from __future__ import annotations

import numpy as np


def ipm_qp(Q, q, G, g, lb, ub, tol: float = 1e-11, max_iter: int = 200, E=None, e=None):
    """Returns (x, F, z_G) (and the equality multipliers y as a 4th value when
    E is given)."""
    n = Q.shape[0]
    C = np.vstack([G, np.eye(n), -np.eye(n)])
    d = np.concatenate([-g, ub, -lb])
    m = C.shape[0]
    ne = 0 if E is None else E.shape[0]
    x = np.zeros(n)
    s = np.maximum(d - C @ x, 1.0)
    z = np.ones(m)
    y = np.zeros(ne)
    for _ in range(max_iter):
        rd = Q @ x + q + C.T @ z          # dual residual
        if ne:
            rd = rd + E.T @ y
        rp = C @ x + s - d                # primal residual
        re = E @ x + e if ne else np.zeros(0)
        mu = float(s @ z) / m
        if (np.linalg.norm(rd) <= tol * (1 + np.linalg.norm(q))
                and np.linalg.norm(rp) <= tol * (1 + np.linalg.norm(d))
                and np.linalg.norm(re) <= tol * (1 + (np.linalg.norm(e) if ne else 0.0))
                and mu <= tol * (1 + abs(float(0.5 * x @ Q @ x + q @ x)))):
            break
        w = z / s
        M = Q + C.T @ (w[:, None] * C)
        try:
            Lc = np.linalg.cholesky(M) if not ne else None
        except np.linalg.LinAlgError:   # near the end W is badly scaled
            Lc = None
        K = None
        if ne:
            K = np.block([[M, E.T], [E, np.zeros((ne, ne))]])

        def solve(rs):
            # Newton system: Q dx + C^T dz + E^T dy = -rd ; C dx + ds = -rp ;
            # E dx = -re ; Z ds + S dz = rs
            rhs = -rd - C.T @ ((rs + z * rp) / s)
            dy = np.zeros(0)
            if ne:
                sol = np.linalg.solve(K, np.concatenate([rhs, -re]))
                dx, dy = sol[:n], sol[n:]
            elif Lc is None:
                dx = np.linalg.solve(M, rhs)
            else:
                dx = np.linalg.solve(Lc.T, np.linalg.solve(Lc, rhs))
            ds = -rp - C @ dx
            dz = (rs - z * ds) / s
            return dx, ds, dz, dy

        def step_len(v, dv):
            neg = dv < 0
            return min(1.0, float(np.min(-v[neg] / dv[neg]))) if neg.any() else 1.0

        dxa, dsa, dza, _ = solve(-s * z)
        aa = min(step_len(s, dsa), step_len(z, dza))
        mu_aff = float((s + aa * dsa) @ (z + aa * dza)) / m
        sigma = (mu_aff / mu) ** 3
        dx, ds, dz, dy = solve(-s * z - dsa * dza + sigma * mu)
        a = 0.99 * min(step_len(s, ds), step_len(z, dz))
        x = x + a * dx
        s = s + a * ds
        z = z + a * dz
        if ne:
            y = y + a * dy
    f = 0.5 * x @ Q @ x + q @ x
    if E is not None:
        return x, float(f), z[:G.shape[0]], y
    return x, float(f), z[:G.shape[0]]
