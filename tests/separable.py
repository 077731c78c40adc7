"""Closed-form optimum of a diagonal QP with one constraint row (test helper).

min 1/2 sum d_i u_i^2 + q^T u  s.t.  a^T u - b <= 0,  lb <= u <= ub,  d > 0.

For a multiplier m >= 0 the Lagrangian separates and its box minimiser is
u_i(m) = clip(-(q_i + m a_i) / d_i, lb_i, ub_i); phi(m) = a^T u(m) - b is
non-increasing in m.  The optimal multiplier is 0 if phi(0) <= 0, otherwise
the root of phi, found here by bisection to machine precision (KKT of a
strongly convex problem: the pair (u(m*), m*) is the unique optimum).
"""
import numpy as np


def u_of(m, d, q, a, lb, ub):
    return np.clip(-(q + m * a) / d, lb, ub)


def solve(d, q, a, b, lb, ub):
    """(u*, m*, F*) by bisection on the multiplier."""
    phi = lambda m: float(a @ u_of(m, d, q, a, lb, ub) - b)
    if phi(0.0) <= 0.0:
        m = 0.0
    else:
        lo, hi = 0.0, 1.0
        while phi(hi) > 0.0:
            lo, hi = hi, 2.0 * hi
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if phi(mid) > 0.0:
                lo = mid
            else:
                hi = mid
        m = 0.5 * (lo + hi)
    u = u_of(m, d, q, a, lb, ub)
    return u, m, objective(u, d, q)


def objective(u, d, q):
    return float(0.5 * np.sum(d * u * u) + q @ u)


def error_bounds(x, d, q, a, b, lb, ub):
    """For a box point x: (F(x) - F*, lower bound on it, bound on ||x - u*||).

    Weak duality with the optimal multiplier gives F(x) >= F* - m* viol(x),
    and strong convexity of the Lagrangian at m* (modulus min d) gives
    ||x - u*||^2 <= 2 (F(x) + m* (a^T x - b) - F*) / min d."""
    u, m, F = solve(d, q, a, b, lb, ub)
    Fx = objective(x, d, q)
    lag_gap = Fx + m * float(a @ x - b) - F
    dist = np.sqrt(max(0.0, 2.0 * lag_gap / float(np.min(d))))
    return Fx - F, -m * max(0.0, float(a @ x - b)), dist, lag_gap
