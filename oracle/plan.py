"""Parameter planning from the complexity results, FP64 (TEST INFRASTRUCTURE
ONLY: see the package docstring).

* Sec. 3.1, eq. choose_ein: the inner accuracy eps_in and the number of outer
  iterations k_out that make both terms of the dual rate bound of Theorem
  lemma_sublin_dfg_inexact at most eps/2, for DGM (p = 1) and DFGM (p = 2).
* Sec. 5, Theorem in:th_last: the penalty rho* = 8 R_d^2 / eps.
* The inner count of Sec. 5 (k_in) at the planned eps_in, and the predicted
  total k_out * k_in.
* planned_solve: R_d = min ||lambda* - lambda^0|| is unknown; the paper leaves
  an implementable scheme open (a search on R_d, mentioned and left out before
  Sec. 6.2).  Reading taken here: guess R, run DFOM with the planned (eps_in,
  k_out) and the outer test at eps; if the test has not passed after k_out
  outer iterations, double R and continue from the last x and lambda.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from .dfom import DFGM, DGM, LAST, Options, dfom_solve, problem_constants, STATUS_OK


@dataclass
class Plan:
    eps_in: float
    k_out: int
    rho_star: float
    k_in: Optional[int] = None
    k_total: Optional[int] = None


def plan(method: int, eps: float, Ld: float, Rd: float, L_in: Optional[float] = None,
         sigma_in: Optional[float] = None, D_U: Optional[float] = None) -> Plan:
    """eq. choose_ein (eps_in, k_out), rho* of Theorem in:th_last, and the
    inner count k_in of Sec. 5 at that eps_in when L_in, sigma_in, D_U are
    given (natural log, rounded up, as everywhere in this oracle)."""
    if method == DGM:
        eps_in = eps / 4.0
        k_out = math.ceil(8.0 * Ld * Rd * Rd / eps)
    else:
        eps_in = eps * math.sqrt(eps) / (8.0 * Rd * math.sqrt(2.0 * Ld))
        k_out = math.ceil(math.sqrt(8.0 * Ld * Rd * Rd / eps))
    k_out = max(k_out, 1)
    p = Plan(eps_in, k_out, 8.0 * Rd * Rd / eps)
    if L_in is not None and sigma_in is not None and D_U is not None:
        if sigma_in > 0.0:
            arg = L_in * D_U * D_U / eps_in
            k_in = math.ceil(math.sqrt(L_in / sigma_in) * math.log(arg)) + 1 if arg > 1.0 else 1
        else:
            k_in = math.ceil(math.sqrt(2.0 * L_in * D_U * D_U / eps_in))
        p.k_in = max(k_in, 1)
        p.k_total = p.k_in * p.k_out
    return p


def dual_rate_terms(method: int, Ld: float, Rd: float, k: int, eps_in: float):
    """The two terms of the bound of Theorem lemma_sublin_dfg_inexact after k
    outer iterations: 4 L_d R_d^2 / (k+1)^p and 2 (k+1)^(p-1) eps_in."""
    pw = 1 if method == DGM else 2
    return 4.0 * Ld * Rd * Rd / (k + 1) ** pw, 2.0 * (k + 1) ** (pw - 1) * eps_in


@dataclass
class PlannedResult:
    x: np.ndarray
    lam: np.ndarray
    status: int
    rounds: int
    R: float
    outer_iters: int
    inner_iters: int
    F: float
    plans: List[Plan]


def planned_solve(qp, method: int, eps: float, R0: float, max_rounds: int = 12, output: int = LAST,
                  consts=None) -> PlannedResult:
    """DFOM with eps_in and max_outer from eq. choose_ein for a guess R of R_d,
    doubling R whenever the outer test (at eps) has not passed within k_out
    iterations; each round starts from the previous round's x and lambda."""
    c = consts or problem_constants(qp.Q, qp.G, qp.lb, qp.ub, 0.0, 1e-6)
    R = R0
    x0 = lam0 = None
    outer = inner = 0
    plans = []
    r = None
    for rnd in range(1, max_rounds + 1):
        pl = plan(method, eps, c.Ld, R)
        plans.append(pl)
        cr = problem_constants(qp.Q, qp.G, qp.lb, qp.ub, 0.0, pl.eps_in, c.lam_min, c.lam_max, c.G_norm2)
        r = dfom_solve(qp, Options(method=method, output=output, eps_out=eps, eps_in=pl.eps_in,
                                   max_outer=pl.k_out), consts=cr, x_start=x0, lam_start=lam0)
        outer += r.outer_iters
        inner += r.inner_iters
        if r.status == STATUS_OK:
            return PlannedResult(r.x, r.lam, r.status, rnd, R, outer, inner, r.F, plans)
        x0, lam0 = r.x, r.lam
        R *= 2.0
    return PlannedResult(r.x, r.lam, r.status, max_rounds, R / 2.0, outer, inner, r.F, plans)
