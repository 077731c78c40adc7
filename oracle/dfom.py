"""Algorithm DFOM (Sec. 3) with the inner Algorithm FOM (Sec. 2.1), FP64 NumPy.

TEST INFRASTRUCTURE ONLY: see the package docstring.  Plain and slow on
purpose: every product is taken directly from its definition, with no
blocking, fusion or reuse beyond what the algorithms state.

QP class: Sec. 2, eq. original_primal, with K = R^p_- (G u + g <= 0) and
the box U = [lb, ub].

Readings of points the paper leaves open (each is listed again in the
design notes):
  * Inner stopping test (Step 1, eq. duquad_in).  The criterion needs the
    unknown d_rho(mu).  It is replaced by a computable certificate that is
    a rigorous upper bound on L_rho(x, mu) - d_rho(mu):
      - at a point x of the box with the exact gradient g = grad phi(x):
        min(FW gap  sum_i max(g_i (x_i - lb_i), g_i (x_i - ub_i)),
            ||pi||^2 / (2 sigma))       [second term only when sigma > 0]
        with pi the minimum-norm element of g + N_U(x);
      - after a projected step x = [y - grad phi(y)/L]_U, with the gradient
        mapping G_L = L (y - x):
        min(sum_i max(G_i (y_i - lb_i), G_i (y_i - ub_i)) - ||G_L||^2/(2L),
            ||G_L||^2 (1/sigma - 1/L) / 2)  [second term only when sigma > 0].
    With rho = 0, and with rho > 0 when every row is an equality (the inner
    gradient is then affine in u: constant Hessian Q + rho G^T G, Sec. 5.1),
    the exact-gradient form is used at every inner iterate.  Otherwise, with
    rho > 0, the exact form is used for the warm start x^0 and the
    gradient-mapping form after each step (it needs no extra product).
    The loop also stops at the iteration count k_in of Sec. 5 (natural log,
    rounded up), which by Lemma lemma_sublin_dfg already implies the
    criterion when the constants are exact.
  * Inner variant: FGM_sigma when sigma_in > 0, FGM otherwise (Sec. 2.1);
    sigma_in = lambda_min(Q) (the strong convexity of L_rho(., mu) that
    survives the [.]_+ term).  Inner momentum restarts every outer
    iteration; only x is warm-started (Sec. 3, warm start).
  * First inner start: the projection of the origin onto U.
  * lambda^0 = 0 unless given (Sec. 4), lambda^{-1} = lambda^0, theta_1 = 1.
  * Primal average over j = 1..k with weights theta_j (eq. average_primal).
  * Outer test (the paper's experiments use the unknown F*): on the
    candidate x (last or averaged iterate)
        ||[Gx+g]_+|| <= eps_out max(1, ||g||),
        F(x) - LB   <= eps_out max(1, |F(x)|),
        ||lambda^k|| ||[Gx+g]_+|| <= eps_out max(1, |F(x)|),
    with LB = max_j (dbar_j - gap_j) over multipliers where weak duality
    holds (mu^j >= 0 when rho = 0, every mu^j when rho > 0).
  * The ||pi||^2/(2 sigma) and gradient-mapping sigma terms bound the inner
    gap only when sigma is a true lower bound on the strong convexity.  An
    estimated sigma (a Lanczos Ritz value lies above lambda_min) may be too
    large, so with Options.lb_sigma_free the gap that enters LB is the
    sigma-free part (the FW gap, or the gradient-mapping bound without the
    sigma term); the inner stopping test keeps the sigma form.
  * Last iterate of DFGM is u(lambda^k) (eq. last_primal): when ubar^k
    passes the test, one more inner solve at lambda^k, warm-started from
    ubar^k, is tested and returned if it passes; otherwise the iteration
    continues from ubar^k unchanged (the extra solve only raises LB).
  * Infeasible constraints (outside the paper, which assumes a finite
    optimal multiplier, Sec. 2): with rho = 0, before each inner solve a
    mu^k >= 0 is tested as a certificate that no u in U has G u + g <= 0
    (infeasibility_certificate); the run then ends with mu^k as the
    multipliers and the warm start as x.
  * Equality rows (K = {0}, Sec. 2) and the user form lbar <= Gbar u + gbar
    <= ubar: stack_rows turns the user form into rows of G u + g in
    K = R^m_- x {0}^e (an equality where lbar = ubar, else one inequality per
    finite side); `eq` marks the equality rows.  Their multipliers are free
    (K_d = R there), their distance to K is |r| and, with rho > 0, they add
    rho G_eq^T G_eq to the inner Hessian: sigma_in = lambda_min(Q + rho
    G_eq^T G_eq) (Sec. 3, Step 1, the K = {0} case).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

DGM, DFGM = 0, 1
LAST, AVG = 0, 1
CERT, FIXED = 0, 1
INNER_AUTO, INNER_GM, INNER_FGM, INNER_FGM_SIGMA = 0, 1, 2, 3

STATUS_OK = 0
STATUS_MAXITER = 1
STATUS_INFEASIBLE = 2

# Relative margin of the infeasibility certificate (see infeasibility_certificate)
# and the outer iterations at which it is tested: k = 1, 1 + INFEAS_EVERY, ...
INFEAS_MARGIN = 1e-6
INFEAS_EVERY = 8


@dataclass
class Options:
    method: int = DFGM
    output: int = LAST
    inner_rule: int = CERT
    inner_variant: int = INNER_AUTO
    eps_out: float = 1e-4
    eps_in: float = 1e-6
    rho: float = 0.0
    max_outer: int = 10000
    max_inner: int = 0            # 0: use the k_in count of Sec. 5
    lam_min: Optional[float] = None
    lam_max: Optional[float] = None
    G_norm2: Optional[float] = None
    log_vectors: int = 0          # outer iterations whose vectors are logged
    lb_sigma_free: bool = False   # LB from sigma-free inner certificates (sigma estimated)


@dataclass
class Constants:
    lam_min: float
    lam_max: float
    G_norm2: float
    Ld: float
    alpha: float
    L_in: float
    sigma_in: float
    beta_in: float
    D_U: float
    k_in_max: int
    Kd_nonneg: bool


@dataclass
class Result:
    x: np.ndarray
    lam: np.ndarray
    F: float
    LB: float
    feas: float
    status: int
    outer_iters: int
    inner_iters: int
    consts: Constants
    log: List[dict] = field(default_factory=list)


# ----------------------------------------------------------------------------
# Constants (Sec. 2 eq. Ld, Sec. 3 Step 1, Sec. 5 k_in)
# ----------------------------------------------------------------------------

def problem_constants(Q, G, lb, ub, rho: float, eps_in: float,
                      lam_min=None, lam_max=None, G_norm2=None,
                      max_inner: int = 0, eq=None, sigma_in=None) -> Constants:
    """L_d, the outer step 1/(2 L_d), the inner L and sigma, beta, D_U, k_in.

    Spectral quantities default to exact dense eigen/singular values.  With
    rho > 0 and equality rows (eq), sigma_in = lambda_min(Q + rho G_eq^T G_eq)
    (Sec. 3, Step 1) unless given."""
    if sigma_in is None and rho > 0.0 and eq is not None and np.any(eq):
        Ge = G[np.asarray(eq, bool)]
        sigma_in = float(np.linalg.eigvalsh(Q + rho * (Ge.T @ Ge))[0])
    if lam_min is None or lam_max is None:
        ev = np.linalg.eigvalsh(Q)
        lam_min = float(ev[0]) if lam_min is None else lam_min
        lam_max = float(ev[-1]) if lam_max is None else lam_max
    if G_norm2 is None:
        G_norm2 = float(np.linalg.norm(G, 2) ** 2) if G.shape[0] > 0 else 0.0
    denom = lam_min + rho * G_norm2
    if G_norm2 == 0.0:
        Ld = 0.0
    elif denom <= 0.0:
        raise ValueError("lambda_min(Q) = 0 needs rho > 0 (Sec. 2, Case 2)")
    else:
        Ld = G_norm2 / denom                       # eq. Ld
    alpha = 0.0 if Ld == 0.0 else 1.0 / (2.0 * Ld)  # Algorithm DFOM step 2
    L_in = lam_max + rho * G_norm2                  # Sec. 3, Step 1
    sigma_in = max(lam_min if sigma_in is None else sigma_in, 0.0)
    sqL, sqs = math.sqrt(L_in), math.sqrt(sigma_in)
    beta_in = (sqL - sqs) / (sqL + sqs)             # FGM_sigma, Sec. 2.1
    D_U = float(np.linalg.norm(ub - lb))
    if max_inner > 0:
        k_in = int(max_inner)
    elif sigma_in > 0.0:                            # Sec. 5, k_in
        arg = L_in * D_U * D_U / eps_in
        k_in = int(math.ceil(math.sqrt(L_in / sigma_in) * math.log(arg))) + 1 if arg > 1.0 else 1
    else:
        k_in = int(math.ceil(math.sqrt(2.0 * L_in * D_U * D_U / eps_in)))
    k_in = max(k_in, 1)
    return Constants(lam_min, lam_max, G_norm2, Ld, alpha, L_in, sigma_in,
                     beta_in, D_U, k_in, lam_min > 0.0)


# ----------------------------------------------------------------------------
# Objective, (augmented) Lagrangian, dual gradient (Sec. 2, Sec. 3)
# ----------------------------------------------------------------------------

def objective(Q, q, u) -> float:
    """F(u) = 1/2 u^T Q u + q^T u (eq. original_primal)."""
    return float(0.5 * u @ (Q @ u) + q @ u)


def _ineq(G, eq):
    """Boolean mask of the inequality rows (K_i = R_-); eq marks K_i = {0}."""
    return np.ones(G.shape[0], bool) if eq is None else ~np.asarray(eq, bool)


def proj_K(v, eq=None) -> np.ndarray:
    """Projection onto K = R^m_- x {0}^e (rows in place)."""
    return np.where(_ineq(np.zeros((len(v), 0)), eq), np.minimum(v, 0.0), 0.0)


def dist_K(v, eq=None) -> float:
    """Distance of v to K: ||v - [v]_K||."""
    return float(np.linalg.norm(v - proj_K(v, eq)))


def slack(G, g, u, lam, rho: float, eq=None) -> np.ndarray:
    """s(u, lambda): [G u + g + lambda/rho]_K for rho > 0, 0 for rho = 0 (Sec. 2)."""
    if rho > 0.0:
        return proj_K(G @ u + g + lam / rho, eq)
    return np.zeros(G.shape[0])


def lagrangian(Q, q, G, g, u, lam, rho: float, eq=None) -> float:
    """L_rho(u, lambda) of eq. auglag1 (dist_K(v) = ||[v]_+|| on rows in R_-,
    |v| on rows in {0})."""
    r = G @ u + g
    if rho > 0.0:
        d = dist_K(r + lam / rho, eq)
        return objective(Q, q, u) + 0.5 * rho * d * d - float(lam @ lam) / (2.0 * rho)
    return objective(Q, q, u) + float(lam @ r)


def dual_gradient(G, g, u, lam, rho: float, eq=None) -> np.ndarray:
    """bar-nabla d_rho(lambda) = G u + g - s(u, lambda) (eq. inexact_framework)."""
    return G @ u + g - slack(G, g, u, lam, rho, eq)


def inner_gradient(Q, q, G, g, u, mu, rho: float, eq=None) -> np.ndarray:
    """Gradient in u of L_rho(u, mu).

    rho = 0: Q u + q + G^T mu.  rho > 0: Q u + q + G^T w with
    w = mu + rho (G u + g) - rho s (the derivative of (rho/2) dist_K(G u + g +
    mu/rho)^2): [mu + rho (G u + g)]_+ on rows in R_-, mu + rho (G u + g) on
    rows in {0}."""
    if rho > 0.0:
        v = mu + rho * (G @ u + g)
        w = np.where(_ineq(G, eq), np.maximum(v, 0.0), v)
        return Q @ u + q + G.T @ w
    return Q @ u + q + G.T @ mu


def stack_rows(G, g, rlo, rhi):
    """The user form rlo <= G u + g <= rhi (Sec. 2; -inf / +inf for an absent
    side) as rows of Gs u + gs in K = R^m_- x {0}^e: an equality row
    G_i u + g_i - rhi_i = 0 where rlo_i = rhi_i, else G_i u + g_i - rhi_i <= 0
    for a finite rhi_i and -G_i u - g_i + rlo_i <= 0 for a finite rlo_i.
    Returns (Gs, gs, eq, src, sign): row j of the stack is sign_j times row
    src_j of G.  The order is: for each i in turn, its upper (or equality)
    row, then its lower row."""
    rows, off, eq, src, sign = [], [], [], [], []
    for i in range(G.shape[0]):
        lo, hi = float(rlo[i]), float(rhi[i])
        if lo == hi:
            rows.append(G[i]); off.append(g[i] - hi); eq.append(True); src.append(i); sign.append(1.0)
            continue
        if math.isfinite(hi):
            rows.append(G[i]); off.append(g[i] - hi); eq.append(False); src.append(i); sign.append(1.0)
        if math.isfinite(lo):
            rows.append(-G[i]); off.append(lo - g[i]); eq.append(False); src.append(i); sign.append(-1.0)
    n = G.shape[1]
    Gs = np.array(rows, float).reshape(-1, n)
    return (Gs, np.array(off, float), np.array(eq, bool), np.array(src, int), np.array(sign, float))


# ----------------------------------------------------------------------------
# Inner certificates
# ----------------------------------------------------------------------------

def inner_certificate(x, grad, lb, ub, sigma: float) -> float:
    """Upper bound on phi(x) - min_U phi at a box point x with gradient grad."""
    fw = float(np.sum(np.maximum(grad * (x - lb), grad * (x - ub))))
    if sigma <= 0.0:
        return fw
    pi = grad.copy()
    at_lb = x <= lb
    at_ub = x >= ub
    pi[at_lb] = np.minimum(grad[at_lb], 0.0)
    pi[at_ub] = np.maximum(grad[at_ub], 0.0)
    pi[at_lb & at_ub] = 0.0
    return min(fw, float(pi @ pi) / (2.0 * sigma))


def gradmap_certificate(y, x, L: float, lb, ub, sigma: float) -> float:
    """Upper bound on phi(x) - min_U phi for x = [y - grad phi(y)/L]_U.

    With G_L = L (y - x): phi(x) - phi(z) <= <G_L, y - z> - ||G_L||^2/(2L)
    - (sigma/2) ||z - y||^2 for every z in U; maximise over z."""
    gm = L * (y - x)
    gg = float(gm @ gm)
    fw = float(np.sum(np.maximum(gm * (y - lb), gm * (y - ub)))) - gg / (2.0 * L)
    if sigma <= 0.0:
        return fw
    return min(fw, 0.5 * gg * (1.0 / sigma - 1.0 / L))


# ----------------------------------------------------------------------------
# Algorithm FOM on the inner problem (Sec. 2.1)
# ----------------------------------------------------------------------------

def _inner_beta_schedule(variant: int, sigma: float, beta_in: float):
    """Yields beta_1, beta_2, ... of Algorithm FOM for the chosen variant."""
    if variant == INNER_AUTO:
        variant = INNER_FGM_SIGMA if sigma > 0.0 else INNER_FGM
    if variant == INNER_GM:
        while True:
            yield 0.0
    elif variant == INNER_FGM_SIGMA:
        while True:
            yield beta_in
    else:  # FGM: theta_1 = 1, theta_{k+1} = (1 + sqrt(1 + 4 theta_k^2)) / 2
        th = 1.0
        while True:
            th_next = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * th * th))
            yield (th - 1.0) / th_next
            th = th_next


def fom_inner(Q, q, G, g, lb, ub, mu, rho: float, c: Constants, x0,
              eps_in: float, rule: int = CERT, variant: int = INNER_AUTO, eq=None,
              sigma_free: bool = False):
    """Approximate u(mu) by Algorithm FOM(L_rho(., mu), U) from x^0 = y^1 = x0.

    Returns (x, steps, gap) with gap the certificate value of x; with
    sigma_free also the certificate of x without its sigma term (valid for
    any strong convexity constant): (x, steps, gap, gap_sigma_free)."""
    L, sigma, k_max = c.L_in, c.sigma_in, c.k_in_max
    betas = _inner_beta_schedule(variant, sigma, c.beta_in)

    def grad(u):
        return inner_gradient(Q, q, G, g, u, mu, rho, eq)

    def done(gap, t):
        return (rule == CERT and gap <= eps_in) or t >= k_max

    # The gradient is affine in u when rho = 0, and when rho > 0 with every row
    # an equality (the constant inner Hessian Q + rho G^T G of Sec. 5.1): then
    # the exact-gradient certificate is taken at every iterate.
    affine = rho == 0.0 or (eq is not None and G.shape[0] > 0 and bool(np.all(eq)))
    if affine:
        x_prev = x = x0.copy()
        t = 0
        while True:
            gx = grad(x)
            gap = inner_certificate(x, gx, lb, ub, sigma)
            if done(gap, t):
                return (x, t, gap, inner_certificate(x, gx, lb, ub, 0.0)) if sigma_free else (x, t, gap)
            if t == 0:
                y = x                                   # y^1 = x^0
            else:
                y = x + next(betas) * (x - x_prev)      # y^{t+1}
            x_prev = x
            x = np.clip(y - grad(y) / L, lb, ub)        # x^{t+1}
            t += 1
    # rho > 0: gradient at y only; exact certificate at x^0, gradient-mapping after
    x_prev = x0.copy()
    y = x0.copy()
    t = 0
    while True:
        gy = grad(y)
        if t == 0:
            gap = inner_certificate(x0, gy, lb, ub, sigma)
            if rule == CERT and gap <= eps_in:
                return ((x0.copy(), 0, gap, inner_certificate(x0, gy, lb, ub, 0.0)) if sigma_free
                        else (x0.copy(), 0, gap))
        x = np.clip(y - gy / L, lb, ub)
        t += 1
        gap = gradmap_certificate(y, x, L, lb, ub, sigma)
        if done(gap, t):
            return (x, t, gap, gradmap_certificate(y, x, L, lb, ub, 0.0)) if sigma_free else (x, t, gap)
        y = x + next(betas) * (x - x_prev)
        x_prev = x


# ----------------------------------------------------------------------------
# Algorithm DFOM (Sec. 3) with last / averaged primal output (Sec. 4)
# ----------------------------------------------------------------------------

def _outer_test(Q, q, G, g, x, lam, LB, eps, gnorm, eq=None):
    Fx = objective(Q, q, x)
    feas = dist_K(G @ x + g, eq)
    scale = max(1.0, abs(Fx))
    ok = (feas <= eps * max(1.0, gnorm) and Fx - LB <= eps * scale
          and float(np.linalg.norm(lam)) * feas <= eps * scale)
    return ok, Fx, feas


def infeasibility_certificate(G, g, lb, ub, mu):
    """v = min over the box U of mu^T (G u + g), and the scale of its terms.

    The paper assumes a finite optimal multiplier exists (Sec. 2, strong
    duality).  When no point of U satisfies G u + g in K the dual is unbounded
    above and the multipliers grow without bound; a mu with mu_i >= 0 on the
    inequality rows (any sign on equality rows) and v > 0 proves it: every u
    in U has mu^T (G u + g) >= v > 0, while a feasible u would give <= 0.
    The box minimum is separable: sum_j min(lb_j w_j, ub_j w_j), w = G^T mu.
    Returns (v, scale) with scale = sum |mu_i g_i| + sum |w_j| max(|lb_j|, |ub_j|);
    the run stops when v > INFEAS_MARGIN * scale."""
    w = G.T @ mu
    v = float(mu @ g + np.sum(np.minimum(lb * w, ub * w)))
    scale = float(np.sum(np.abs(mu * g)) + np.sum(np.abs(w) * np.maximum(np.abs(lb), np.abs(ub))))
    return v, scale


def dfom_solve(qp, opts: Options, consts: Optional[Constants] = None,
               x_start=None, lam_start=None) -> Result:
    """Inexact (augmented) dual first-order method DFOM(d_rho, K_d).

    qp.eq (optional) marks equality rows (K_i = {0}); the others are
    inequalities (K_i = R_-)."""
    Q, q, G, g, lb, ub = qp.Q, qp.q, qp.G, qp.g, qp.lb, qp.ub
    eq = getattr(qp, "eq", None)
    if eq is not None and not np.any(eq):
        eq = None
    rho = float(opts.rho)
    c = consts or problem_constants(Q, G, lb, ub, rho, opts.eps_in,
                                    opts.lam_min, opts.lam_max, opts.G_norm2,
                                    opts.max_inner, eq=eq)
    p = G.shape[0]
    gnorm = float(np.linalg.norm(g))
    ineq = _ineq(G, eq)

    def proj_Kd(v):
        # K_d = R_+ on inequality rows when Q > 0 (after eq. dual_pr), R elsewhere
        return np.where(ineq, np.maximum(v, 0.0), v) if c.Kd_nonneg else v

    def in_Kd(v):
        return bool(np.all(v[ineq] >= 0.0))

    lam = proj_Kd(np.zeros(p) if lam_start is None else np.asarray(lam_start, float))
    lam_prev = lam.copy()                          # lambda^{-1} = lambda^0
    mu = lam.copy()                                # mu^1 = lambda^0
    theta = 1.0                                    # theta_1
    S = 0.0
    u_sum = np.zeros_like(q)
    x_warm = np.clip(np.zeros_like(q), lb, ub) if x_start is None else np.asarray(x_start, float).copy()
    LB = -math.inf
    inner_total = 0
    log: List[dict] = []
    last = None

    for k in range(1, opts.max_outer + 1):
        # Before step 1 (rho = 0, mu^k >= 0): a Farkas-type certificate that
        # no feasible point exists ends the run with mu^k as the certificate.
        if rho == 0.0 and p > 0 and k % INFEAS_EVERY == 1 and in_Kd(mu):
            v, scale = infeasibility_certificate(G, g, lb, ub, mu)
            if v > INFEAS_MARGIN * scale:
                Fx = objective(Q, q, x_warm)
                feas = dist_K(G @ x_warm + g, eq)
                return Result(x_warm.copy(), mu.copy(), Fx, LB, feas, STATUS_INFEASIBLE,
                              k, inner_total, c, log)
        # Step 1: ubar^k approximately minimises L_rho(., mu^k) over U
        u, t, gap, gap_lb = fom_inner(Q, q, G, g, lb, ub, mu, rho, c, x_warm, opts.eps_in, opts.inner_rule,
                                      opts.inner_variant, eq, sigma_free=True)
        if not opts.lb_sigma_free:
            gap_lb = gap
        inner_total += t
        dg = dual_gradient(G, g, u, mu, rho, eq)
        dbar = lagrangian(Q, q, G, g, u, mu, rho, eq)
        if rho > 0.0 or in_Kd(mu):                 # weak duality holds at mu^k
            LB = max(LB, dbar - gap_lb)
        # Step 2: projected inexact dual gradient step
        lam_k = proj_Kd(mu + c.alpha * dg)
        # Step 3: momentum (DGM: theta = 1; DFGM: theta rule)
        if opts.method == DFGM:
            theta_next = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * theta * theta))
        else:
            theta_next = 1.0
        beta = (theta - 1.0) / theta_next
        mu_next = lam_k + beta * (lam_k - lam_prev)
        # eq. average_primal, weights theta_j, j = 1..k
        S += theta
        u_sum = u_sum + theta * u
        u_hat = u_sum / S
        cand = u if opts.output == LAST else u_hat
        ok, Fx, feas = _outer_test(Q, q, G, g, cand, lam_k, LB, opts.eps_out, gnorm, eq)
        entry = dict(k=k, t=t, gap=gap, dbar=dbar, LB=LB, theta=theta, S=S,
                     F=Fx, feas=feas, lam_norm=float(np.linalg.norm(lam_k)), passed=ok)
        if k <= opts.log_vectors:
            entry.update(mu=mu.copy(), u=u.copy(), lam=lam_k.copy())
        result_x = cand
        if ok and opts.output == LAST and opts.method == DFGM:
            # last primal iterate u(lambda^k), eq. last_primal
            u2, t2, gap2, gap2_lb = fom_inner(Q, q, G, g, lb, ub, lam_k, rho, c, u, opts.eps_in, opts.inner_rule,
                                              opts.inner_variant, eq, sigma_free=True)
            if not opts.lb_sigma_free:
                gap2_lb = gap2
            inner_total += t2
            if rho > 0.0 or in_Kd(lam_k):
                LB = max(LB, lagrangian(Q, q, G, g, u2, lam_k, rho, eq) - gap2_lb)
            ok, Fx, feas = _outer_test(Q, q, G, g, u2, lam_k, LB, opts.eps_out, gnorm, eq)
            entry.update(extra_t=t2, extra_gap=gap2, LB=LB, F2=Fx, feas2=feas, passed2=ok)
            result_x = u2
        log.append(entry)
        last = (result_x, lam_k, Fx, feas)
        if ok:
            return Result(result_x.copy(), lam_k.copy(), Fx, LB, feas, STATUS_OK,
                          k, inner_total, c, log)
        lam_prev = lam_k
        mu = mu_next
        theta = theta_next
        x_warm = u
    x, lam_k, Fx, feas = last
    return Result(x.copy(), lam_k.copy(), Fx, LB, feas, STATUS_MAXITER,
                  opts.max_outer, inner_total, c, log)
