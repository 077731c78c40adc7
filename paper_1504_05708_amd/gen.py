"""Seeded synthetic QP generators.

This module only draws problem data; it holds none of the solver's
arithmetic.  Both the CPU oracle tests and the HIP path take their inputs
from here, so the two sides always see the same bits.

Problem class (Sec. 2, eq. original_primal):
    min 1/2 u^T Q u + q^T u   s.t.  G u + g <= 0,  lb <= u <= ub.

The paper's experiments use "random QPs" without a published generator
(Sec. 6.2, 6.3) and motivate the method with linear MPC (Sec. 1, Sec. 2).
The recipes below stand in for those workloads:

* random_dense_qp: Q = A^T A / n + reg*I with A (2n x n) i.i.d. N(0,1),
  q ~ N(0,1), G (p x n) i.i.d. N(0,1), g = -(G x0) - s with
  x0 ~ U(-.5,.5)^n and s ~ U(.1,1)^p so that x0 is strictly feasible,
  box [-1, 1].  Draw order A, q, G, x0, s from numpy's PCG64.
* mpc_system / mpc_instance: condensed linear MPC with nx states, nu
  inputs, horizon N; input box |u| <= 1 and state bounds |x_k| <= 5 as
  2*N*nx rows of G; the Hessian and G are shared, q and g depend on x0.
* uneven_batch: many independent random_dense_qp instances of uneven n.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class QP:
    """One QP in the form of Sec. 2.

    Constraints: G u + g <= 0 when rlo/rhi are None; otherwise the user form
    rlo <= G u + g <= rhi (row-wise, -inf / +inf for an absent side, rlo = rhi
    an equality).  `eq` marks rows of G u + g that are equalities (K_i = {0})
    for a problem already written in cone form."""
    Q: np.ndarray          # (n, n) float64, symmetric
    q: np.ndarray          # (n,)
    G: np.ndarray          # (p, n)
    g: np.ndarray          # (p,)
    lb: np.ndarray         # (n,)
    ub: np.ndarray         # (n,)
    meta: dict = field(default_factory=dict)
    rlo: Optional[np.ndarray] = None
    rhi: Optional[np.ndarray] = None
    eq: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.Q.shape[0])

    @property
    def p(self) -> int:
        return int(self.G.shape[0])

    def rounded(self, dtype) -> "QP":
        """Same QP with Q and G rounded (RNE) to `dtype` and promoted back.

        The FP32 storage path solves exactly this problem."""
        Q = self.Q.astype(dtype).astype(np.float64)
        G = self.G.astype(dtype).astype(np.float64)
        cp = lambda v: None if v is None else v.copy()
        return QP(Q, self.q.copy(), G, self.g.copy(), self.lb.copy(),
                  self.ub.copy(), dict(self.meta, storage=np.dtype(dtype).name),
                  cp(self.rlo), cp(self.rhi), cp(self.eq))


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.Generator):
        return seed
    return np.random.default_rng(seed)


def random_dense_qp(n: int, p: int, seed=0, reg: float = 0.1,
                    box: float = 1.0, s_lo: float = 0.1,
                    s_hi: float = 1.0) -> QP:
    """Random dense strongly convex QP with a strictly feasible point."""
    rng = _rng(seed)
    A = rng.standard_normal((2 * n, n))
    Q = (A.T @ A) / n
    del A
    Q = 0.5 * (Q + Q.T)
    Q[np.diag_indices(n)] += reg
    q = rng.standard_normal(n)
    G = rng.standard_normal((p, n))
    x0 = rng.uniform(-0.5, 0.5, n)
    s = rng.uniform(s_lo, s_hi, p)
    g = -(G @ x0) - s
    lb = np.full(n, -box)
    ub = np.full(n, box)
    return QP(Q, q, G, g, lb, ub,
              dict(kind="random_dense", n=n, p=p, reg=reg,
                   seed=seed if not isinstance(seed, np.random.Generator) else None))


def fresh_linear_terms(G: np.ndarray, seed, s_lo: float = 0.1, s_hi: float = 1.0):
    """New (q, g) for fixed Q, G, drawn like random_dense_qp: q ~ N(0, I),
    g = -(G x0) - s with x0 ~ U(-1/2, 1/2)^n, s ~ U(s_lo, s_hi)^p (x0 strictly
    feasible)."""
    rng = _rng(seed)
    p, n = G.shape
    q = rng.standard_normal(n)
    x0 = rng.uniform(-0.5, 0.5, n)
    s = rng.uniform(s_lo, s_hi, p)
    return q, -(G @ x0) - s


def separable_terms(n: int, seed=7, box: float = 1.0):
    """Diagonal QP with one dense constraint row, drawn so that the row is
    active: d ~ U(1, 2) (Q = diag(d)), a ~ N(0, 1), q = -d * (0.8 sign(a) + 0.1 z)
    with z ~ N(0, 1), and b = a^T x0 + s with x0 ~ U(-1/2, 1/2)^n, s ~ U(0.1, 1)
    (x0 strictly feasible); the row is a^T u - b <= 0, box [-box, box].
    Draw order d, a, z, x0, s.  Returns (d, q, a, b, lb, ub); Q is never formed
    here, so n can be as large as the device allows."""
    rng = _rng(seed)
    d = rng.uniform(1.0, 2.0, n)
    a = rng.standard_normal(n)
    z = rng.standard_normal(n)
    q = -d * (0.8 * np.sign(a) + 0.1 * z)
    x0 = rng.uniform(-0.5, 0.5, n)
    s = rng.uniform(0.1, 1.0)
    b = float(a @ x0 + s)
    return d, q, a, b, np.full(n, -box), np.full(n, box)


def separable_qp(n: int, seed=7) -> QP:
    """separable_terms as a dense QP (small n)."""
    d, q, a, b, lb, ub = separable_terms(n, seed)
    return QP(np.diag(d), q, a[None, :].copy(), np.array([-b]), lb, ub,
              dict(kind="separable", n=n, p=1, seed=seed))


def infeasible_qp(kind: str, seed=1, n: int = 5) -> QP:
    """Small strongly convex QP whose constraints have no solution in the box
    [-1, 1]^n.  kind "pair": rows a and -a with g = (0.3, 0.2) (their sum
    reads 0.5 <= 0) plus a slack row; kind "triple": rows b1, b2, -(b1 + b2)
    with g = (0.1, 0.2, 0.3) (their sum reads 0.6 <= 0).  Q = A^T A / n + I/2
    with A ~ N(0,1)^{n x n}, q ~ N(0, 1).  Draw order A, q, then the rows."""
    rng = _rng(seed)
    A = rng.standard_normal((n, n))
    Q = A.T @ A / n + 0.5 * np.eye(n)
    q = rng.standard_normal(n)
    if kind == "pair":
        a = rng.standard_normal(n)
        G = np.stack([a, -a, rng.standard_normal(n)])
        g = np.array([0.3, 0.2, -5.0])
    else:
        B = rng.standard_normal((2, n))
        G = np.stack([B[0], B[1], -(B[0] + B[1])])
        g = np.array([0.1, 0.2, 0.3])
    return QP(Q, q, G, g, -np.ones(n), np.ones(n), dict(kind="infeasible_" + kind, n=n, p=3, seed=seed))


def random_eq_qp(n: int, p: int, seed=0, rank: Optional[int] = None, reg: float = 0.0,
                 box: float = 1.0) -> QP:
    """Equality-constrained dense QP (Sec. 2 with K = {0}; the QP class of the
    paper's Sec. 6 CPU-time study): Q = A^T A / n + reg I with A (rank x n)
    i.i.d. N(0,1), so Q is singular when rank < n and reg = 0 (Sec. 2, Case 2);
    q ~ N(0,1); G (p x n) i.i.d. N(0,1); g = -(G x0) with x0 ~ U(-box/2, box/2),
    so x0 is feasible and interior to the box.  Returned in the user form
    rlo = rhi = 0.  Draw order: A, q, G, x0."""
    rng = _rng(seed)
    r = n if rank is None else rank
    A = rng.standard_normal((r, n))
    Q = A.T @ A / n + reg * np.eye(n)
    Q = 0.5 * (Q + Q.T)
    q = rng.standard_normal(n)
    G = rng.standard_normal((p, n))
    x0 = rng.uniform(-0.5 * box, 0.5 * box, n)
    g = -(G @ x0)
    z = np.zeros(p)
    return QP(Q, q, G, g, -box * np.ones(n), box * np.ones(n), dict(kind="eq", seed=seed), z.copy(), z.copy())


def random_rows_qp(n: int, p: int, seed=0, reg: float = 0.1) -> QP:
    """Dense QP in the user form rlo <= G u + g <= rhi (Sec. 2) with every
    kind of row: row i draws its kind uniformly from {equality, upper side
    only, lower side only, both sides}.  Q = A^T A / n + reg I (A 2n x n),
    q ~ N(0,1), G ~ N(0,1), x0 ~ U(-.5,.5), g = -(G x0); sides at distance
    s ~ U(0.1, 1) from G x0 + g = 0 (an equality row at 0), so x0 satisfies
    every inequality strictly.  Draw order: A, q, G, x0, kinds, s_lo, s_hi."""
    rng = _rng(seed)
    A = rng.standard_normal((2 * n, n))
    Q = A.T @ A / n + reg * np.eye(n)
    Q = 0.5 * (Q + Q.T)
    q = rng.standard_normal(n)
    G = rng.standard_normal((p, n))
    x0 = rng.uniform(-0.5, 0.5, n)
    g = -(G @ x0)
    kind = rng.integers(0, 4, p)
    s_lo = rng.uniform(0.1, 1.0, p)
    s_hi = rng.uniform(0.1, 1.0, p)
    rlo = np.where((kind == 2) | (kind == 3), -s_lo, -np.inf)
    rhi = np.where((kind == 1) | (kind == 3), s_hi, np.inf)
    rlo = np.where(kind == 0, 0.0, rlo)
    rhi = np.where(kind == 0, 0.0, rhi)
    return QP(Q, q, G, g, -np.ones(n), np.ones(n), dict(kind="rows", seed=seed), rlo, rhi)


@dataclass
class CSR:
    """A matrix in compressed sparse row form (row pointers int64, column
    indices int32 in ascending order within each row, values)."""
    rows: int
    cols: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def dense(self) -> np.ndarray:
        """The dense matrix; a repeated index in a row adds its values."""
        M = np.zeros((self.rows, self.cols), dtype=np.float64)
        rows = np.repeat(np.arange(self.rows), np.diff(self.rowptr))
        np.add.at(M, (rows, self.col), self.val.astype(np.float64))
        return M


def to_csr(M: np.ndarray, dtype=np.float64) -> CSR:
    """The nonzero entries of a dense matrix, row by row."""
    rows, cols = M.shape
    nzr, nzc = np.nonzero(M)
    rowptr = np.zeros(rows + 1, np.int64)
    np.add.at(rowptr, nzr + 1, 1)
    rowptr = np.cumsum(rowptr)
    return CSR(rows, cols, rowptr, nzc.astype(np.int32), M[nzr, nzc].astype(dtype))


@dataclass
class SparseQP:
    """A QP with compressed-row Q (n x n) and G (p x n); the vectors as in QP."""
    Q: CSR
    q: np.ndarray
    G: CSR
    g: np.ndarray
    lb: np.ndarray
    ub: np.ndarray
    meta: dict

    @property
    def n(self) -> int:
        return self.Q.rows

    @property
    def p(self) -> int:
        return self.G.rows

    def dense(self) -> QP:
        return QP(self.Q.dense(), self.q, self.G.dense(), self.g, self.lb, self.ub, dict(self.meta))


def _routes(rng, n: int, p: int, k: int) -> np.ndarray:
    """n rows of k distinct link ids in [0, p): redraw the rows that repeat."""
    R = rng.integers(0, p, size=(n, k))
    while True:
        S = np.sort(R, axis=1)
        bad = (np.diff(S, axis=1) == 0).any(axis=1) if k > 1 else np.zeros(n, bool)
        if not bad.any():
            return S
        R = S
        R[bad] = rng.integers(0, p, size=(int(bad.sum()), k))


def sparse_num_qp(n: int, p: int, seed=0, path_len: int = 8, band: int = 2, cap_slack: float = 0.3) -> SparseQP:
    """A sparse QP shaped like network utility maximisation (the sparse
    application Sec. 2 and Sec. 5.1 name): n flows with rates u in [0, 1], p
    links; G (p x n) is the 0/1 routing matrix, each flow crossing `path_len`
    distinct random links; G u <= c with c = G x0 + slack (x0 ~ U(0.2, 0.6),
    slack ~ U(0, cap_slack)), written as G u + g <= 0 with g = -c.  The
    objective is a concave quadratic utility to maximise, i.e. F = 1/2 u^T Q u
    + q^T u with Q = diag(d) + a symmetric band coupling neighbouring flows
    (d ~ U(1, 2), off-diagonals ~ U(-0.1, 0.1) within `band`, Q > 0 by
    diagonal dominance) and q ~ -U(0.5, 1.5).  Draw order: routes (rows of
    link ids, redrawn where a flow repeats a link), x0, slack, d, the
    off-diagonals of distance 1..band, q.  Built in compressed-row form
    without dense matrices, so it serves sizes far beyond dense memory."""
    if path_len > p:
        raise ValueError("path_len must not exceed p")
    rng = _rng(seed)
    R = _routes(rng, n, p, path_len)
    x0 = rng.uniform(0.2, 0.6, n)
    slack = rng.uniform(0.0, cap_slack, p)
    d = rng.uniform(1.0, 2.0, n)
    offs = [rng.uniform(-0.1, 0.1, n - k) if n > k else np.zeros(0) for k in range(1, band + 1)]
    q = -rng.uniform(0.5, 1.5, n)
    # G: entry (link, flow) = 1, rows ordered by link, flows ascending inside
    links = R.ravel()
    flows = np.repeat(np.arange(n, dtype=np.int64), path_len)
    order = np.lexsort((flows, links))
    grp = np.zeros(p + 1, np.int64)
    np.add.at(grp, links + 1, 1)
    G = CSR(p, n, np.cumsum(grp), flows[order].astype(np.int32), np.ones(links.size))
    g = -(np.bincount(links, weights=x0[flows], minlength=p) + slack)
    # Q: band rows, columns ascending
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [d]
    for k, off in enumerate(offs, start=1):
        i = np.arange(n - k)
        rows += [i, i + k]
        cols += [i + k, i]
        vals += [off, off]
    r, c, v = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    o = np.lexsort((c, r))
    qrp = np.zeros(n + 1, np.int64)
    np.add.at(qrp, r + 1, 1)
    Qm = CSR(n, n, np.cumsum(qrp), c[o].astype(np.int32), v[o])
    return SparseQP(Qm, q, G, g, np.zeros(n), np.ones(n), dict(kind="num", seed=seed, path_len=path_len, band=band))


def config0() -> QP:
    """Small dense QP: n=50, p=25, reg 0.1, seed 0."""
    return random_dense_qp(50, 25, seed=0, reg=0.1)


def config1(n: int = 8192, p: int = 4096, seed: int = 1) -> QP:
    """Large dense QP: n=8192, p=4096, reg 0.01, seed 1 (smaller n for tests)."""
    return random_dense_qp(n, p, seed=seed, reg=0.01)


# ----------------------------------------------------------------------------
# Condensed linear MPC (shared Hessian, per-instance linear terms)
# ----------------------------------------------------------------------------

@dataclass
class MPCSystem:
    Ad: np.ndarray        # (nx, nx)
    Bd: np.ndarray        # (nx, nu)
    Gamma: np.ndarray     # (N*nx, N*nu)  stacked input-to-state map
    Phi: np.ndarray       # (N*nx, nx)    stacked free response
    H: np.ndarray         # (n, n) shared Hessian
    G: np.ndarray         # (2*N*nx, n) shared constraint matrix
    lb: np.ndarray
    ub: np.ndarray
    xmax: float
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.H.shape[0])

    @property
    def p(self) -> int:
        return int(self.G.shape[0])


def mpc_system(seed=2, nx: int = 12, nu: int = 4, N: int = 30,
               rho_spec: float = 0.95, xmax: float = 5.0, umax: float = 1.0,
               r_weight: float = 0.1, max_tries: int = 100000) -> MPCSystem:
    """Random condensed MPC system.

    A_d ~ N(0,1) scaled to spectral radius `rho_spec`, resampled until
    max_{k<=N} ||A_d^k||_inf < xmax so that u = 0 is strictly feasible
    for every |x0|_inf <= 1.  B_d ~ N(0,1)/2.  Stage cost x^T x and
    r_weight*u^T u, terminal cost x^T x (constant term dropped).
    """
    rng = _rng(seed)
    for _ in range(max_tries):
        Ad = rng.standard_normal((nx, nx))
        Ad *= rho_spec / np.max(np.abs(np.linalg.eigvals(Ad)))
        P = np.eye(nx)
        ok = True
        for _k in range(N):
            P = Ad @ P
            if np.max(np.sum(np.abs(P), axis=1)) >= xmax:
                ok = False
                break
        if ok:
            break
    else:  # pragma: no cover - the recipe accepts quickly in practice
        raise RuntimeError("mpc_system: no admissible A_d found")
    Bd = rng.standard_normal((nx, nu)) / 2.0
    n = N * nu
    Gamma = np.zeros((N * nx, n))
    Phi = np.zeros((N * nx, nx))
    Apow = [np.eye(nx)]
    for _k in range(N):
        Apow.append(Ad @ Apow[-1])
    for k in range(1, N + 1):          # state x_k, rows (k-1)*nx
        Phi[(k - 1) * nx:k * nx, :] = Apow[k]
        for j in range(k):             # input u_j, cols j*nu
            Gamma[(k - 1) * nx:k * nx, j * nu:(j + 1) * nu] = Apow[k - 1 - j] @ Bd
    H = Gamma.T @ Gamma
    H = 0.5 * (H + H.T)
    H[np.diag_indices(n)] += r_weight
    G = np.vstack([Gamma, -Gamma])
    lb = np.full(n, -umax)
    ub = np.full(n, umax)
    return MPCSystem(Ad, Bd, Gamma, Phi, H, G, lb, ub, xmax,
                     dict(kind="mpc", nx=nx, nu=nu, N=N,
                          seed=seed if not isinstance(seed, np.random.Generator) else None))


def mpc_linear_terms(sys: MPCSystem, x0: np.ndarray):
    """q and g of one MPC instance with initial state x0."""
    fx = sys.Phi @ x0
    q = sys.Gamma.T @ fx
    g = np.concatenate([fx - sys.xmax, -fx - sys.xmax])
    return q, g


def mpc_batch(sys: MPCSystem, B: int, seed=20):
    """B initial states x0 ~ U(-1,1)^nx and their (q, g); returns (X0, Qlin, Glin)."""
    rng = _rng(seed)
    nx = sys.Ad.shape[0]
    X0 = rng.uniform(-1.0, 1.0, (B, nx))
    FX = X0 @ sys.Phi.T                                  # (B, N*nx)
    Qlin = FX @ sys.Gamma                                # (B, n)
    Glin = np.concatenate([FX - sys.xmax, -FX - sys.xmax], axis=1)
    return X0, Qlin, Glin


def mpc_instance(sys: MPCSystem, x0: np.ndarray) -> QP:
    q, g = mpc_linear_terms(sys, x0)
    return QP(sys.H.copy(), q, sys.G.copy(), g, sys.lb.copy(), sys.ub.copy(),
              dict(kind="mpc_instance"))


# ----------------------------------------------------------------------------
# Uneven independent batch
# ----------------------------------------------------------------------------

@dataclass
class UnevenBatch:
    """Packed batch of independent QPs of different sizes.

    Q of instance i is rows [qoff[i], qoff[i]+n_i*n_i) of the flat array
    `Q` (row-major n_i x n_i), G likewise at goff[i] (p_i x n_i), vectors
    q/lb/ub at voff[i] (n_i) and g at coff[i] (p_i)."""
    n: np.ndarray
    p: np.ndarray
    Q: np.ndarray
    G: np.ndarray
    q: np.ndarray
    g: np.ndarray
    lb: np.ndarray
    ub: np.ndarray
    qoff: np.ndarray
    goff: np.ndarray
    voff: np.ndarray
    coff: np.ndarray

    @property
    def B(self) -> int:
        return int(self.n.shape[0])

    def instance(self, i: int) -> QP:
        n, p = int(self.n[i]), int(self.p[i])
        Q = self.Q[self.qoff[i]:self.qoff[i] + n * n].reshape(n, n).astype(np.float64)
        G = self.G[self.goff[i]:self.goff[i] + p * n].reshape(p, n).astype(np.float64)
        sl = slice(self.voff[i], self.voff[i] + n)
        sc = slice(self.coff[i], self.coff[i] + p)
        return QP(Q, self.q[sl].copy(), G, self.g[sc].copy(),
                  self.lb[sl].copy(), self.ub[sl].copy(), dict(kind="uneven", index=i))


def pack_uneven(qps, dtype=np.float64) -> "UnevenBatch":
    """Pack a list of QPs into an UnevenBatch (instances in list order)."""
    n = np.array([qp.n for qp in qps], dtype=np.int32)
    p = np.array([qp.p for qp in qps], dtype=np.int32)
    off = lambda sizes: np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)[:len(sizes)]
    n64, p64 = n.astype(np.int64), p.astype(np.int64)
    cat = lambda parts, dt=np.float64: (np.concatenate(parts).astype(dt) if parts else np.zeros(0, dt))
    return UnevenBatch(n, p, cat([qp.Q.ravel() for qp in qps], dtype), cat([qp.G.ravel() for qp in qps], dtype),
                       cat([qp.q for qp in qps]), cat([qp.g for qp in qps]), cat([qp.lb for qp in qps]),
                       cat([qp.ub for qp in qps]), off(n64 * n64), off(p64 * n64), off(n64), off(p64))


def _uneven_chunk(args):
    children, ns, ps, reg, dtype = args
    out = []
    try:   # small products: one BLAS thread per worker is fastest
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(1)
    except Exception:  # pragma: no cover
        limiter = None
    for ch, n, p in zip(children, ns, ps):
        qp = random_dense_qp(int(n), int(p), seed=np.random.default_rng(ch), reg=reg)
        out.append((qp.Q.astype(dtype).ravel(), qp.G.astype(dtype).ravel(), qp.q, qp.g, qp.lb, qp.ub))
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else limiter.restore_original_limits()
    return out


def uneven_batch(B: int = 10000, seed: int = 3, n_lo: int = 20, n_hi: int = 512,
                 reg: float = 0.1, dtype=np.float32, workers: int = 1) -> UnevenBatch:
    """B random_dense_qp instances with n ~ U{n_lo..n_hi}, p = n // 2.

    Instance i draws from SeedSequence(seed).spawn(B + 1)[i + 1]; sizes come
    from child 0.  `workers` > 1 draws instances in parallel processes (the
    result does not depend on it)."""
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(B + 1)
    size_rng = np.random.default_rng(children[0])
    ns = size_rng.integers(n_lo, n_hi + 1, size=B).astype(np.int64)
    ps = ns // 2
    qoff = np.zeros(B, np.int64)
    goff = np.zeros(B, np.int64)
    voff = np.zeros(B, np.int64)
    coff = np.zeros(B, np.int64)
    qoff[1:] = np.cumsum(ns * ns)[:-1]
    goff[1:] = np.cumsum(ps * ns)[:-1]
    voff[1:] = np.cumsum(ns)[:-1]
    coff[1:] = np.cumsum(ps)[:-1]
    Qf = np.empty(int((ns * ns).sum()), dtype)
    Gf = np.empty(int((ps * ns).sum()), dtype)
    qf = np.empty(int(ns.sum()))
    gf = np.empty(int(ps.sum()))
    lbf = np.empty(int(ns.sum()))
    ubf = np.empty(int(ns.sum()))
    chunks = [(children[1 + a:1 + min(B, a + 256)], ns[a:a + 256], ps[a:a + 256], reg, dtype)
              for a in range(0, B, 256)]
    if workers > 1 and B > 256:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_uneven_chunk, chunks)
    else:
        parts = [_uneven_chunk(c) for c in chunks]
    i = 0
    for part in parts:
        for Qi, Gi, qi, gi, lbi, ubi in part:
            n, p = int(ns[i]), int(ps[i])
            Qf[qoff[i]:qoff[i] + n * n] = Qi
            Gf[goff[i]:goff[i] + p * n] = Gi
            qf[voff[i]:voff[i] + n] = qi
            lbf[voff[i]:voff[i] + n] = lbi
            ubf[voff[i]:voff[i] + n] = ubi
            gf[coff[i]:coff[i] + p] = gi
            i += 1
    return UnevenBatch(ns, ps, Qf, Gf, qf, gf, lbf, ubf, qoff, goff, voff, coff)
