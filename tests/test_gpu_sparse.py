"""GPU parity of the compressed-row path (duq_setup_csr: sparse Q and G, whose
products cost their nonzeros, Sec. 5.1) through the C ABI, against the FP64
oracle run on the same matrices in dense form.  The GPU sums each product row
over its nonzeros only, in another order than the oracle's dense products, so
iterates agree to rounding (1e-9 relative), inner counts exactly."""
import math

import numpy as np
import pytest

from oracle import dfom
from paper_1504_05708_amd import duq, gen

pytestmark = pytest.mark.gpu

REL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    duq.lib()


def close(a, b, rel=REL, what=""):
    a, b = np.asarray(a, float), np.asarray(b, float)
    if a.size == 0:
        return
    scale = max(1.0, float(np.max(np.abs(b))))
    err = float(np.max(np.abs(a - b)))
    assert err <= rel * scale, f"{what}: max err {err:.3e} > {rel:.1e} * {scale:.3e}"


def with_dtype(sq, dtype):
    """The sparse QP with Q and G values stored in `dtype`, and its dense form
    with the same (rounded) values for the oracle."""
    Q = gen.CSR(sq.Q.rows, sq.Q.cols, sq.Q.rowptr, sq.Q.col, sq.Q.val.astype(dtype))
    G = gen.CSR(sq.G.rows, sq.G.cols, sq.G.rowptr, sq.G.col, sq.G.val.astype(dtype))
    s2 = gen.SparseQP(Q, sq.q, G, sq.g, sq.lb, sq.ub, dict(sq.meta))
    return s2, s2.dense()


def sparse_solver(sq, c, rlo=None, rhi=None, **kw):
    kw.setdefault("lam_min", c.lam_min)
    kw.setdefault("lam_max", c.lam_max)
    kw.setdefault("G_norm2", c.G_norm2 if sq.p else 0.0)
    return duq.Solver(sq.Q, sq.q, sq.G if sq.p else None, sq.g, sq.lb, sq.ub, rlo=rlo, rhi=rhi, **kw)


def compare_trace(tr, log, K, what):
    S = tr["scalars"]
    assert S.shape[0] == K
    for k in range(K):
        e = log[k]
        assert int(S[k, 1]) == e["t"], f"{what}: inner count differs at k={k + 1}: {int(S[k, 1])} vs {e['t']}"
        close(tr["lam"][k], e["lam"], what=f"{what} lambda^{k + 1}")
        close(tr["mu"][k], e["mu"], what=f"{what} mu^{k + 1}")
        close(tr["u"][k], e["u"], what=f"{what} ubar^{k + 1}")
        sc = max(1.0, abs(e["dbar"]))
        assert abs(S[k, 3] - e["dbar"]) <= REL * sc, (what, k)
        assert abs(S[k, 2] - e["gap"]) <= REL * sc, (what, k)
        if math.isfinite(e["LB"]):
            assert abs(S[k, 4] - e["LB"]) <= REL * sc, (what, k)


def run_sparse_trace(sq, method, output, rho=0.0, K=200, engine=duq.ENGINE_AUTO, dtype=np.float64,
                     eps_in=1e-6, sparse_x=duq.SPX_AUTO):
    sq, qp = with_dtype(sq, dtype)
    c = dfom.problem_constants(qp.Q, qp.G, qp.lb, qp.ub, rho, eps_in)
    ref = dfom.dfom_solve(qp, dfom.Options(method=method, output=output, rho=rho, eps_out=1e-13, eps_in=eps_in,
                                           max_outer=K, log_vectors=K), consts=c)
    with sparse_solver(sq, c, method=method, output=output, rho=rho, eps_out=1e-13, eps_in=eps_in,
                       max_outer=K, trace_outer=K, engine=engine, sparse_x=sparse_x) as s:
        x, lam, res = s.solve(check=False)
        tr = s.trace(K)
    what = f"sparse n={sq.n} p={sq.p} m={method} o={output} rho={rho} engine={engine} x={sparse_x}"
    assert res["outer_iters"] == ref.outer_iters == K, what
    compare_trace(tr, ref.log, K, what)
    assert res["inner_iters"] == ref.inner_iters, what
    close(x, ref.x, what=f"{what} x")
    close(lam, ref.lam, what=f"{what} lambda")
    return ref, res


@pytest.mark.parametrize("engine", [duq.ENGINE_BLOCK, duq.ENGINE_GRID])
@pytest.mark.parametrize("method,output", [(duq.DFGM, duq.LAST), (duq.DGM, duq.AVG)])
def test_sparse_trace_parity(engine, method, output):
    print(f"[case] sparse trace engine={engine} m={method} o={output}", flush=True)
    sq = gen.sparse_num_qp(300, 120, seed=401)
    run_sparse_trace(sq, method, output, K=200, engine=engine)


@pytest.mark.parametrize("engine", [duq.ENGINE_BLOCK, duq.ENGINE_GRID])
@pytest.mark.parametrize("method,output", [(duq.DFGM, duq.LAST), (duq.DGM, duq.AVG)])
def test_sparse_in_place_trace_parity(engine, method, output):
    # x read from device memory by the products instead of an LDS copy
    print(f"[case] sparse in place engine={engine} m={method} o={output}", flush=True)
    sq = gen.sparse_num_qp(300, 120, seed=401)
    run_sparse_trace(sq, method, output, K=200, engine=engine, sparse_x=duq.SPX_IN_PLACE)


@pytest.mark.parametrize("engine", [duq.ENGINE_BLOCK, duq.ENGINE_GRID])
def test_sparse_in_place_augmented_fp32(engine):
    print(f"[case] sparse in place rho=0.5 fp32 engine={engine}", flush=True)
    sq = gen.sparse_num_qp(260, 100, seed=413)
    run_sparse_trace(sq, duq.DFGM, duq.LAST, rho=0.5, K=60, engine=engine, dtype=np.float32,
                     sparse_x=duq.SPX_IN_PLACE)


@pytest.mark.parametrize("n,p", [(4000, 1500), (16000, 5000)])
def test_sparse_in_place_bitwise_equals_lds(n, p):
    # the two ways of reading x (a staged LDS copy; plain loads of the buffer
    # itself after an acquire) feed the same sums in the same order: every
    # traced iterate must be bitwise equal, so a stale read would show here
    print(f"[case] sparse in place vs LDS n={n}", flush=True)
    sq = gen.sparse_num_qp(n, p, seed=414)
    K = 150
    out = []
    for mode in (duq.SPX_LDS, duq.SPX_IN_PLACE):
        with duq.Solver(sq.Q, sq.q, sq.G, sq.g, sq.lb, sq.ub, eps_out=1e-13, eps_in=1e-8, max_outer=K,
                        trace_outer=K, engine=duq.ENGINE_GRID, sparse_x=mode, rho=0.0) as s:
            x, lam, res = s.solve(check=False)
            out.append((x, lam, res, s.trace(K)))
    (x0, l0, r0, t0), (x1, l1, r1, t1) = out
    assert r0["outer_iters"] == r1["outer_iters"] == K and r0["inner_iters"] == r1["inner_iters"]
    assert np.array_equal(x0, x1) and np.array_equal(l0, l1)
    for key in ("lam", "mu", "u", "scalars"):
        assert np.array_equal(t0[key], t1[key]), key


def test_sparse_in_place_grid_medium_parity():
    print("[case] sparse in place grid n=4000", flush=True)
    sq = gen.sparse_num_qp(4000, 1500, seed=403)
    run_sparse_trace(sq, duq.DFGM, duq.LAST, K=30, engine=duq.ENGINE_GRID, sparse_x=duq.SPX_IN_PLACE)


@pytest.mark.parametrize("engine", [duq.ENGINE_BLOCK, duq.ENGINE_GRID])
def test_sparse_augmented_trace_parity(engine):
    # rho > 0: every inner step reads G y and G^T w through the sparse products
    print(f"[case] sparse rho=0.5 engine={engine}", flush=True)
    sq = gen.sparse_num_qp(260, 100, seed=402)
    run_sparse_trace(sq, duq.DFGM, duq.LAST, rho=0.5, K=60, engine=engine)


def test_sparse_grid_medium_parity():
    print("[case] sparse grid n=4000", flush=True)
    sq = gen.sparse_num_qp(4000, 1500, seed=403)
    run_sparse_trace(sq, duq.DFGM, duq.LAST, K=30, engine=duq.ENGINE_GRID)


@pytest.mark.parametrize("engine", [duq.ENGINE_BLOCK, duq.ENGINE_GRID])
def test_sparse_fp32_storage_parity(engine):
    print(f"[case] sparse FP32 storage engine={engine}", flush=True)
    sq = gen.sparse_num_qp(300, 120, seed=404)
    run_sparse_trace(sq, duq.DFGM, duq.LAST, K=100, engine=engine, dtype=np.float32)


@pytest.mark.parametrize("n,p", [(1, 1), (9, 8), (65, 8), (129, 300)])
def test_sparse_ragged_shapes_parity(n, p):
    # few rows, links no flow uses (empty rows of G), more links than flows
    print(f"[case] sparse ragged n={n} p={p}", flush=True)
    sq = gen.sparse_num_qp(n, p, seed=405, path_len=min(8, p), band=min(2, max(n - 1, 0)))
    for engine in (duq.ENGINE_BLOCK, duq.ENGINE_GRID):
        run_sparse_trace(sq, duq.DFGM, duq.LAST, K=40, engine=engine)


def test_sparse_unordered_and_repeated_entries():
    # any order inside a row and a repeated index (its values add) give the
    # same problem: compare with the oracle on the summed dense matrices
    print("[case] sparse unordered entries", flush=True)
    sq = gen.sparse_num_qp(200, 80, seed=406)
    rng = np.random.default_rng(7)

    def scramble(M):
        rp, ci, v = [0], [], []
        for i in range(M.rows):
            a, b = int(M.rowptr[i]), int(M.rowptr[i + 1])
            cols, vals = list(M.col[a:b]), list(M.val[a:b])
            if cols:   # split the first entry into two halves
                cols.append(cols[0])
                vals[0] *= 0.5
                vals.append(vals[0])
            o = rng.permutation(len(cols))
            ci += [cols[j] for j in o]
            v += [vals[j] for j in o]
            rp.append(len(ci))
        return gen.CSR(M.rows, M.cols, np.array(rp, np.int64), np.array(ci, np.int32), np.array(v))

    s2 = gen.SparseQP(scramble(sq.Q), sq.q, scramble(sq.G), sq.g, sq.lb, sq.ub, dict(sq.meta))
    close(s2.Q.dense(), sq.Q.dense(), rel=1e-15, what="scrambled Q")
    run_sparse_trace(s2, duq.DFGM, duq.LAST, K=100, engine=duq.ENGINE_BLOCK)


def test_sparse_without_rows():
    # p = 0: a box-constrained QP, the inner solve alone
    print("[case] sparse p=0", flush=True)
    sq = gen.sparse_num_qp(150, 10, seed=407)
    qp = sq.dense()
    c = dfom.problem_constants(qp.Q, np.zeros((0, qp.n)), qp.lb, qp.ub, 0.0, 1e-10)
    ref = dfom.dfom_solve(gen.QP(qp.Q, qp.q, np.zeros((0, qp.n)), np.zeros(0), qp.lb, qp.ub, {}),
                          dfom.Options(eps_out=1e-6, eps_in=1e-10, max_outer=10), consts=c)
    with duq.Solver(sq.Q, sq.q, None, None, sq.lb, sq.ub, eps_out=1e-6, eps_in=1e-10, max_outer=10,
                    lam_min=c.lam_min, lam_max=c.lam_max, G_norm2=0.0) as s:
        x, _, res = s.solve()
    assert res["inner_iters"] == ref.inner_iters
    close(x, ref.x, what="p=0 x")


def test_sparse_rows_trace_parity():
    # the user form rlo <= G u + g <= rhi on sparse G: equalities, two-sided
    # rows and upper rows, against the oracle on the stacked cone form
    print("[case] sparse rows", flush=True)
    sq = gen.sparse_num_qp(240, 90, seed=408)
    qp = sq.dense()
    p = qp.p
    rhi = np.zeros(p)
    rlo = np.full(p, -np.inf)
    rlo[::3] = -0.6            # two-sided: c - 0.6 <= G u <= c
    rlo[1:4] = 0.0             # three equalities G u = c
    Gs, gs, eq, src, sign = dfom.stack_rows(qp.G, qp.g, rlo, rhi)
    sqp = gen.QP(qp.Q, qp.q, Gs, gs, qp.lb, qp.ub, eq=eq)
    c = dfom.problem_constants(sqp.Q, sqp.G, sqp.lb, sqp.ub, 0.0, 1e-6, eq=eq)
    K = 150
    ref = dfom.dfom_solve(sqp, dfom.Options(eps_out=1e-13, eps_in=1e-6, max_outer=K, log_vectors=K), consts=c)
    with sparse_solver(sq, c, rlo=rlo, rhi=rhi, eps_out=1e-13, eps_in=1e-6, max_outer=K, trace_outer=K,
                       engine=duq.ENGINE_BLOCK) as s:
        x, nu, res = s.solve(check=False)
        tr = s.trace(K)
    assert res["outer_iters"] == K and res["inner_iters"] == ref.inner_iters
    for k in range(K):
        e = ref.log[k]
        assert int(tr["scalars"][k, 1]) == e["t"], k
        lp = np.zeros(p)
        lm = np.zeros(p)
        lp[src[sign > 0]] = e["lam"][sign > 0]
        lm[src[sign < 0]] = e["lam"][sign < 0]
        close(tr["lam"][k], lp, what=f"lambda+^{k + 1}")
        close(tr["lam_lo"][k], lm, what=f"lambda-^{k + 1}")
        close(tr["u"][k], e["u"], what=f"ubar^{k + 1}")
    close(x, ref.x, what="rows x")


@pytest.mark.timeout(300)
@pytest.mark.parametrize("engine", [duq.ENGINE_BLOCK, duq.ENGINE_GRID])
def test_sparse_converged_solution_matches_oracle(engine):
    print(f"[case] sparse converged engine={engine}", flush=True)
    sq = gen.sparse_num_qp(300, 120, seed=409)
    qp = sq.dense()
    c = dfom.problem_constants(qp.Q, qp.G, qp.lb, qp.ub, 0.0, 1e-8)
    ref = dfom.dfom_solve(qp, dfom.Options(method=dfom.DFGM, eps_out=1e-5, eps_in=1e-8, max_outer=100000), consts=c)
    with sparse_solver(sq, c, method=duq.DFGM, eps_out=1e-5, eps_in=1e-8, max_outer=100000, engine=engine) as s:
        x, lam, res = s.solve()
    assert res["status"] == duq.DUQ_OK and ref.status == dfom.STATUS_OK
    assert res["outer_iters"] == ref.outer_iters and res["inner_iters"] == ref.inner_iters
    close(x, ref.x, rel=1e-8, what="converged x")
    assert res["f"] == pytest.approx(ref.F, rel=1e-9)


@pytest.mark.parametrize("engine", [duq.ENGINE_BLOCK, duq.ENGINE_GRID])
@pytest.mark.parametrize("sparse_x", [duq.SPX_LDS, duq.SPX_IN_PLACE])
def test_sparse_lanczos_constants(engine, sparse_x):
    # the Lanczos estimate through the sparse operators Q v and G^T (G v)
    print(f"[case] sparse lanczos engine={engine} x={sparse_x}", flush=True)
    sq = gen.sparse_num_qp(700, 250, seed=410)
    qp = sq.dense()
    ev = np.linalg.eigvalsh(qp.Q)
    g2 = np.linalg.norm(qp.G, 2) ** 2
    with duq.Solver(sq.Q, sq.q, sq.G, sq.g, sq.lb, sq.ub, engine=engine, lanczos_steps=96,
                    sparse_x=sparse_x) as s:
        c = s.constants()
    sf = 1.02
    assert c["lam_max"] >= ev[-1] and c["lam_max"] / sf == pytest.approx(ev[-1], rel=2e-3)
    assert c["lam_min"] <= ev[0] and c["lam_min"] * sf == pytest.approx(ev[0], rel=2e-2)
    assert c["G_norm2"] >= g2 and c["G_norm2"] / sf == pytest.approx(g2, rel=2e-3)


def test_sparse_matches_dense_path():
    # the same instance through duq_setup (dense) and duq_setup_csr agrees to rounding
    print("[case] sparse vs dense", flush=True)
    sq = gen.sparse_num_qp(400, 150, seed=411)
    qp = sq.dense()
    c = dfom.problem_constants(qp.Q, qp.G, qp.lb, qp.ub, 0.0, 1e-6)
    K = 300
    kw = dict(eps_out=1e-13, eps_in=1e-6, max_outer=K, trace_outer=K, lam_min=c.lam_min, lam_max=c.lam_max,
              G_norm2=c.G_norm2, engine=duq.ENGINE_GRID)
    with duq.Solver(qp.Q, qp.q, qp.G, qp.g, qp.lb, qp.ub, **kw) as s:
        xd, ld, rd = s.solve(check=False)
        td = s.trace(K)
    with duq.Solver(sq.Q, sq.q, sq.G, sq.g, sq.lb, sq.ub, **kw) as s:
        xs, ls, rs = s.solve(check=False)
        ts = s.trace(K)
    assert rd["outer_iters"] == rs["outer_iters"] == K and rd["inner_iters"] == rs["inner_iters"]
    for k in range(K):
        close(ts["lam"][k], td["lam"][k], what=f"lambda^{k + 1}")
        close(ts["u"][k], td["u"][k], what=f"ubar^{k + 1}")
    close(xs, xd, rel=1e-9, what="x")
    close(ls, ld, rel=1e-9, what="lambda")


@pytest.mark.timeout(600)
def test_sparse_maximum_size_kkt():
    # the largest n the grid engine stages (LDS bound of duq_max_n): too large
    # for the dense oracle, so the converged point is checked by the KKT
    # conditions of Sec. 2 evaluated with host sparse products
    p = 6000
    n = duq.max_n(p, duq.ENGINE_GRID)
    print(f"[case] sparse max size n={n} p={p}", flush=True)
    sq = gen.sparse_num_qp(n, p, seed=412)
    with duq.Solver(sq.Q, sq.q, sq.G, sq.g, sq.lb, sq.ub, eps_out=1e-5, eps_in=1e-8, max_outer=20000,
                    engine=duq.ENGINE_GRID) as s:
        x, lam, res = s.solve()
    assert res["status"] == duq.DUQ_OK, res

    def mv(M, v):
        out = np.zeros(M.rows)
        rows = np.repeat(np.arange(M.rows), np.diff(M.rowptr))
        np.add.at(out, rows, M.val * v[M.col])
        return out

    def mtv(M, w):
        out = np.zeros(M.cols)
        rows = np.repeat(np.arange(M.rows), np.diff(M.rowptr))
        np.add.at(out, M.col, M.val * w[rows])
        return out

    assert np.all(x >= sq.lb) and np.all(x <= sq.ub) and np.all(lam >= 0)
    r = mv(sq.G, x) + sq.g
    scale = max(1.0, float(np.linalg.norm(sq.g)))
    assert np.linalg.norm(np.maximum(r, 0)) <= 1e-3 * scale          # primal feasibility
    grad = mv(sq.Q, x) + sq.q + mtv(sq.G, lam)                           # stationarity on the box
    pg = x - np.clip(x - grad, sq.lb, sq.ub)
    assert np.linalg.norm(pg) <= 1e-2 * max(1.0, float(np.linalg.norm(sq.q)))
    # complementary slackness of the multipliers against the rows
    assert abs(float(lam @ r)) <= 1e-2 * max(1.0, abs(res["f"]))
    # the reported objective is that of the returned point
    F = 0.5 * float(x @ mv(sq.Q, x)) + float(sq.q @ x)
    assert res["f"] == pytest.approx(F, rel=1e-9, abs=1e-9)
