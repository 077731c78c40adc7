"""GPU tests of the shared-Hessian MFMA tile kernel (duq_solve_batch with
DUQ_ENGINE_TILE): parity with the FP64 oracle per instance, ragged tiles and
sizes, the same bits alone and in any tile position, agreement with the
one-workgroup-per-instance kernel."""
import numpy as np
import pytest

from oracle import dfom
from paper_1504_05708_amd import duq, gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    duq.lib()


def _consts(sysm):
    qp = gen.mpc_instance(sysm, np.zeros(sysm.Ad.shape[0]))
    c = dfom.problem_constants(qp.Q, qp.G, qp.lb, qp.ub, 0.0, 1e-6)
    return c.lam_min, c.lam_max, c.G_norm2


@pytest.mark.parametrize("N,method,output", [(10, duq.DFGM, duq.LAST), (7, duq.DGM, duq.LAST),
                                             (7, duq.DFGM, duq.AVG), (30, duq.DFGM, duq.LAST)])
def test_tile_matches_oracle(N, method, output):
    print(f"[case] tile parity N={N} method={method} output={output}", flush=True)
    sysm = gen.mpc_system(seed=2, N=N)
    B = 21   # two tiles, the second ragged
    X0, Qlin, Glin = gen.mpc_batch(sysm, B, seed=51)
    lmin, lmax, g2 = _consts(sysm)
    eps_in = 1e-8 if method == duq.DFGM else 1e-6
    X, Lam, res = duq.solve_batch_shared(sysm.H, sysm.G, sysm.lb, sysm.ub, Qlin, Glin,
                                         constants=(lmin, lmax, g2), engine=duq.ENGINE_TILE, method=method,
                                         output=output, eps_out=1e-4, eps_in=eps_in, max_outer=20000)
    for b in range(0, B, 4):
        qp = gen.mpc_instance(sysm, X0[b])
        ref = dfom.dfom_solve(qp, dfom.Options(method=dfom.DFGM if method == duq.DFGM else dfom.DGM,
                                               output=dfom.LAST if output == duq.LAST else dfom.AVG,
                                               eps_out=1e-4, eps_in=eps_in, max_outer=20000,
                                               lam_min=lmin, lam_max=lmax, G_norm2=g2))
        r = res[b]
        assert r["status"] == duq.DUQ_OK and r["engine"] == duq.ENGINE_TILE, (b, r)
        assert r["outer_iters"] == ref.outer_iters and r["inner_iters"] == ref.inner_iters, (b, r, ref.outer_iters)
        np.testing.assert_allclose(X[b], ref.x, rtol=0, atol=1e-7)
        np.testing.assert_allclose(Lam[b], ref.lam, rtol=0, atol=1e-7 * max(1.0, np.abs(ref.lam).max()))
        assert abs(r["f"] - ref.F) <= 1e-9 * max(1.0, abs(ref.F))


def test_tile_alone_equals_any_position_bitwise():
    print("[case] tile alone vs mix", flush=True)
    sysm = gen.mpc_system(seed=3, N=12)
    X0, Qlin, Glin = gen.mpc_batch(sysm, 40, seed=52)
    c = _consts(sysm)
    kw = dict(constants=c, engine=duq.ENGINE_TILE, method=duq.DFGM, eps_out=1e-4, eps_in=1e-8, max_outer=20000)
    X, Lam, res = duq.solve_batch_shared(sysm.H, sysm.G, sysm.lb, sysm.ub, Qlin, Glin, **kw)
    for b in (0, 17, 39):
        X1, L1, r1 = duq.solve_batch_shared(sysm.H, sysm.G, sysm.lb, sysm.ub, Qlin[b:b + 1], Glin[b:b + 1], **kw)
        assert np.array_equal(X1[0], X[b]) and np.array_equal(L1[0], Lam[b]), b
        assert r1[0]["outer_iters"] == res[b]["outer_iters"] and r1[0]["inner_iters"] == res[b]["inner_iters"]
    perm = np.random.default_rng(0).permutation(40)
    Xp, Lp, rp = duq.solve_batch_shared(sysm.H, sysm.G, sysm.lb, sysm.ub, Qlin[perm], Glin[perm], **kw)
    assert np.array_equal(Xp, X[perm]) and np.array_equal(Lp, Lam[perm])


def test_tile_agrees_with_block_engine_and_estimates_constants():
    print("[case] tile vs block, estimated constants, fp32 storage", flush=True)
    sysm = gen.mpc_system(seed=2, N=30)
    X0, Qlin, Glin = gen.mpc_batch(sysm, 64, seed=53)
    kw = dict(method=duq.DFGM, eps_out=1e-4, eps_in=1e-8, max_outer=20000)
    for dt in (np.float64, np.float32):
        H, G = sysm.H.astype(dt), sysm.G.astype(dt)
        Xt, Lt, rt = duq.solve_batch_shared(H, G, sysm.lb, sysm.ub, Qlin, Glin, engine=duq.ENGINE_TILE, **kw)
        Xb, Lb, rb = duq.solve_batch_shared(H, G, sysm.lb, sysm.ub, Qlin, Glin, engine=duq.ENGINE_BLOCK, **kw)
        for b in range(64):
            assert rt[b]["status"] == duq.DUQ_OK and rb[b]["status"] == duq.DUQ_OK
            assert rt[b]["lam_min"] == rb[b]["lam_min"] and rt[b]["G_norm2"] == rb[b]["G_norm2"]
            assert abs(rt[b]["outer_iters"] - rb[b]["outer_iters"]) <= 1
            np.testing.assert_allclose(Xt[b], Xb[b], rtol=0, atol=1e-6)


def test_tile_engine_rejects_what_it_cannot_run():
    sysm = gen.mpc_system(seed=2, N=10)
    X0, Qlin, Glin = gen.mpc_batch(sysm, 4, seed=54)
    with pytest.raises(duq.DuqError) as e:
        duq.solve_batch_shared(sysm.H, sysm.G, sysm.lb, sysm.ub, Qlin, Glin, engine=duq.ENGINE_TILE, rho=1.0)
    assert e.value.code == duq.DUQ_EINVAL
    ub = gen.uneven_batch(B=3, seed=55, n_lo=20, n_hi=40)
    with pytest.raises(duq.DuqError) as e:
        duq.solve_batch_uneven(ub, engine=duq.ENGINE_TILE)
    assert e.value.code == duq.DUQ_EINVAL


@pytest.mark.parametrize("n,p", [(37, 21), (1, 3), (13, 0), (121, 50), (128, 40)])
def test_tile_ragged_generic_shapes_match_oracle(n, p):
    """Shapes the MPC systems never produce: n not a multiple of 4 (a partial
    last k-step), p not a multiple of 16, no constraints, n = 1, and n = 128,
    the largest n the tile holds (eight row tiles of 16, 32 k-steps of Q per
    lane in registers)."""
    print(f"[case] tile generic shape n={n} p={p}", flush=True)
    base = gen.random_dense_qp(n, max(p, 1), seed=60 + n, reg=0.1)
    G = base.G[:p]
    B = 19
    qs, gs = [], []
    for b in range(B):
        q, g = gen.fresh_linear_terms(base.G, seed=1000 * n + b)
        qs.append(q)
        gs.append(g[:p])
    Q = np.stack(qs)
    Gl = np.stack(gs) if p else np.zeros((B, 0))
    qp0 = gen.QP(base.Q, Q[0], G, Gl[0], base.lb, base.ub)
    c = dfom.problem_constants(qp0.Q, qp0.G, qp0.lb, qp0.ub, 0.0, 1e-6)
    consts = (c.lam_min, c.lam_max, c.G_norm2 if p else 1.0)
    X, Lam, res = duq.solve_batch_shared(base.Q, G if p else np.zeros((0, n)), base.lb, base.ub, Q, Gl,
                                         constants=consts, engine=duq.ENGINE_TILE, method=duq.DFGM,
                                         eps_out=1e-4, eps_in=1e-8, max_outer=20000)
    for b in (0, 7, 18):
        qp = gen.QP(base.Q, Q[b], G, Gl[b], base.lb, base.ub)
        ref = dfom.dfom_solve(qp, dfom.Options(method=dfom.DFGM, eps_out=1e-4, eps_in=1e-8, max_outer=20000,
                                               lam_min=c.lam_min, lam_max=c.lam_max, G_norm2=c.G_norm2))
        r = res[b]
        assert r["status"] == duq.DUQ_OK and ref.status == 0, (b, r)
        assert r["outer_iters"] == ref.outer_iters and r["inner_iters"] == ref.inner_iters, (b, r, ref.outer_iters)
        np.testing.assert_allclose(X[b], ref.x, rtol=0, atol=1e-7)
        if p:
            np.testing.assert_allclose(Lam[b], ref.lam, rtol=0, atol=1e-7 * max(1.0, np.abs(ref.lam).max()))


@pytest.mark.parametrize("method", [duq.DFGM, duq.DGM])
def test_tile_infeasible_instances_certified(method):
    # a shared system whose per-instance g makes every other instance infeasible:
    # those end with the oracle's certificate and iterate, the others are solved
    print(f"[case] tile infeasible instances method={method}", flush=True)
    base = gen.infeasible_qp("pair", 1)
    B = 19
    rng = np.random.default_rng(78)
    Qlin = rng.standard_normal((B, base.n))
    Glin = np.tile(base.g, (B, 1))
    Glin[0::2, :2] = -Glin[0::2, :2]          # even instances: a u <= 0.3, -a u <= 0.2 (feasible)
    c = dfom.problem_constants(base.Q, base.G, base.lb, base.ub, 0.0, 1e-6)
    opts = dict(method=method, eps_out=1e-4, eps_in=1e-8 if method == duq.DFGM else 1e-6, max_outer=20000)
    X, Lam, res = duq.solve_batch_shared(base.Q, base.G, base.lb, base.ub, Qlin, Glin,
                                         constants=(c.lam_min, c.lam_max, c.G_norm2), engine=duq.ENGINE_TILE, **opts)
    codes = {dfom.STATUS_OK: duq.DUQ_OK, dfom.STATUS_MAXITER: duq.DUQ_EMAXITER,
             dfom.STATUS_INFEASIBLE: duq.DUQ_EINFEASIBLE}
    for b in range(B):
        qp = gen.QP(base.Q, Qlin[b], base.G, Glin[b], base.lb, base.ub)
        ref = dfom.dfom_solve(qp, dfom.Options(method=dfom.DFGM if method == duq.DFGM else dfom.DGM,
                                               lam_min=c.lam_min, lam_max=c.lam_max, G_norm2=c.G_norm2,
                                               eps_out=opts["eps_out"], eps_in=opts["eps_in"], max_outer=20000))
        assert (ref.status == dfom.STATUS_INFEASIBLE) == (b % 2 == 1), (b, ref.status)
        r = res[b]
        assert r["status"] == codes[ref.status] and r["engine"] == duq.ENGINE_TILE, (b, r)
        assert r["outer_iters"] == ref.outer_iters and r["inner_iters"] == ref.inner_iters, (b, r, ref.outer_iters)
        np.testing.assert_allclose(X[b], ref.x, rtol=0, atol=1e-7)
        np.testing.assert_allclose(Lam[b], ref.lam, rtol=0, atol=1e-7 * max(1.0, np.abs(ref.lam).max()))
