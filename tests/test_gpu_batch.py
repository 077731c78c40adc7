"""GPU parity of the batched forms (duq_solve_batch) against the FP64 oracle."""
import numpy as np
import pytest

from oracle import dfom
from oracle.ipm import ipm_qp
from paper_1504_05708_amd import duq, gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    duq.lib()


def exact_constants(qp):
    c = dfom.problem_constants(qp.Q, qp.G, qp.lb, qp.ub, 0.0, 1e-6)
    return c.lam_min, c.lam_max, c.G_norm2


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_uneven_batch_matches_oracle_per_instance(dtype):
    print(f"[case] uneven batch parity {np.dtype(dtype).name}", flush=True)
    ub = gen.uneven_batch(B=24, seed=31, n_lo=20, n_hi=160, dtype=dtype)
    consts = [exact_constants(ub.instance(i)) for i in range(ub.B)]
    C = [np.array([c[j] for c in consts]) for j in range(3)]
    X, Lam, res = duq.solve_batch_uneven(ub, constants=C, method=duq.DFGM, eps_out=1e-4, eps_in=1e-8,
                                         max_outer=20000)
    for i in range(ub.B):
        qp = ub.instance(i)
        lmin, lmax, g2 = consts[i]
        ref = dfom.dfom_solve(qp, dfom.Options(method=dfom.DFGM, eps_out=1e-4, eps_in=1e-8, max_outer=20000,
                                               lam_min=lmin, lam_max=lmax, G_norm2=g2))
        r = res[i]
        assert r["status"] == duq.DUQ_OK, (i, r)
        assert r["outer_iters"] == ref.outer_iters, (i, r["outer_iters"], ref.outer_iters)
        assert r["inner_iters"] == ref.inner_iters, i
        x = X[ub.voff[i]:ub.voff[i] + qp.n]
        lam = Lam[ub.coff[i]:ub.coff[i] + qp.p]
        np.testing.assert_allclose(x, ref.x, rtol=0, atol=1e-7)
        np.testing.assert_allclose(lam, ref.lam, rtol=0, atol=1e-7 * max(1, np.abs(ref.lam).max()))


def test_uneven_batch_with_infeasible_instances():
    # infeasible instances end with their certificate; the others are unaffected
    print("[case] uneven batch with infeasible instances", flush=True)
    qps = [gen.random_dense_qp(12, 6, seed=60), gen.infeasible_qp("pair", 1),
           gen.random_dense_qp(20, 9, seed=61), gen.infeasible_qp("triple", 3)]
    ub = gen.pack_uneven(qps)
    consts = [exact_constants(qp) for qp in qps]
    C = [np.array([c[j] for c in consts]) for j in range(3)]
    opts = dict(method=duq.DFGM, eps_out=1e-4, eps_in=1e-8, max_outer=20000)
    X, Lam, res = duq.solve_batch_uneven(ub, constants=C, **opts)
    codes = {dfom.STATUS_OK: duq.DUQ_OK, dfom.STATUS_MAXITER: duq.DUQ_EMAXITER,
             dfom.STATUS_INFEASIBLE: duq.DUQ_EINFEASIBLE}
    for i, qp in enumerate(qps):
        lmin, lmax, g2 = consts[i]
        ref = dfom.dfom_solve(qp, dfom.Options(lam_min=lmin, lam_max=lmax, G_norm2=g2, **opts))
        r = res[i]
        want = codes[ref.status]
        assert (ref.status == dfom.STATUS_INFEASIBLE) == (i % 2 == 1), (i, ref.status)
        assert r["status"] == want, (i, r)
        assert r["outer_iters"] == ref.outer_iters and r["inner_iters"] == ref.inner_iters, i
        x = X[ub.voff[i]:ub.voff[i] + qp.n]
        lam = Lam[ub.coff[i]:ub.coff[i] + qp.p]
        np.testing.assert_allclose(x, ref.x, rtol=0, atol=1e-7)
        np.testing.assert_allclose(lam, ref.lam, rtol=0, atol=1e-7 * max(1, np.abs(ref.lam).max()))
    assert [res[i]["status"] for i in range(4)].count(duq.DUQ_EINFEASIBLE) == 2


def test_uneven_batch_estimated_constants_accuracy():
    print("[case] uneven batch with in-kernel Lanczos", flush=True)
    ub = gen.uneven_batch(B=16, seed=32, n_lo=20, n_hi=300, dtype=np.float32)
    X, Lam, res = duq.solve_batch_uneven(ub, method=duq.DFGM, eps_out=1e-4, eps_in=1e-8, max_outer=50000)
    for i in range(ub.B):
        qp = ub.instance(i)
        _, fstar, _ = ipm_qp(qp.Q, qp.q, qp.G, qp.g, qp.lb, qp.ub)
        r = res[i]
        assert r["status"] == duq.DUQ_OK
        assert abs(r["f"] - fstar) / max(1.0, abs(fstar)) <= 1e-4
        assert r["feas"] / max(1.0, np.linalg.norm(qp.g)) <= 1e-4
        ev = np.linalg.eigvalsh(qp.Q)
        assert r["lam_max"] >= ev[-1] and r["lam_min"] <= ev[0] * (1 + 1e-9)


def test_alone_equals_in_the_mix_bitwise():
    print("[case] alone vs mix", flush=True)
    # sizes on both sides of the short/long-row split (n = 256 in FP64)
    ub = gen.uneven_batch(B=12, seed=33, n_lo=20, n_hi=400, dtype=np.float64)
    assert ub.n.min() <= 256 < ub.n.max()
    X, Lam, res = duq.solve_batch_uneven(ub, method=duq.DGM, eps_out=1e-4, eps_in=1e-6, max_outer=50000)
    for i in sorted({int(np.argmin(ub.n)), int(np.argmax(ub.n)), 5}):
        one = gen.UnevenBatch(ub.n[i:i + 1], ub.p[i:i + 1],
                              ub.Q[ub.qoff[i]:ub.qoff[i] + ub.n[i] ** 2],
                              ub.G[ub.goff[i]:ub.goff[i] + ub.p[i] * ub.n[i]],
                              ub.q[ub.voff[i]:ub.voff[i] + ub.n[i]], ub.g[ub.coff[i]:ub.coff[i] + ub.p[i]],
                              ub.lb[ub.voff[i]:ub.voff[i] + ub.n[i]], ub.ub[ub.voff[i]:ub.voff[i] + ub.n[i]],
                              np.zeros(1, np.int64), np.zeros(1, np.int64), np.zeros(1, np.int64),
                              np.zeros(1, np.int64))
        X1, L1, r1 = duq.solve_batch_uneven(one, method=duq.DGM, eps_out=1e-4, eps_in=1e-6, max_outer=50000)
        assert np.array_equal(X1, X[ub.voff[i]:ub.voff[i] + ub.n[i]])
        assert np.array_equal(L1, Lam[ub.coff[i]:ub.coff[i] + ub.p[i]])
        assert r1[0]["outer_iters"] == res[i]["outer_iters"] and r1[0]["inner_iters"] == res[i]["inner_iters"]


def test_shared_hessian_batch_matches_oracle():
    print("[case] shared MPC batch parity", flush=True)
    sysm = gen.mpc_system(seed=2, N=10)
    X0, Qlin, Glin = gen.mpc_batch(sysm, 12, seed=21)
    qp0 = gen.mpc_instance(sysm, X0[0])
    lmin, lmax, g2 = exact_constants(qp0)
    X, Lam, res = duq.solve_batch_shared(sysm.H, sysm.G, sysm.lb, sysm.ub, Qlin, Glin,
                                         constants=(lmin, lmax, g2), method=duq.DFGM, eps_out=1e-4,
                                         eps_in=1e-8, max_outer=50000)
    for b in range(12):
        qp = gen.mpc_instance(sysm, X0[b])
        ref = dfom.dfom_solve(qp, dfom.Options(method=dfom.DFGM, eps_out=1e-4, eps_in=1e-8, max_outer=50000,
                                               lam_min=lmin, lam_max=lmax, G_norm2=g2))
        assert res[b]["status"] == duq.DUQ_OK
        assert res[b]["outer_iters"] == ref.outer_iters and res[b]["inner_iters"] == ref.inner_iters
        np.testing.assert_allclose(X[b], ref.x, rtol=0, atol=1e-7)


def test_batch_rejects_bad_input():
    ub = gen.uneven_batch(B=3, seed=34, n_lo=20, n_hi=40)
    ub.Q[5] = np.nan
    with pytest.raises(duq.DuqError) as e:
        duq.solve_batch_uneven(ub)
    assert e.value.code == duq.DUQ_EINVAL
    # an empty batch is an argument error, not an empty success
    with pytest.raises(duq.DuqError) as e:
        duq.solve_batch_uneven(gen.pack_uneven([]))
    assert e.value.code == duq.DUQ_EINVAL


def test_device_outputs_equal_host_outputs():
    print("[case] batch outputs in device memory", flush=True)
    ub = gen.uneven_batch(B=9, seed=35, n_lo=20, n_hi=300, dtype=np.float64)
    kw = dict(method=duq.DFGM, eps_out=1e-4, eps_in=1e-8, max_outer=20000)
    X, Lam, res = duq.solve_batch_uneven(ub, **kw)
    Xd, Ld, rd = duq.solve_batch_uneven(ub, device_out=True, **kw)
    assert Xd.is_cuda and Ld.is_cuda
    assert np.array_equal(Xd.cpu().numpy()[:X.size], X) and np.array_equal(Ld.cpu().numpy()[:Lam.size], Lam)
    assert [r["outer_iters"] for r in rd] == [r["outer_iters"] for r in res]
    sysm = gen.mpc_system(seed=2, N=10)
    X0, Qlin, Glin = gen.mpc_batch(sysm, 20, seed=36)
    for eng in (duq.ENGINE_TILE, duq.ENGINE_BLOCK):
        Xh, Lh, _ = duq.solve_batch_shared(sysm.H, sysm.G, sysm.lb, sysm.ub, Qlin, Glin, engine=eng, **kw)
        Xd, Ld, _ = duq.solve_batch_shared(sysm.H, sysm.G, sysm.lb, sysm.ub, Qlin, Glin, engine=eng,
                                           device_out=True, **kw)
        assert np.array_equal(Xd.cpu().numpy().reshape(Xh.shape), Xh)
        assert np.array_equal(Ld.cpu().numpy().reshape(Lh.shape), Lh)


@pytest.mark.parametrize("method,output,rho", [(duq.DFGM, duq.LAST, 1.0), (duq.DGM, duq.AVG, 0.5),
                                               (duq.DFGM, duq.AVG, 0.0)])
def test_uneven_batch_other_options_match_oracle(method, output, rho):
    """The per-instance batch kernel with the augmented Lagrangian (rho > 0)
    and the averaged output, against the oracle instance by instance."""
    print(f"[case] uneven batch method={method} output={output} rho={rho}", flush=True)
    ub = gen.uneven_batch(B=8, seed=37, n_lo=10, n_hi=140, dtype=np.float64)
    consts = [exact_constants(ub.instance(i)) for i in range(ub.B)]
    C = [np.array([c[j] for c in consts]) for j in range(3)]
    eps_in = 1e-8 if method == duq.DFGM else 1e-6
    X, Lam, res = duq.solve_batch_uneven(ub, constants=C, method=method, output=output, rho=rho, eps_out=1e-4,
                                         eps_in=eps_in, max_outer=20000)
    for i in range(ub.B):
        qp = ub.instance(i)
        lmin, lmax, g2 = consts[i]
        ref = dfom.dfom_solve(qp, dfom.Options(method=dfom.DFGM if method == duq.DFGM else dfom.DGM,
                                               output=dfom.LAST if output == duq.LAST else dfom.AVG, rho=rho,
                                               eps_out=1e-4, eps_in=eps_in, max_outer=20000,
                                               lam_min=lmin, lam_max=lmax, G_norm2=g2))
        r = res[i]
        assert r["status"] == (duq.DUQ_OK if ref.status == 0 else duq.DUQ_EMAXITER), (i, r, ref.status)
        if ref.outer_iters <= 300:
            assert r["outer_iters"] == ref.outer_iters and r["inner_iters"] == ref.inner_iters, (i, r, ref.outer_iters)
            np.testing.assert_allclose(X[ub.voff[i]:ub.voff[i] + qp.n], ref.x, rtol=0, atol=1e-7)
        else:
            # long runs whose warm-started inner certificates sit at eps_in: a
            # rounding-level difference can move a stop decision by one step
            assert abs(r["outer_iters"] - ref.outer_iters) <= 2, (i, r["outer_iters"], ref.outer_iters)
            assert abs(r["inner_iters"] - ref.inner_iters) <= 0.01 * ref.inner_iters, (i, r, ref.inner_iters)
            np.testing.assert_allclose(X[ub.voff[i]:ub.voff[i] + qp.n], ref.x, rtol=0, atol=1e-5)


def test_tuned_launch_shape_leaves_results_unchanged(tmp_path):
    # duq_tune_batch times 1, 2 and 3 workgroups per CU (checking inside that
    # all three give the same bits), records the fastest, and later batches
    # with batch_wpc = 0 use it: results equal a run at every explicit shape
    print("[case] batch launch-shape tuning", flush=True)
    ub = gen.uneven_batch(B=60, seed=71, n_lo=20, n_hi=300, dtype=np.float32)
    kw = dict(method=duq.DFGM, eps_out=1e-4, eps_in=1e-8, max_outer=20000)
    best, ms = duq.tune_batch(ub, **kw)
    assert best in (1, 2, 3) and ms[best - 1] > 0.0
    X, Lam, res = duq.solve_batch_uneven(ub, **kw)
    for wpc in (1, 2, 3):
        Xw, Lw, rw = duq.solve_batch_uneven(ub, batch_wpc=wpc, **kw)
        assert np.array_equal(X, Xw) and np.array_equal(Lam, Lw), wpc
        assert [r["inner_iters"] for r in res] == [r["inner_iters"] for r in rw]
    duq.tune_save(str(tmp_path / "tune.txt"))
    assert (tmp_path / "tune.txt").read_text().strip()


def test_concurrent_batches_give_the_same_bits():
    """duq_solve_batch keeps its device workspace between calls: calls from
    two host threads at once (one takes the kept block, the other allocates
    its own) give the bits of a call made alone."""
    import threading
    print("[case] batch calls from two threads", flush=True)
    ub = gen.uneven_batch(B=24, seed=77, n_lo=20, n_hi=300, dtype=np.float64)
    kw = dict(method=duq.DFGM, eps_out=1e-4, eps_in=1e-8, max_outer=20000)
    X0, L0, r0 = duq.solve_batch_uneven(ub, **kw)
    out = [None, None, None]

    def run(i):
        out[i] = duq.solve_batch_uneven(ub, **kw)

    th = [threading.Thread(target=run, args=(i,)) for i in range(3)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    for i, o in enumerate(out):
        assert o is not None, i
        X, L, r = o
        assert np.array_equal(X, X0) and np.array_equal(L, L0), i
        assert [q["inner_iters"] for q in r] == [q["inner_iters"] for q in r0], i
