"""GPU tests of the serving loop (duq_server_*): parity with the FP64 oracle,
the same bits alone and in a mix, admission by footprint, EAGAIN/ENOTFOUND."""
import numpy as np
import pytest

from oracle import dfom
from paper_1504_05708_amd import duq, gen

pytestmark = pytest.mark.gpu

OPTS = dict(method=duq.DFGM, eps_out=1e-4, eps_in=1e-8, max_outer=20000, serve_slice=4)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    duq.lib()


def _own(qp):
    return dict(Q=qp.Q, q=qp.q, G=qp.G, g=qp.g, lb=qp.lb, ub=qp.ub)


def _mix():
    ub = gen.uneven_batch(B=10, seed=41, n_lo=20, n_hi=400, dtype=np.float64)
    sysm = gen.mpc_system(seed=2, N=10)
    X0, Qlin, Glin = gen.mpc_batch(sysm, 6, seed=42)
    return ub, sysm, Qlin, Glin


def _serve(server, own, shared_id, Qlin, Glin):
    tickets = [server.submit(**_own(qp)) for qp in own]
    tickets += [server.submit(q=Qlin[b], g=Glin[b], shared_id=shared_id) for b in range(len(Qlin))]
    return [server.wait(t) for t in tickets]


def test_served_requests_match_oracle():
    print("[case] serve parity vs oracle", flush=True)
    ub, sysm, Qlin, Glin = _mix()
    own = [ub.instance(i) for i in range(ub.B)]
    with duq.Server(1 << 28, **OPTS) as s:
        sid = s.register_shared(sysm.H, sysm.G, sysm.lb, sysm.ub)
        out = _serve(s, own, sid, Qlin, Glin)
    for i, qp in enumerate(own):
        rc, x, lam, r = out[i]
        assert rc == duq.DUQ_OK, (i, r)
        # the constants the request ran with (estimated in its first slice) lie on
        # the safe side of the true spectrum, and near it
        ev = np.linalg.eigvalsh(qp.Q)
        g2 = np.linalg.norm(qp.G, 2) ** 2
        assert 0.0 < r["lam_min"] <= ev[0] * (1 + 1e-9) and r["lam_min"] >= ev[0] / 1.5, (i, r, ev[0])
        assert ev[-1] <= r["lam_max"] <= 1.05 * ev[-1], (i, r, ev[-1])
        assert g2 <= r["G_norm2"] <= 1.05 * g2, (i, r, g2)
        ref = dfom.dfom_solve(qp, dfom.Options(method=dfom.DFGM, eps_out=1e-4, eps_in=1e-8, max_outer=20000,
                                               lam_min=r["lam_min"], lam_max=r["lam_max"], G_norm2=r["G_norm2"]))
        assert ref.status == 0, (i, r)
        assert r["outer_iters"] == ref.outer_iters and r["inner_iters"] == ref.inner_iters, (i, r, ref.outer_iters)
        np.testing.assert_allclose(x, ref.x, rtol=0, atol=1e-7)
        np.testing.assert_allclose(lam, ref.lam, rtol=0, atol=1e-7 * max(1, np.abs(ref.lam).max()))
        assert r["time_ms"] > 0
    ev = np.linalg.eigvalsh(sysm.H)
    g2 = np.linalg.norm(sysm.G, 2) ** 2
    for b in range(len(Qlin)):
        rc, x, lam, r = out[ub.B + b]
        # a registered system's constants (estimated once at registration)
        assert 0.0 < r["lam_min"] <= ev[0] * (1 + 1e-9) and ev[-1] <= r["lam_max"] and g2 <= r["G_norm2"], (b, r)
        qp = gen.QP(sysm.H, Qlin[b], sysm.G, Glin[b], sysm.lb, sysm.ub)
        ref = dfom.dfom_solve(qp, dfom.Options(method=dfom.DFGM, eps_out=1e-4, eps_in=1e-8, max_outer=20000,
                                               lam_min=r["lam_min"], lam_max=r["lam_max"], G_norm2=r["G_norm2"]))
        assert rc == duq.DUQ_OK
        assert r["engine"] == duq.ENGINE_TILE, (b, r)   # a shared system with n <= 128: the MFMA tiles
        assert r["outer_iters"] == ref.outer_iters and r["inner_iters"] == ref.inner_iters, (b, r)
        np.testing.assert_allclose(x, ref.x, rtol=0, atol=1e-7)


def test_served_alone_equals_in_the_mix_bitwise():
    print("[case] serve alone vs mix", flush=True)
    ub, sysm, Qlin, Glin = _mix()
    own = [ub.instance(i) for i in range(ub.B)]
    with duq.Server(1 << 28, **OPTS) as s:
        sid = s.register_shared(sysm.H, sysm.G, sysm.lb, sysm.ub)
        mix = _serve(s, own, sid, Qlin, Glin)
    for i in (0, 3, 9):
        with duq.Server(1 << 28, **OPTS) as s:
            rc, x, lam, r = s.wait(s.submit(**_own(own[i])))
        assert rc == mix[i][0]
        assert np.array_equal(x, mix[i][1]) and np.array_equal(lam, mix[i][2]), i
        assert r["outer_iters"] == mix[i][3]["outer_iters"] and r["inner_iters"] == mix[i][3]["inner_iters"]
    with duq.Server(1 << 28, **OPTS) as s:
        sid = s.register_shared(sysm.H, sysm.G, sysm.lb, sysm.ub)
        rc, x, lam, r = s.wait(s.submit(q=Qlin[2], g=Glin[2], shared_id=sid))
    assert np.array_equal(x, mix[ub.B + 2][1]) and np.array_equal(lam, mix[ub.B + 2][2])


def test_large_request_runs_on_the_single_qp_engine():
    print("[case] serve large request (grid engine)", flush=True)
    qp = gen.random_dense_qp(2048, 1024, seed=43)
    with duq.Server(1 << 30, **OPTS) as s:
        rc, x, lam, r = s.wait(s.submit(**_own(qp)), timeout=120)
    assert rc == duq.DUQ_OK and r["engine"] == duq.ENGINE_GRID
    with duq.Solver(qp.Q, qp.q, qp.G, qp.g, qp.lb, qp.ub, **{k: v for k, v in OPTS.items() if k != "serve_slice"}) as sv:
        x1, lam1, r1 = sv.solve()
    assert r1["status"] == duq.DUQ_OK
    # slices resume from the stored iterates and products: the same bits as one piece
    assert r["outer_iters"] == r1["outer_iters"] and r["inner_iters"] == r1["inner_iters"]
    assert np.array_equal(x, x1) and np.array_equal(lam, lam1)


def test_served_equals_one_batch_bitwise():
    print("[case] serve vs duq_solve_batch", flush=True)
    ub, sysm, Qlin, Glin = _mix()
    own = [ub.instance(i) for i in range(ub.B)]
    with duq.Server(1 << 28, **OPTS) as s:
        out = [s.wait(s.submit(**_own(qp))) for qp in own]
    X, Lam, res = duq.solve_batch_uneven(ub, **{k: v for k, v in OPTS.items() if k != "serve_slice"})
    for i, qp in enumerate(own):
        rc, x, lam, r = out[i]
        assert r["outer_iters"] == res[i]["outer_iters"] and r["inner_iters"] == res[i]["inner_iters"], i
        assert np.array_equal(x, X[ub.voff[i]:ub.voff[i] + qp.n]), i
        assert np.array_equal(lam, Lam[ub.coff[i]:ub.coff[i] + qp.p]), i


def test_poll_states_and_errors():
    print("[case] serve EAGAIN / ENOTFOUND / ENOMEM / EINVAL", flush=True)
    qp = gen.random_dense_qp(1200, 600, seed=44)
    with duq.Server(1 << 28, **OPTS) as s:
        t = s.submit(**_own(qp))
        assert s.poll(t) is None          # just queued: DUQ_EAGAIN
        rc, x, lam, r = s.wait(t, timeout=120)
        assert rc == duq.DUQ_OK
        with pytest.raises(duq.DuqError) as e:
            s.poll(t)                     # collected: forgotten
        assert e.value.code == duq.DUQ_ENOTFOUND
        with pytest.raises(duq.DuqError) as e:
            s.poll(987654321)
        assert e.value.code == duq.DUQ_ENOTFOUND
        bad = gen.random_dense_qp(30, 10, seed=45)
        q = bad.q.copy()
        q[3] = np.nan
        with pytest.raises(duq.DuqError) as e:
            s.submit(Q=bad.Q, q=q, G=bad.G, g=bad.g, lb=bad.lb, ub=bad.ub)
        assert e.value.code == duq.DUQ_EINVAL
        with pytest.raises(duq.DuqError) as e:
            s.submit(q=bad.q, g=bad.g, shared_id=5)
    small = duq.Server(1 << 20, **OPTS)   # 1 MiB arena: smaller than one n=512 request
    try:
        big = gen.random_dense_qp(512, 256, seed=46)
        with pytest.raises(duq.DuqError) as e:
            small.submit(**_own(big))
        assert e.value.code == duq.DUQ_ENOMEM
    finally:
        small.close()


def test_infeasible_request_is_certified():
    print("[case] serve infeasible request", flush=True)
    qp = gen.random_dense_qp(40, 20, seed=47)
    # G u + g <= 0 with a row and its negative both strictly violated on the box
    G = np.vstack([qp.G, qp.G[:1], -qp.G[:1]])
    big = np.abs(qp.G[0]).sum() * 2 + 10
    g = np.concatenate([qp.g, [big, big]])
    opts = dict(OPTS, max_outer=300)
    with duq.Server(1 << 26, **opts) as s:
        rc, x, lam, r = s.wait(s.submit(Q=qp.Q, q=qp.q, G=G, g=g, lb=qp.lb, ub=qp.ub), timeout=120)
    # ends before max_outer with a certificate: mu >= 0, min over the box of
    # mu^T (G u + g) > 0 (the box minimum of a linear function, coordinatewise)
    assert rc == duq.DUQ_EINFEASIBLE and r["outer_iters"] < 300
    w = G.T @ lam
    assert np.all(lam >= 0.0) and lam @ g + np.sum(np.minimum(qp.lb * w, qp.ub * w)) > 0.0


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_served_tile_requests_equal_the_shared_batch_bitwise(dt):
    """Requests against a registered system run on the MFMA tiles: the same
    bits as duq_solve_batch on the same system with the same constants (one
    tile there, tiles of the round's requests here)."""
    print(f"[case] serve tiles vs shared batch dtype={np.dtype(dt).name}", flush=True)
    sysm = gen.mpc_system(seed=5, N=12)
    X0, Qlin, Glin = gen.mpc_batch(sysm, 19, seed=55)
    H, G = sysm.H.astype(dt), sysm.G.astype(dt)
    with duq.Server(1 << 28, **OPTS) as s:
        sid = s.register_shared(H, G, sysm.lb, sysm.ub)
        out = [s.wait(s.submit(q=Qlin[b], g=Glin[b], shared_id=sid)) for b in range(len(Qlin))]
    c = (out[0][3]["lam_min"], out[0][3]["lam_max"], out[0][3]["G_norm2"])
    X, Lam, res = duq.solve_batch_shared(H, G, sysm.lb, sysm.ub, Qlin, Glin, constants=c, engine=duq.ENGINE_TILE,
                                         **{k: v for k, v in OPTS.items() if k != "serve_slice"})
    for b, (rc, x, lam, r) in enumerate(out):
        assert rc == duq.DUQ_OK and r["engine"] == duq.ENGINE_TILE, (b, r)
        assert (r["lam_min"], r["lam_max"], r["G_norm2"]) == c
        assert r["outer_iters"] == res[b]["outer_iters"] and r["inner_iters"] == res[b]["inner_iters"], b
        assert np.array_equal(x, X[b]) and np.array_equal(lam, Lam[b]), b
