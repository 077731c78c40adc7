"""The allocation-free entry point (duq_solve_static) against duq_setup +
duq_solve on the same device data: the same kernels on the same inputs, so
the answers are bitwise equal.  Two calls in a row, the second smaller, so
the shared static scratch is reused with stale contents from the first."""
import numpy as np
import pytest

from paper_1504_05708_amd import duq, gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    duq.lib()


def _dev(qp, dtype):
    import torch
    d = lambda a, dt=np.float64: torch.from_numpy(np.ascontiguousarray(np.asarray(a, dt))).cuda()
    return d(qp.Q, dtype), d(qp.q), d(qp.G, dtype), d(qp.g), d(qp.lb), d(qp.ub)


def _constants(qp):
    ev = np.linalg.eigvalsh(qp.Q)
    g2 = float(np.linalg.norm(qp.G, 2) ** 2) if qp.p else 0.0
    return dict(lam_min=float(ev[0]), lam_max=float(ev[-1]), G_norm2=g2)


def _compare(qp, dtype=np.float64, **opts):
    import torch
    Q, q, G, g, lb, ub = _dev(qp, dtype)
    kw = dict(_constants(qp), **opts)
    x = torch.full((qp.n,), np.nan, dtype=torch.float64, device="cuda")
    lam = torch.full((max(qp.p, 1),), np.nan, dtype=torch.float64, device="cuda")
    rc, r = duq.solve_static(Q, q, G, g, lb, ub, x, lam[:qp.p] if qp.p else lam[:0], **kw)
    torch.cuda.synchronize()
    with duq.Solver(Q, q, G, g, lb, ub, **kw) as s:
        x1, lam1, r1 = s.solve(check=False)
    assert rc == r1["status"]
    assert r["engine"] == r1["engine"]
    assert r["outer_iters"] == r1["outer_iters"] and r["inner_iters"] == r1["inner_iters"]
    assert r["f"] == r1["f"] and r["lb_dual"] == r1["lb_dual"] and r["feas"] == r1["feas"]
    assert np.array_equal(x.cpu().numpy(), x1)
    assert np.array_equal(lam[:qp.p].cpu().numpy(), lam1)
    return r


@pytest.mark.parametrize("engine", [duq.ENGINE_BLOCK, duq.ENGINE_GRID])
def test_static_equals_allocating_entry_point_twice(engine):
    # first call larger, second smaller: the scratch keeps the first call's
    # bytes, and the second must not depend on them
    print(f"[case] no-alloc engine={engine}", flush=True)
    big = gen.random_dense_qp(300, 140, seed=61)
    small = gen.random_dense_qp(57, 23, seed=62)
    opts = dict(method=duq.DFGM, eps_out=1e-4, eps_in=1e-8, max_outer=100000, engine=engine)
    r1 = _compare(big, **opts)
    r2 = _compare(small, **opts)
    assert r1["status"] == duq.DUQ_OK and r2["status"] == duq.DUQ_OK


def test_static_large_grid_then_small_fp32():
    print("[case] no-alloc grid n=2048 then block n=100 FP32", flush=True)
    big = gen.config1(n=2048, p=1024, seed=63)
    _compare(big, method=duq.DFGM, eps_out=1e-13, eps_in=1e-8, max_outer=20)
    small = gen.random_dense_qp(100, 50, seed=64)
    _compare(small, dtype=np.float32, method=duq.DGM, output=duq.AVG, eps_out=1e-4, eps_in=1e-6,
             max_outer=20000)


def test_static_rejects_what_it_cannot_run():
    import torch
    qp = gen.random_dense_qp(40, 20, seed=65)
    Q, q, G, g, lb, ub = _dev(qp, np.float64)
    x = torch.zeros(qp.n, dtype=torch.float64, device="cuda")
    lam = torch.zeros(qp.p, dtype=torch.float64, device="cuda")
    with pytest.raises(duq.DuqError) as e:           # constants are required
        duq.solve_static(Q, q, G, g, lb, ub, x, lam)
    assert e.value.code == duq.DUQ_EINVAL
    c = _constants(qp)
    with pytest.raises(duq.DuqError) as e:           # no tracing
        duq.solve_static(Q, q, G, g, lb, ub, x, lam, trace_outer=3, **c)
    assert e.value.code == duq.DUQ_EINVAL
    bad = lb.clone()
    bad[3] = 5.0                                     # lb > ub, found on the device
    with pytest.raises(duq.DuqError) as e:
        duq.solve_static(Q, q, G, g, bad, ub, x, lam, **c)
    assert e.value.code == duq.DUQ_EINVAL
    # a workspace beyond the static scratch: about 12 p doubles of multiplier
    # vectors for p = 10^6 rows on the grid engine (96 MB > 64 MiB); rejected
    # from the sizes alone, before any data is read
    n, p = 256, 1_000_000
    Gbig = torch.zeros((p, n), dtype=torch.float32, device="cuda")
    Qs = torch.eye(n, dtype=torch.float32, device="cuda")
    v = lambda m: torch.zeros(m, dtype=torch.float64, device="cuda")
    with pytest.raises(duq.DuqError) as e:
        duq.solve_static(Qs, v(n), Gbig, v(p), v(n) - 1.0, v(n) + 1.0, v(n), v(p), engine=duq.ENGINE_GRID,
                         lam_min=1.0, lam_max=1.0, G_norm2=1.0)
    assert e.value.code == duq.DUQ_EINVAL and "exceeds the static scratch" in str(e.value)
    del Gbig
    torch.cuda.empty_cache()
