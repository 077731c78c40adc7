"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

FP64 path: iterates lambda^k, mu^k, ubar^k match to 1e-9 relative over the
first 200 outer iterations and the inner step counts t_k match exactly.
Both sides get the same spectral constants (the oracle's exact ones).
"""
import math
import os
import sys

import numpy as np
import pytest

from oracle import dfom
from oracle.ipm import ipm_qp
from paper_1504_05708_amd import duq, gen

pytestmark = pytest.mark.gpu

REL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    duq.lib()


def consts_of(qp, rho=0.0, eps_in=1e-6):
    return dfom.problem_constants(qp.Q, qp.G, qp.lb, qp.ub, rho, eps_in)


def gpu_solver(qp, c, dtype=np.float64, **kw):
    kw.setdefault("lam_min", c.lam_min)
    kw.setdefault("lam_max", c.lam_max)
    kw.setdefault("G_norm2", c.G_norm2 if qp.p else 0.0)
    return duq.Solver(qp.Q.astype(dtype), qp.q, qp.G.astype(dtype), qp.g, qp.lb, qp.ub, **kw)


def close(a, b, rel=REL, what=""):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    if a.size == 0:
        return
    scale = max(1.0, float(np.max(np.abs(b))))
    err = float(np.max(np.abs(a - b)))
    assert err <= rel * scale, f"{what}: max err {err:.3e} > {rel:.1e} * {scale:.3e}"


def compare_trace(tr, log, K, what):
    S = tr["scalars"]
    assert S.shape[0] == K, (S.shape, K)
    assert len(log) >= K
    for k in range(K):
        e = log[k]
        assert int(S[k, 0]) == e["k"]
        assert int(S[k, 1]) == e["t"], f"{what}: inner count differs at k={k + 1}: {int(S[k, 1])} vs {e['t']}"
        close(tr["lam"][k], e["lam"], what=f"{what} lambda^{k + 1}")
        close(tr["mu"][k], e["mu"], what=f"{what} mu^{k + 1}")
        close(tr["u"][k], e["u"], what=f"{what} ubar^{k + 1}")
        sc = max(1.0, abs(e["dbar"]))
        assert abs(S[k, 3] - e["dbar"]) <= REL * sc, (what, k)
        assert abs(S[k, 2] - e["gap"]) <= REL * sc, (what, k)
        if math.isfinite(e["LB"]):
            assert abs(S[k, 4] - e["LB"]) <= REL * sc, (what, k)
        assert S[k, 5] == pytest.approx(e["theta"], rel=1e-14)
        assert S[k, 6] == pytest.approx(e["S"], rel=1e-14)


def run_trace_case(qp, method, output, rho=0.0, K=200, engine=duq.ENGINE_AUTO, dtype=np.float64,
                   eps_in=1e-6, variant=dfom.INNER_AUTO):
    qpo = qp if dtype == np.float64 else qp.rounded(dtype)
    c = consts_of(qpo, rho, eps_in)
    opts = dfom.Options(method=method, output=output, rho=rho, eps_out=1e-13, eps_in=eps_in,
                        max_outer=K, log_vectors=K, inner_variant=variant)
    ref = dfom.dfom_solve(qpo, opts, consts=c)
    with gpu_solver(qp, c, dtype, method=method, output=output, rho=rho, eps_out=1e-13, eps_in=eps_in,
                    max_outer=K, trace_outer=K, engine=engine, inner_variant=variant) as s:
        x, lam, res = s.solve()
        tr = s.trace(K)
    Kg, Ko = res["outer_iters"], ref.outer_iters
    what = f"n={qp.n} p={qp.p} m={method} o={output} rho={rho}"
    # Tiny instances reach the 1e-13 outer test at the rounding floor, where the
    # two summation orders may decide one iteration apart: compare the common
    # prefix and require the later side to sit at the floor where the other stopped.
    Kc = min(Kg, Ko)
    compare_trace({k: v[:Kc] for k, v in tr.items()}, ref.log, Kc, what)
    if Kg != Ko:
        e = ref.log[Kc - 1] if Ko > Kg else None
        Fk, LBk, fk = (e["F"], e["LB"], e["feas"]) if e else (tr["scalars"][Kc - 1, 7], tr["scalars"][Kc - 1, 4],
                                                               tr["scalars"][Kc - 1, 8])
        sc = max(1.0, abs(Fk))
        assert Fk - LBk <= 1e-11 * sc and fk <= 1e-11 * max(1.0, np.linalg.norm(qp.g)), (what, Kg, Ko)
    else:
        assert res["inner_iters"] == ref.inner_iters
        assert res["status"] == (duq.DUQ_EMAXITER if ref.status == dfom.STATUS_MAXITER else duq.DUQ_OK)
    return ref, x, lam, res


# ----------------------------------------------------------------------------
# config 0 (n=50, p=25): iterate parity over 200 outer iterations
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("method,output", [(duq.DFGM, duq.LAST), (duq.DGM, duq.AVG),
                                           (duq.DGM, duq.LAST), (duq.DFGM, duq.AVG)])
def test_config0_trace_parity(method, output):
    print(f"[case] config0 trace m={method} o={output}", flush=True)
    run_trace_case(gen.config0(), method, output)


@pytest.mark.parametrize("rho", [0.5, 1.0])
def test_config0_augmented_trace_parity(rho):
    print(f"[case] config0 augmented rho={rho}", flush=True)
    run_trace_case(gen.config0(), duq.DFGM, duq.LAST, rho=rho, K=120)


def test_config0_inner_fgm_variant_parity():
    print("[case] config0 inner FGM theta rule", flush=True)
    run_trace_case(gen.config0(), duq.DFGM, duq.LAST, K=60, variant=dfom.INNER_FGM)


@pytest.mark.parametrize("method,output,eps_in", [(duq.DFGM, duq.LAST, 1e-8), (duq.DGM, duq.LAST, 1e-6),
                                                  (duq.DFGM, duq.AVG, 1e-8), (duq.DGM, duq.AVG, 1e-6)])
@pytest.mark.timeout(300)
def test_config0_converged_solution(method, output, eps_in):
    # (DGM, AVG) at eps_in = 1e-6 is the small QP's second run: about 2.4e5 outer
    # iterations to the 1e-4 test
    print(f"[case] config0 converged m={method} o={output}", flush=True)
    qp = gen.config0()
    c = consts_of(qp, 0.0, eps_in)
    ref = dfom.dfom_solve(qp, dfom.Options(method=method, output=output, eps_out=1e-4, eps_in=eps_in,
                                           max_outer=2000000), consts=c)
    with gpu_solver(qp, c, method=method, output=output, eps_out=1e-4, eps_in=eps_in, max_outer=2000000) as s:
        x, lam, res = s.solve()
    assert res["status"] == duq.DUQ_OK
    if (method, output) == (duq.DGM, duq.AVG):
        # ~2.4e5 warm-started outer iterations, most with no inner step: a
        # warm-start certificate that sits within rounding of eps_in may take its
        # stop decision one iteration apart on the two sides
        print(f"DGM-AVG outer {res['outer_iters']} vs {ref.outer_iters}, inner {res['inner_iters']} vs "
              f"{ref.inner_iters}", flush=True)
        assert abs(res["outer_iters"] - ref.outer_iters) <= 1e-3 * ref.outer_iters
        assert abs(res["inner_iters"] - ref.inner_iters) <= 1e-2 * ref.inner_iters
        close(x, ref.x, rel=1e-6, what="x")
        close(lam, ref.lam, rel=1e-6, what="lambda")
    else:
        assert res["outer_iters"] == ref.outer_iters
        assert res["inner_iters"] == ref.inner_iters
        close(x, ref.x, rel=1e-7, what="x")
        close(lam, ref.lam, rel=1e-7, what="lambda")
    _, fstar, _ = ipm_qp(qp.Q, qp.q, qp.G, qp.g, qp.lb, qp.ub)
    assert abs(res["f"] - fstar) / abs(fstar) <= 1e-4
    assert res["feas"] / max(1.0, np.linalg.norm(qp.g)) <= 1e-4
    assert res["lb_dual"] <= fstar + 1e-9 * abs(fstar)


# ----------------------------------------------------------------------------
# ragged shapes, both engines
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("engine", [duq.ENGINE_BLOCK, duq.ENGINE_GRID])
@pytest.mark.parametrize("n,p", [(1, 1), (2, 0), (3, 5), (63, 31), (64, 64), (65, 1), (130, 257), (257, 100)])
def test_ragged_shapes_parity(engine, n, p):
    print(f"[case] ragged n={n} p={p} engine={engine}", flush=True)
    qp = gen.random_dense_qp(n, p, seed=1000 + n + 7 * p)
    run_trace_case(qp, duq.DFGM, duq.LAST, K=40, engine=engine)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_grid_medium_parity(dtype):
    print(f"[case] grid n=1536 dtype={np.dtype(dtype).name}", flush=True)
    qp = gen.config1(n=1536, p=768, seed=11)
    run_trace_case(qp, duq.DFGM, duq.LAST, K=30, engine=duq.ENGINE_GRID, dtype=dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_grid_unaligned_rows_parity(dtype):
    """Odd n on the grid engine: rows are not 16-byte aligned, so the products
    take the scalar path (same summation order) across every workgroup."""
    print(f"[case] grid n=2049 dtype={np.dtype(dtype).name}", flush=True)
    qp = gen.config1(n=2049, p=1023, seed=16)
    run_trace_case(qp, duq.DFGM, duq.LAST, K=12, engine=duq.ENGINE_GRID, dtype=dtype)


def test_fp32_storage_block_parity():
    print("[case] fp32 storage block", flush=True)
    qp = gen.random_dense_qp(301, 150, seed=5)
    run_trace_case(qp, duq.DGM, duq.AVG, K=60, engine=duq.ENGINE_BLOCK, dtype=np.float32)


def test_grid_augmented_parity():
    print("[case] grid rho=1 n=1024", flush=True)
    qp = gen.config1(n=1024, p=512, seed=12)
    run_trace_case(qp, duq.DFGM, duq.LAST, rho=1.0, K=20, engine=duq.ENGINE_GRID)


# ----------------------------------------------------------------------------
# full size of the large single QP (n=8192, p=4096): first outer iterations
# ----------------------------------------------------------------------------

_CONFIG1 = {}


def _config1_full():
    # the large dense QP (n = 8192, p = 4096) and its exact constants, made once
    if not _CONFIG1:
        qp = gen.config1()
        _CONFIG1["qp"] = qp
        _CONFIG1["c"] = consts_of(qp)
    return _CONFIG1["qp"], _CONFIG1["c"]


def run_trace_given(qp, c, method, output, K, dtype=np.float64, rho=0.0, eps_in=1e-6, engine=duq.ENGINE_GRID):
    """Trace parity over K outer iterations with constants c given to both sides."""
    qpo = qp if dtype == np.float64 else qp.rounded(dtype)
    opts = dfom.Options(method=method, output=output, rho=rho, eps_out=1e-13, eps_in=eps_in,
                        max_outer=K, log_vectors=K)
    ref = dfom.dfom_solve(qpo, opts, consts=c)
    with duq.Solver(qp.Q.astype(dtype), qp.q, qp.G.astype(dtype), qp.g, qp.lb, qp.ub, method=method,
                    output=output, rho=rho, eps_out=1e-13, eps_in=eps_in, max_outer=K, trace_outer=K,
                    engine=engine, lam_min=c.lam_min, lam_max=c.lam_max, G_norm2=c.G_norm2) as s:
        x, lam, res = s.solve(check=False)
        tr = s.trace(K)
    assert res["engine"] == engine
    assert res["outer_iters"] == ref.outer_iters == K
    compare_trace(tr, ref.log, K, f"n={qp.n} p={qp.p} dtype={np.dtype(dtype).name} rho={rho}")
    assert res["inner_iters"] == ref.inner_iters
    # the transposed product touched rows of G with nonzero multipliers (mu^1 = 0
    # skips every row): the full-row load path of G^T mu ran in most iterations
    assert res["gt_rows"] > (K // 2) * qp.p // 4
    return ref, res


@pytest.mark.timeout(900)
def test_config1_full_size_200_outer_iterations():
    # the headline engine at the headline size: 200 traced outer iterations at
    # 1e-9 relative, inner counts exact
    print("[case] config1 full size FP64, 200 outer iterations", flush=True)
    qp, c = _config1_full()
    run_trace_given(qp, c, duq.DFGM, duq.LAST, K=200)


@pytest.mark.timeout(900)
def test_config1_full_size_fp32_storage_50_outer_iterations():
    # FP32 storage of Q and G (FP64 accumulation): the oracle runs on the same
    # FP32-rounded data in FP64; both sides get the FP64 problem's exact constants
    print("[case] config1 full size FP32 storage, 50 outer iterations", flush=True)
    qp, c = _config1_full()
    run_trace_given(qp, c, duq.DFGM, duq.LAST, K=50, dtype=np.float32)


@pytest.mark.timeout(600)
def test_grid_augmented_parity_n4096():
    # rho = 1 (inner steps read Q and G) on the grid engine at n = 4096: the
    # largest size at which the oracle runs 20 outer iterations (~5300 inner
    # steps) in well under a minute
    print("[case] grid rho=1 n=4096, 20 outer iterations", flush=True)
    qp = gen.config1(n=4096, p=2048, seed=17)
    c = consts_of(qp, rho=1.0)
    run_trace_given(qp, c, duq.DFGM, duq.LAST, K=20, rho=1.0)


def test_config1_full_size_first_iterations():
    print("[case] config1 full size, 2 outer iterations", flush=True)
    qp = gen.config1()
    run_trace_case(qp, duq.DFGM, duq.LAST, K=2, engine=duq.ENGINE_GRID)


def test_grid_maximum_size():
    # The largest n the grid engine accepts (every workgroup stages x in LDS):
    # a diagonal QP with one dense active row, pinned by its closed form (the
    # multiplier by bisection); n + 1 is rejected with the bound in the message.
    import torch
    import separable
    n = duq.max_n(1, duq.ENGINE_GRID)
    print(f"[case] grid maximum size n={n} p=1", flush=True)
    assert 8192 < n < (1 << 20)
    d, q, a, b, lb, ub = gen.separable_terms(n, seed=7)
    dev = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()
    Q = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    Q.diagonal().copy_(dev(d))
    kw = dict(engine=duq.ENGINE_GRID, method=duq.DFGM, eps_out=1e-4, eps_in=1e-8,
              lam_min=float(d.min()), lam_max=float(d.max()), G_norm2=float(a @ a))
    with duq.Solver(Q, dev(q), dev(a[None, :]), dev(np.array([-b])), dev(lb), dev(ub), **kw) as s:
        x, lam, res = s.solve()
    x = x.cpu().numpy() if hasattr(x, "cpu") else np.asarray(x)
    assert res["engine"] == duq.ENGINE_GRID and res["status"] == duq.DUQ_OK
    u, m, F = separable.solve(d, q, a, b, lb, ub)
    dF, lower, dist, lag_gap = separable.error_bounds(x, d, q, a, b, lb, ub)
    scale = max(1.0, abs(F))
    assert np.all(x >= lb) and np.all(x <= ub)
    assert a @ x - b <= 1e-4 * max(1.0, abs(b))             # feasibility test of the outer loop
    assert dF <= 1.1e-4 * scale and dF >= lower - 1e-9 * scale  # F - LB test; weak duality
    assert np.linalg.norm(x - u) <= dist + 1e-9 and dist <= 1e-2 * np.linalg.norm(u)
    del Q
    torch.cuda.empty_cache()
    n1 = n + 1
    d, q, a, b, lb, ub = gen.separable_terms(n1, seed=7)
    Q = torch.zeros((n1, n1), dtype=torch.float64, device="cuda")
    Q.diagonal().copy_(dev(d))
    with pytest.raises(duq.DuqError) as e:
        duq.Solver(Q, dev(q), dev(a[None, :]), dev(np.array([-b])), dev(lb), dev(ub), **kw)
    assert e.value.code == duq.DUQ_EINVAL and f"n <= {n} " in str(e.value)
    del Q
    torch.cuda.empty_cache()


@pytest.mark.parametrize("engine", [duq.ENGINE_BLOCK, duq.ENGINE_GRID])
@pytest.mark.parametrize("kind,seed,method", [("pair", 1, duq.DFGM), ("pair", 2, duq.DGM),
                                              ("triple", 3, duq.DFGM), ("triple", 3, duq.DGM)])
def test_infeasible_certificate_parity(engine, kind, seed, method):
    # same iteration, same certificate (the multipliers) and iterate as the oracle
    print(f"[case] infeasible {kind} seed={seed} method={method} engine={engine}", flush=True)
    qp = gen.infeasible_qp(kind, seed)
    c = consts_of(qp)
    opts = dict(method=method, eps_out=1e-6, eps_in=1e-10, max_outer=100000)
    ref = dfom.dfom_solve(qp, dfom.Options(**opts), consts=c)
    assert ref.status == dfom.STATUS_INFEASIBLE
    with gpu_solver(qp, c, engine=engine, **opts) as s:
        x, lam, res = s.solve()
    assert res["status"] == duq.DUQ_EINFEASIBLE
    assert res["outer_iters"] == ref.outer_iters and res["inner_iters"] == ref.inner_iters
    close(lam, ref.lam, what="certificate")
    close(x, ref.x, what="x")
    w = qp.G.T @ lam
    assert np.all(lam >= 0.0) and lam @ qp.g + np.sum(np.minimum(qp.lb * w, qp.ub * w)) > 0.0


# ----------------------------------------------------------------------------
# constants (Lanczos) and robustness
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n,p,engine", [(50, 25, duq.ENGINE_BLOCK), (1536, 768, duq.ENGINE_GRID)])
def test_lanczos_constants(n, p, engine):
    print(f"[case] lanczos n={n}", flush=True)
    qp = gen.config1(n=n, p=p, seed=13) if n > 100 else gen.config0()
    ev = np.linalg.eigvalsh(qp.Q)
    g2 = np.linalg.norm(qp.G, 2) ** 2
    with duq.Solver(qp.Q, qp.q, qp.G, qp.g, qp.lb, qp.ub, engine=engine, lanczos_steps=96) as s:
        c = s.constants()
    sf = 1.02
    # safe side after the safety factor, and accurate before it
    assert c["lam_max"] >= ev[-1] and c["lam_max"] / sf == pytest.approx(ev[-1], rel=2e-3)
    assert c["lam_min"] <= ev[0] and c["lam_min"] * sf == pytest.approx(ev[0], rel=2e-2)
    assert c["G_norm2"] >= g2 and c["G_norm2"] / sf == pytest.approx(g2, rel=2e-3)


def test_estimated_constants_reach_accuracy():
    print("[case] estimated constants solve", flush=True)
    qp = gen.config0()
    with duq.Solver(qp.Q, qp.q, qp.G, qp.g, qp.lb, qp.ub, method=duq.DGM, eps_out=1e-4) as s:
        x, lam, res = s.solve()
    _, fstar, _ = ipm_qp(qp.Q, qp.q, qp.G, qp.g, qp.lb, qp.ub)
    assert res["status"] == duq.DUQ_OK
    assert abs(res["f"] - fstar) / abs(fstar) <= 1e-4


def test_invalid_inputs_rejected():
    qp = gen.random_dense_qp(10, 4, seed=3)
    Q = qp.Q.copy()
    Q[2, 3] = np.nan
    with pytest.raises(duq.DuqError) as e:
        duq.Solver(Q, qp.q, qp.G, qp.g, qp.lb, qp.ub)
    assert e.value.code == duq.DUQ_EINVAL
    lb = qp.lb.copy()
    lb[0] = 2.0
    with pytest.raises(duq.DuqError) as e:
        duq.Solver(qp.Q, qp.q, qp.G, qp.g, lb, qp.ub)
    assert e.value.code == duq.DUQ_EINVAL
    with pytest.raises(duq.DuqError):
        duq.Solver(qp.Q, qp.q, qp.G, qp.g, qp.lb, qp.ub, eps_out=0.0)


def test_max_outer_one_writes_iterate():
    qp = gen.config0()
    c = consts_of(qp)
    ref = dfom.dfom_solve(qp, dfom.Options(max_outer=1), consts=c)
    with gpu_solver(qp, c, max_outer=1) as s:
        x, lam, res = s.solve(check=False)
    assert res["status"] == duq.DUQ_EMAXITER and res["outer_iters"] == 1
    close(x, ref.x, what="x after one iteration")
    close(lam, ref.lam, what="lambda after one iteration")


def test_warm_start_inputs():
    qp = gen.config0()
    c = consts_of(qp)
    rng = np.random.default_rng(0)
    x0 = rng.uniform(-1.2, 1.2, qp.n)
    l0 = np.abs(rng.standard_normal(qp.p))
    ref = dfom.dfom_solve(qp, dfom.Options(max_outer=30, eps_out=1e-13, log_vectors=30), consts=c,
                          x_start=np.clip(x0, qp.lb, qp.ub), lam_start=l0)
    with gpu_solver(qp, c, max_outer=30, eps_out=1e-13, trace_outer=30) as s:
        x, lam, res = s.solve(x0=x0, lam0=l0, check=False)
        tr = s.trace(30)
    compare_trace(tr, ref.log, 30, "warm start")


def test_device_resident_inputs():
    import torch
    qp = gen.config0()
    c = consts_of(qp)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ref = dfom.dfom_solve(qp, dfom.Options(max_outer=50, eps_out=1e-13), consts=c)
    with duq.Solver(d(qp.Q), d(qp.q), d(qp.G), d(qp.g), d(qp.lb), d(qp.ub), max_outer=50, eps_out=1e-13,
                    lam_min=c.lam_min, lam_max=c.lam_max, G_norm2=c.G_norm2) as s:
        x, lam, res = s.solve(check=False)
    close(x, ref.x, what="x")


def test_deterministic_across_runs():
    qp = gen.config1(n=1536, p=768, seed=14)
    c = consts_of(qp)
    with gpu_solver(qp, c, max_outer=25, eps_out=1e-13, engine=duq.ENGINE_GRID) as s:
        x1, l1, r1 = s.solve(check=False)
        x2, l2, r2 = s.solve(check=False)
    assert np.array_equal(x1, x2) and np.array_equal(l1, l2)
    assert r1["inner_iters"] == r2["inner_iters"]


# ----------------------------------------------------------------------------
# a8: FP32-accumulated first phase, FP64 refinement from the same state
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n,p,engine,key", [(50, 25, duq.ENGINE_BLOCK, "config0"),
                                            (1536, 768, duq.ENGINE_GRID, None)])
def test_mixed_precision_switch_accuracy(n, p, engine, key):
    print(f"[case] two-phase precision n={n}", flush=True)
    qp = gen.config0() if key else gen.config1(n=n, p=p, seed=15)
    qp32 = qp.rounded(np.float32)
    _, fstar, _ = ipm_qp(qp32.Q, qp32.q, qp32.G, qp32.g, qp32.lb, qp32.ub)
    c = consts_of(qp32)
    with gpu_solver(qp, c, np.float32, method=duq.DFGM, eps_out=1e-4, eps_in=1e-8, engine=engine,
                    accumulate=duq.ACC_F32, switch_factor=10.0, switch_stall=20, trace_outer=4000) as s:
        x, lam, res = s.solve()
        tr = s.trace(4000)
    assert res["status"] == duq.DUQ_OK
    assert 0 < res["f64_outer_iters"] < res["outer_iters"]
    assert abs(res["f"] - fstar) / max(1.0, abs(fstar)) <= 1e-4
    assert res["feas"] / max(1.0, np.linalg.norm(qp.g)) <= 1e-4
    ks = tr["scalars"][:, 0]
    assert np.array_equal(ks, np.arange(1, len(ks) + 1))     # one numbering across both phases
    # the returned point is feasible to the tolerance on the FP64 data as well
    feas64 = np.linalg.norm(np.maximum(qp32.G @ x + qp32.g, 0))
    assert feas64 / max(1.0, np.linalg.norm(qp.g)) <= 1e-4 * (1 + 1e-6)


# ----------------------------------------------------------------------------
# planned solve: eq. choose_ein with a doubling guess of R_d (Sec. 3.1, Sec. 5)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("method", [duq.DFGM, duq.DGM])
def test_planned_solve_matches_oracle(method):
    from oracle import plan as oplan
    print(f"[case] planned solve m={method}", flush=True)
    qp = gen.config0()
    c = consts_of(qp)
    eps = 1e-3 if method == duq.DFGM else 1e-2
    ref = oplan.planned_solve(qp, method, eps, R0=0.05, max_rounds=16, consts=c)
    assert ref.status == dfom.STATUS_OK
    with gpu_solver(qp, c, method=method) as s:
        x, lam, r = s.solve_planned(eps, 0.05, max_rounds=16)
    assert r["status"] == duq.DUQ_OK and r["rounds"] == ref.rounds
    assert r["R"] == pytest.approx(ref.R, rel=1e-15)
    assert r["outer_iters"] == ref.outer_iters and r["inner_iters"] == ref.inner_iters
    close(x, ref.x, rel=1e-7, what="x")
    close(lam, ref.lam, rel=1e-7, what="lambda")
