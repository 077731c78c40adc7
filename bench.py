"""Benchmark of the DFOM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision f64|f32]
                    [--method dfgm|dgm] [--eps-in E] [--rho R] [--no-cpu]

Workload (one step = one end-to-end solve of the large single QP):
  random_dense_qp(n=8192, p=4096, seed=1, reg=0.01): Q = A^T A / n + 0.01 I with
  A (2n x n) i.i.d. N(0,1), G i.i.d. N(0,1), g = -(G x0) - s (strictly
  feasible), box [-1, 1].  Inputs are resident in HBM before timing.  A step
  runs duq_setup (Lanczos constants on the device, workspace) + duq_solve
  (Algorithm DFOM to the on-device outer test at eps_out = 1e-4) +
  duq_destroy.

Prints one JSON line.  `roofline` covers the dominant kernel (the
persistent DFOM kernel, one launch per solve): algorithmic matrix bytes per
launch / its HIP-event duration on the stream it runs on.  `cpu_baseline`
times the FP64 NumPy oracle on a bounded sample of the same solve.  The
default run adds `batched`: the shared-Hessian MPC batch (B = 4096) and the
uneven batch (B = 10 000) measured in the same process, each with its own
steps, roofline, plain per-QP rate, oracle check and CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFS = 78.6
METRIC = "QP solves/s at 1e-4 subopt+feas, batched vs plain; HBM GB/s; p50/p99 latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["f64", "f32"], default="f64")
    ap.add_argument("--accumulate", choices=["f64", "f32"], default="f64",
                    help="single QP with f32 storage: FP32-accumulated products until the test passes at "
                         "10 eps_out or stalls, then FP64 (the precision switch)")
    ap.add_argument("--method", choices=["dfgm", "dgm"], default="dfgm")
    ap.add_argument("--output", choices=["last", "avg"], default="last")
    ap.add_argument("--eps-in", type=float, default=None)
    ap.add_argument("--eps-out", type=float, default=1e-4)
    ap.add_argument("--rho", type=float, default=0.0)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--p", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="single workload: leave out the batched sub-results (MPC B=4096, uneven B=10000)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--workload", choices=["single", "uneven", "mpc", "serve", "studies", "sparse"],
                    default="single",
                    help="single large QP (default), uneven batch, or shared-Hessian MPC batch")
    ap.add_argument("--batch", type=int, default=None, help="instances of a batch workload")
    ap.add_argument("--plain-sample", type=int, default=48)
    ap.add_argument("--batch-max-outer", type=int, default=5000,
                    help="outer iteration cap per instance in the batched forms")
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="processes generating uneven instances (1: in-process, e.g. under a profiler)")
    ap.add_argument("--batch-engine", choices=["auto", "block", "tile"], default="auto",
                    help="batch kernel: tiles of 16 on MFMA (shared batches) or one workgroup per instance")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: Poisson arrivals per second")
    ap.add_argument("--duration", type=float, default=10.0, help="serve: seconds of arrivals")
    ap.add_argument("--large-frac", type=float, default=0.01, help="serve: share of n=4096 requests")
    ap.add_argument("--slice", type=int, default=16, help="serve: outer iterations per round")
    ap.add_argument("--serve-protocol", action="store_true",
                    help="serve: measure the saturation rate first, then serve at --load-frac of it")
    ap.add_argument("--sat-window", type=float, default=10.0, help="serve: seconds of the saturation run")
    ap.add_argument("--load-fracs", default="0.8,0.5,0.25",
                    help="serve: offered shares of the saturation rate, one run each")
    ap.add_argument("--sparse-n", type=int, default=2_000_000, help="sparse: flows (variables)")
    ap.add_argument("--sparse-p", type=int, default=500_000, help="sparse: links (rows of G)")
    ap.add_argument("--print-source-hash", action="store_true", help="hashes of the profiled kernels' sources")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a plain device copy of 1 GiB (counter calibration)")
    return ap.parse_args()


def copy_probe():
    import torch
    x = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)   # 1 GiB
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": x.numel() * 8, "launches": 3}))


def source_hash(files) -> str:
    """Hash of the HIP sources a kernel is built from; counter figures are
    only valid for the build they came from."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(files):
        path = os.path.join(ROOT, "paper_1504_05708_amd", "csrc", name)
        h.update(name.encode())
        h.update(open(path, "rb").read() if os.path.exists(path) else b"missing")
    return h.hexdigest()[:16]


# Sources of each profiled kernel (its entry file and the headers it uses).
KERNEL_SOURCES = {
    "dfom_kernel": ["kernels.hip", "dfom_solver.h", "device_common.h", "internal.h", "launch_util.h"],
    "dfom_batch_kernel": ["batch_kernels.hip", "batch.h", "lanczos.h", "dfom_solver.h", "device_common.h",
                          "internal.h", "launch_util.h"],
    "dfom_tile_kernel": ["batch_kernels.hip", "shared_tile.h", "device_common.h", "internal.h", "launch_util.h"],
}


def measured_traffic(profile_name: str, kernel: str):
    """HBM bytes per launch from a committed rocprofv3 summary (FETCH_SIZE and
    WRITE_SIZE, scaled by the copy calibration), or None when the kernel
    sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", profile_name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_hash") != source_hash(KERNEL_SOURCES[kernel]):
        return None
    return float(kv["traffic_bytes_per_launch"])


def lam_min_is_lower_bound(Q, lam_min) -> bool:
    """Whether Q - lam_min I has a Cholesky factor, i.e. whether an estimated
    lambda_min(Q) (the sigma_in of the inner certificate) is below the true
    one, to rounding."""
    try:
        np.linalg.cholesky(np.asarray(Q, np.float64) - lam_min * np.eye(Q.shape[0]))
        return True
    except np.linalg.LinAlgError:
        return False


def reference_fstar(key):
    path = os.path.join(ROOT, "tests", "golden", "reference_values.json")
    if os.path.exists(path):
        vals = json.load(open(path))
        if key in vals:
            return vals[key]["fstar"]
    return None


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {a.gpus}); "
              "the single large QP would shard by rows over RCCL, which is not built.", file=sys.stderr)
        sys.exit(2)
    if a.print_source_hash:
        print(json.dumps({k: source_hash(v) for k, v in KERNEL_SOURCES.items()}))
        return
    if a.copy_probe:
        copy_probe()
        return
    if a.workload == "serve":
        bench_serve(a)
        return
    if a.workload == "studies":
        bench_studies(a)
        return
    if a.workload == "sparse":
        r = sparse_result(a, a.sparse_n, a.sparse_p, a.steps, a.warmup)
        r["metric"] = METRIC
        print(json.dumps(r), flush=True)
        return
    if a.workload != "single":
        bench_batch(a)
        return
    import torch
    from paper_1504_05708_amd import duq, gen

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    duq.lib()   # fails loudly when the HIP library is missing
    method = duq.DFGM if a.method == "dfgm" else duq.DGM
    output = duq.LAST if a.output == "last" else duq.AVG
    eps_in = a.eps_in if a.eps_in is not None else (1e-8 if method == duq.DFGM else 1e-6)
    t0 = time.time()
    qp = gen.config1(n=a.n, p=a.p, seed=1)
    gen_s = time.time() - t0
    npdt = np.float64 if a.precision == "f64" else np.float32
    s_bytes = 8 if a.precision == "f64" else 4
    dev = lambda v, dt=np.float64: torch.from_numpy(np.ascontiguousarray(v.astype(dt))).cuda()
    Qd, Gd = dev(qp.Q, npdt), dev(qp.G, npdt)
    qd, gd, lbd, ubd = dev(qp.q), dev(qp.g), dev(qp.lb), dev(qp.ub)
    torch.cuda.synchronize()
    opts = dict(method=method, output=output, eps_out=a.eps_out, eps_in=eps_in, rho=a.rho,
                max_outer=200000, engine=duq.ENGINE_GRID)
    if a.accumulate == "f32":
        assert a.precision == "f32", "--accumulate f32 needs --precision f32"
        opts.update(accumulate=duq.ACC_F32, switch_factor=10.0, switch_stall=20)

    def step():
        t = time.perf_counter()
        s = duq.Solver(Qd, qd, Gd, gd, lbd, ubd, **opts)
        t_setup = time.perf_counter() - t
        x, lam, res = s.solve()
        consts = s.constants()
        s.close()
        return x, lam, res, consts, t_setup

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    results = []
    t_wall = time.perf_counter()
    ev0.record()
    for _ in range(a.steps):
        results.append(step())
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ev_ms = ev0.elapsed_time(ev1)
    ms_per_step = 1e3 * wall / a.steps
    x, lam, res, consts, _ = results[-1]
    for r in results:
        assert r[2]["status"] == duq.DUQ_OK, r[2]
    n, p = a.n, a.p
    kern_ms = [r[2]["time_ms"] for r in results]
    setup_ms = [1e3 * r[4] for r in results]
    kern_avg = float(np.mean(kern_ms))
    # algorithmic matrix bytes of one launch: every Q product (inner steps +
    # the initial warm-start product), one G product per outer iteration and
    # per extra last-iterate solve (rho = 0), and the G rows actually read by
    # G^T v (rows with v_i = 0 need no read).
    inner, outer, gt_rows = res["inner_iters"], res["outer_iters"], res["gt_rows"]
    nn = float(n) * n * s_bytes
    pn = float(p) * n * s_bytes
    if a.rho > 0.0:
        q_products = inner + 1
        g_products = inner + 1
    else:
        q_products = inner + 1
        g_products = outer + (1 if (method == duq.DFGM and output == duq.LAST) else 0)
    alg_bytes = q_products * nn + g_products * pn + gt_rows * n * s_bytes
    achieved = alg_bytes / (kern_avg * 1e-3) / 1e9
    # the profiled configurations: the default large QP with FP64 or FP32 storage
    profiled = (n == 8192 and p == 4096 and a.precision in ("f64", "f32") and a.accumulate == "f64"
                and method == duq.DFGM and output == duq.LAST and eps_in == 1e-8 and a.rho == 0.0
                and a.eps_out == 1e-4)
    traffic = measured_traffic(f"dfom_kernel_config1_{a.precision}.txt", "dfom_kernel") if profiled else None
    F, LB, feas = res["f"], res["lb_dual"], res["feas"]
    gnorm = float(np.linalg.norm(qp.g))
    acc = {"cert_subopt_rel": (F - LB) / max(1.0, abs(F)), "feas_rel": feas / max(1.0, gnorm)}
    fref = reference_fstar("config1_f64" if a.precision == "f64" else "config1_f32")
    if fref is not None and a.n == 8192 and a.p == 4096:
        acc["subopt_rel_vs_ipm"] = abs(F - fref) / max(1.0, abs(fref))
    value = a.steps / wall
    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "f64" else "f32-storage/f64",
        "data": "synthetic",
        "config": {
            "workload": f"single dense QP n={n} p={p}: Q=A^T A/n+0.01I (A {2 * n}x{n} N(0,1)), G N(0,1), "
                        f"g=-(G x0)-s strictly feasible, box [-1,1], seed 1; "
                        f"{a.method.upper()}-{a.output} eps_out={a.eps_out:g} eps_in={eps_in:g} rho={a.rho:g}; "
                        f"Q,G stored {a.precision}, "
                        + ("FP32-accumulated products, then FP64 (precision switch)" if a.accumulate == "f32"
                           else "FP64 arithmetic")
                        + "; end-to-end step = setup (Lanczos constants) + solve",
            "n": n, "p": p, "storage": a.precision, "method": a.method, "output": a.output,
            "eps_out": a.eps_out, "eps_in": eps_in, "rho": a.rho,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "dfom_kernel (persistent cooperative, one launch per solve)",
            "alg_bytes_per_launch": alg_bytes,
            "launch_ms_avg": round(kern_avg, 3),
        },
        "solve": {"outer_iters": outer, "inner_iters": inner, "gt_rows_read": gt_rows,
                  "f64_outer_iters": res["f64_outer_iters"],
                  "f": F, "lb": LB, "feas": feas, "online_solves_per_s": round(1e3 / kern_avg, 4),
                  "setup_ms_avg": round(float(np.mean(setup_ms)), 2),
                  "event_ms_per_step": round(ev_ms / a.steps, 3),
                  "constants": consts},
        "accuracy": acc,
        "sigma_check": {"lam_min_estimate": consts["lam_min"],
                        "is_lower_bound": lam_min_is_lower_bound(qp.Q if a.precision == "f64"
                                                                 else qp.Q.astype(np.float32), consts["lam_min"]),
                        "how": "Cholesky of Q - lam_min I on the host (the inner certificate's sigma)"},
        "gen_seconds": round(gen_s, 1),
    }
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(qp if a.precision == "f64" else qp.rounded(np.float32), consts, res,
                                            method, output, eps_in, a)
    if not a.no_batched:
        # the batched forms on the same GPU in the same run: the shared-Hessian
        # MPC batch (4096 instances, MFMA tiles) and the uneven batch (10 000
        # independent QPs, FP32 storage), each with its own roofline, plain
        # per-QP rate, oracle check and CPU baseline
        del Qd, Gd
        torch.cuda.empty_cache()
        line["batched"] = {}
        for key, wl, B, st, wu, prec in (("mpc_shared_B4096", "mpc", 4096, 20, 5, "f64"),
                                         ("uneven_B10000", "uneven", 10000, 2, 1, "f32")):
            print(f"[bench] batched {key}", file=sys.stderr, flush=True)
            r = batch_result(a, wl, B, st, wu, prec, not a.no_cpu)
            for k in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
                r.pop(k, None)
            line["batched"][key] = r
            torch.cuda.empty_cache()
        # the compressed-row path on a large sparse QP (Sec. 5.1)
        print("[bench] sparse", file=sys.stderr, flush=True)
        r = sparse_result(a, 2_000_000, 500_000, 5, 1)
        for k in ("n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
            r.pop(k, None)
        line["sparse_num_n2M"] = r
    print(json.dumps(line), flush=True)


def cpu_baseline(qp, consts, res, method, output, eps_in, a):
    """The FP64 oracle on the host cores: the first outer iterations of the same
    solve (same constants), stopped after about `cpu_seconds`, then scaled by
    matrix-pass count to the full solve the GPU performed."""
    from oracle import dfom
    cores = len(os.sched_getaffinity(0))
    opts = dfom.Options(method=method, output=output, eps_out=a.eps_out, eps_in=eps_in, rho=a.rho,
                        lam_min=consts["lam_min"], lam_max=consts["lam_max"], G_norm2=consts["G_norm2"])
    # a one-iteration probe sizes the sample to about `cpu_seconds`
    opts.max_outer = 1
    t0 = time.perf_counter()
    dfom.dfom_solve(qp, opts)
    t_one = time.perf_counter() - t0
    k = int(max(1, min(res["outer_iters"], a.cpu_seconds / max(t_one, 1e-3))))
    opts.max_outer = k
    t1 = time.perf_counter()
    r = dfom.dfom_solve(qp, opts)
    sample_s = time.perf_counter() - t1
    # one inner step of the oracle reads Q twice (gradient at y and at x), one outer
    # iteration reads G twice (G^T mu and G u): weight passes by bytes
    n, p = qp.n, qp.p
    per_inner = 2.0 * n * n
    per_outer = 2.0 * p * n
    sample_work = r.inner_iters * per_inner + k * per_outer
    full_work = res["inner_iters"] * per_inner + res["outer_iters"] * per_outer
    est_s = sample_s * full_work / max(sample_work, 1.0)
    return {"value": round(1.0 / est_s, 6), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"first {k} outer iterations ({r.inner_iters} inner steps) of the same solve in "
                      f"{sample_s:.1f} s, scaled by matrix passes to the full solve "
                      f"({res['outer_iters']} outer, {res['inner_iters']} inner)",
            "est_seconds_per_solve": round(est_s, 1)}


def sparse_alg_bytes(n, p, nnzQ, nnzG, s, inner, outer, dfgm_last=True):
    """Algorithmic HBM bytes of one sparse solve: per product the matrix's
    values and column indices ((s + 4) bytes per nonzero), its row offsets
    and the vector it multiplies read once; per inner step the seven n-vectors
    of the FGM step (x^t, x^{t-1}, Q x^t, Q x^{t-1}, c read; x^{t+1},
    Q x^{t+1} written); per outer iteration the products G u and G^T w and
    five p-vectors of the dual step."""
    q_prod = (s + 4.0) * nnzQ + 8.0 * (n + 1) + 8.0 * n
    g_prod = (s + 4.0) * nnzG + 8.0 * (p + 1) + 8.0 * n
    gt_prod = (s + 4.0) * nnzG + 8.0 * (n + 1) + 8.0 * p
    g_products = outer + (1 if dfgm_last else 0)
    return ((inner + 1) * q_prod + inner * 56.0 * n + g_products * g_prod + outer * (gt_prod + 40.0 * p))


def sparse_result(a, n, p, steps, warmup):
    """The compressed-row path (duq_setup_csr) on a network-utility QP with n
    flows over p links (gen.sparse_num_qp): solves of a set-up handle, inputs
    resident in HBM; roofline on the algorithmic bytes of sparse_alg_bytes;
    accuracy from the on-device certificate and KKT residuals computed on the
    host with sparse products (the dense oracle cannot hold this size)."""
    import torch
    from paper_1504_05708_amd import duq, gen

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    duq.lib()
    t0 = time.time()
    sq = gen.sparse_num_qp(n, p, seed=5)
    gen_s = time.time() - t0
    eps_in = 1e-8
    opts = dict(method=duq.DFGM, output=duq.LAST, eps_out=1e-4, eps_in=eps_in, max_outer=200000,
                engine=duq.ENGINE_GRID)
    t1 = time.perf_counter()
    s = duq.Solver(sq.Q, sq.q, sq.G, sq.g, sq.lb, sq.ub, **opts)
    setup_s = time.perf_counter() - t1
    for _ in range(warmup):
        s.solve()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    results = [s.solve() for _ in range(steps)]
    wall = time.perf_counter() - t2
    consts = s.constants()
    s.close()
    x, lam, res = results[-1]
    ok = sum(r[2]["status"] == duq.DUQ_OK for r in results)
    kern_ms = float(np.mean([r[2]["time_ms"] for r in results]))
    alg = sparse_alg_bytes(n, p, sq.Q.nnz, sq.G.nnz, 8, res["inner_iters"], res["outer_iters"])
    achieved = alg / (kern_ms * 1e-3) / 1e9

    def mv(M, v):
        rows = np.repeat(np.arange(M.rows), np.diff(M.rowptr))
        return np.bincount(rows, weights=M.val * v[M.col], minlength=M.rows)

    def mtv(M, w):
        rows = np.repeat(np.arange(M.rows), np.diff(M.rowptr))
        return np.bincount(M.col, weights=M.val * w[rows], minlength=M.cols)

    r_ = mv(sq.G, x) + sq.g
    grad = mv(sq.Q, x) + sq.q + mtv(sq.G, lam)
    F_host = 0.5 * float(x @ mv(sq.Q, x)) + float(sq.q @ x)
    F, LB = res["f"], res["lb_dual"]
    return {
        "metric": METRIC, "value": round(ok / wall, 4), "unit": "solves/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": round(1e3 * wall / steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"sparse network-utility QP: n={n} flows in [0,1], p={p} links, each flow on 8 "
                               f"random links (G 0/1, nnz {sq.G.nnz}), capacities G x0 + U(0,0.3), Q diagonal "
                               f"U(1,2) + band-2 coupling U(-0.1,0.1) (nnz {sq.Q.nnz}), q ~ -U(0.5,1.5), seed 5; "
                               f"compressed rows (duq_setup_csr), x read in place; DFGM-last eps_out=1e-4 "
                               f"eps_in={eps_in:g}; step = one solve of a set-up handle (inputs in HBM)",
                   "n": n, "p": p, "nnzQ": sq.Q.nnz, "nnzG": sq.G.nnz, "storage": "f64"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": (measured_traffic("dfom_kernel_sparse_num2M_f64.txt", "dfom_kernel")
                                 if (n, p) == (2_000_000, 500_000) else None),
                     "kernel": "dfom_kernel<double,double,false,false,true> (sparse, persistent cooperative)",
                     "alg_bytes_per_launch": alg, "launch_ms_avg": round(kern_ms, 3)},
        "solve": {"instances_ok": ok, "instances_failed": steps - ok, "outer_iters": res["outer_iters"],
                  "inner_iters": res["inner_iters"], "us_per_inner": round(1e3 * kern_ms / res["inner_iters"], 2),
                  "setup_s": round(setup_s, 3), "constants": consts},
        "accuracy": {"cert_subopt_rel": (F - LB) / max(1.0, abs(F)),
                     "feas_rel": float(np.linalg.norm(np.maximum(r_, 0.0))) / max(1.0, float(np.linalg.norm(sq.g))),
                     "stationarity_inf": float(np.max(np.abs(x - np.clip(x - grad, sq.lb, sq.ub)))),
                     "F_device_minus_host_rel": abs(F - F_host) / max(1.0, abs(F_host))},
        "gen_seconds": round(gen_s, 1),
        "cpu_baseline": None,
        "cpu_baseline_note": "the oracle works on dense matrices; at this size they would need "
                             f"{8.0 * n * (n + p) / 1e12:.0f} TB",
    }


def bench_batch(a):
    """--workload uneven|mpc: one JSON line for a batched form."""
    line = batch_result(a, a.workload, a.batch, a.steps, a.warmup, a.precision, not a.no_cpu)
    print(json.dumps(line), flush=True)


def batch_result(a, workload, B, steps, warmup, precision, with_cpu, oracle_sample=None):
    """Batched forms: one duq_solve_batch over the whole batch per step, against
    the plain per-QP GPU solver (duq_setup + duq_solve per instance, constants
    passed so it does not re-estimate them) on a sample of the same instances.
    `value` counts the instances that passed their outer test only.  A seeded
    sample is checked against the oracle: suboptimality against the oracle's
    interior-point optimum, feasibility, and the distance to the oracle's DFOM
    solution of the same instance (same constants)."""
    import torch
    from paper_1504_05708_amd import duq, gen

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    duq.lib()
    method = duq.DFGM if a.method == "dfgm" else duq.DGM
    output = duq.LAST if a.output == "last" else duq.AVG
    eps_in = a.eps_in if a.eps_in is not None else (1e-8 if method == duq.DFGM else 1e-6)
    # max_outer: about 40 times the mean outer count of the uneven batch; the
    # few DFGM instances that plateau above the test (inner accuracy too coarse
    # for DFGM, Sec. 3.1) end there as failures instead of holding one
    # workgroup for 200 000 iterations after every other instance is done
    opts = dict(method=method, output=output, eps_out=a.eps_out,
                eps_in=eps_in, rho=a.rho, max_outer=a.batch_max_outer,
                engine={"auto": duq.ENGINE_AUTO, "block": duq.ENGINE_BLOCK, "tile": duq.ENGINE_TILE}[a.batch_engine])
    npdt = np.float32 if precision == "f32" else np.float64
    s_bytes = 4 if npdt == np.float32 else 8
    cuda = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()
    t0 = time.time()
    workers = max(1, min(a.gen_workers, len(os.sched_getaffinity(0))))
    if workload == "uneven":
        B = B or 10000
        ub = gen.uneven_batch(B=B, seed=3, dtype=npdt, workers=workers)
        gen_s = time.time() - t0
        dev = gen.UnevenBatch(ub.n, ub.p, cuda(ub.Q), cuda(ub.G), cuda(ub.q), cuda(ub.g), cuda(ub.lb),
                              cuda(ub.ub), ub.qoff, ub.goff, ub.voff, ub.coff)
        ns, ps = ub.n.astype(np.int64), ub.p.astype(np.int64)

        def run_batch(consts=None, device_out=True):
            return duq.solve_batch_uneven(dev, device_out=device_out, **opts)

        def plain_one(i, c):
            n, p = int(ns[i]), int(ps[i])
            Qi = dev.Q[ub.qoff[i]:ub.qoff[i] + n * n].view(n, n)
            Gi = dev.G[ub.goff[i]:ub.goff[i] + p * n].view(p, n)
            sl = slice(int(ub.voff[i]), int(ub.voff[i]) + n)
            sc = slice(int(ub.coff[i]), int(ub.coff[i]) + p)
            with duq.Solver(Qi, dev.q[sl], Gi, dev.g[sc], dev.lb[sl], dev.ub[sl], lam_min=c["lam_min"],
                            lam_max=c["lam_max"], G_norm2=c["G_norm2"], **dict(opts, engine=duq.ENGINE_BLOCK)) as sv:
                return sv.solve()[2]

        def instance(i):
            return ub.instance(i)      # the stored (rounded) data, promoted to FP64

        def x_of(X, i):
            return X[int(ub.voff[i]):int(ub.voff[i]) + int(ns[i])]
        desc = (f"uneven batch of {B} independent dense QPs, n~U{{20..512}}, p=n//2, "
                f"Q=A^T A/n+0.1I, box [-1,1], seed 3; Q,G stored {precision}")
    else:
        B = B or 4096
        sysm = gen.mpc_system(seed=2)
        X0, Ql, Gl = gen.mpc_batch(sysm, B, seed=20)
        gen_s = time.time() - t0
        Hd, Gd = cuda(sysm.H.astype(npdt)), cuda(sysm.G.astype(npdt))
        lbd, ubd, Qld, Gld = cuda(sysm.lb), cuda(sysm.ub), cuda(Ql), cuda(Gl)
        ns = np.full(B, sysm.n, np.int64)
        ps = np.full(B, sysm.p, np.int64)

        def run_batch(consts=None, device_out=True):
            # the constants belong to the shared system: estimated once, then given
            return duq.solve_batch_shared(Hd, Gd, lbd, ubd, Qld, Gld, constants=consts, device_out=device_out,
                                          **opts)

        def plain_one(i, c):
            with duq.Solver(Hd, Qld[i], Gd, Gld[i], lbd, ubd, lam_min=c["lam_min"], lam_max=c["lam_max"],
                            G_norm2=c["G_norm2"], **dict(opts, engine=duq.ENGINE_BLOCK)) as sv:
                return sv.solve()[2]

        def instance(i):
            qp = gen.mpc_instance(sysm, X0[i])
            return qp if npdt == np.float64 else qp.rounded(npdt)

        def x_of(X, i):
            return X[i]
        desc = (f"shared-Hessian batch of {B} condensed MPC QPs (nx=12, nu=4, N=30: n=120, p=720, "
                f"|u|<=1, |x_k|<=5), x0~U(-1,1)^12, seed 2/20; H,G stored {precision}")
    torch.cuda.synchronize()
    # end-to-end call: constants estimated, outputs copied to the host
    t = time.perf_counter()
    _, _, res0 = run_batch(None, device_out=False)
    e2e_s = time.perf_counter() - t
    sys_consts = None
    if workload == "mpc":
        sys_consts = (res0[0]["lam_min"], res0[0]["lam_max"], res0[0]["G_norm2"])
    for _ in range(warmup):
        run_batch(sys_consts)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        X, L, res = run_batch(sys_consts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    kern_ms = res[0]["time_ms"]
    ok = sum(r["status"] == duq.DUQ_OK for r in res)
    value = ok * steps / wall
    engine = res[0]["engine"]
    # algorithmic matrix bytes of one launch, per instance: every Q product
    # (inner steps + warm start), the G product of each outer iteration and of
    # the extra last-iterate solve, the rows read by G^T mu, and the Lanczos
    # estimate (k steps on Q and on G^T G) unless the constants were shared
    extra = 1 if (method == duq.DFGM and output == duq.LAST) else 0
    alg = 0.0
    for i, r in enumerate(res):
        n, p = float(ns[i]), float(ps[i])
        k = min(96, n)
        lz = (k * n * n + 2 * k * p * n) if workload == "uneven" else 0.0
        alg += ((r["inner_iters"] + 1) * n * n + (r["outer_iters"] + extra) * p * n + r["gt_rows"] * n + lz) * s_bytes
    achieved = alg / (kern_ms * 1e-3) / 1e9
    if engine == duq.ENGINE_TILE:
        # matrix-core kernel: algorithmic FP64 flops of the Q products (inner
        # steps + warm start), the G products (one per outer iteration and per
        # last-iterate solve) and the G^T rows with a nonzero multiplier
        flops = 0.0
        for i, r in enumerate(res):
            n, p = float(ns[i]), float(ps[i])
            flops += (2.0 * n * n * (r["inner_iters"] + 1) + 2.0 * p * n * (r["outer_iters"] + extra)
                      + 2.0 * n * r["gt_rows"])
        tf = flops / (kern_ms * 1e-3) / 1e12
        tr = (measured_traffic("dfom_tile_kernel_mpc4096_f64.txt", "dfom_tile_kernel")
              if (workload == "mpc" and precision == "f64" and B == 4096) else None)
        roof = {"bound": "mfma", "achieved": round(tf, 2), "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s",
                "frac": round(tf / FP64_MFMA_PEAK_TFS, 4), "traffic": tr, "kernel": "dfom_tile_kernel",
                "alg_flops_per_launch": flops, "launch_ms": round(kern_ms, 3),
                "note": "FP64 MFMA 16x16x4; Q held in registers, X through LDS, G through L2; flops of masked (finished) "
                        "columns, of padding and of G^T products skipped for zero multipliers are not counted"}
    else:
        tr = (measured_traffic(f"dfom_batch_kernel_uneven{B}_{precision}.txt", "dfom_batch_kernel")
              if workload == "uneven" else None)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
                "kernel": "dfom_batch_kernel", "alg_bytes_per_launch": alg, "launch_ms": round(kern_ms, 3),
                "note": "algorithmic bytes: every matrix read of every instance (768 concurrent instances "
                        "exceed L2 and MALL, so they stream from HBM)"}
    # plain per-QP solver on a sample spread over the batch
    S = min(a.plain_sample, B)
    idx = np.linspace(0, B - 1, S).astype(int)
    consts = [dict(lam_min=res[i]["lam_min"], lam_max=res[i]["lam_max"], G_norm2=res[i]["G_norm2"]) for i in idx]
    plain_one(int(idx[0]), consts[0])
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain_ok = 0
    for i, c in zip(idx, consts):
        plain_ok += plain_one(int(i), c)["status"] == duq.DUQ_OK
    torch.cuda.synchronize()
    plain_wall = time.perf_counter() - t
    # plain rate over the whole batch: the sample's mean time per solve, weighted
    # by the work of the sampled instances relative to the batch, counting the
    # share of instances that pass
    w_all = float(np.sum(ns * ns + ps * ns))
    w_s = float(np.sum(ns[idx] * ns[idx] + ps[idx] * ns[idx]))
    plain_rate = (plain_ok / S) * B / (plain_wall * (w_all / w_s))
    feas_rel = max(r["feas"] for r in res)
    cert = max((r["f"] - r["lb_dual"]) / max(1.0, abs(r["f"])) for r in res)
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "solves/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": round(1e3 * wall / steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if precision == "f64" else "f32-storage/f64",
        "data": "synthetic",
        "config": {"workload": desc + f"; {a.method.upper()}-{a.output} eps_out={a.eps_out:g} eps_in={eps_in:g}; "
                               f"one persistent launch per batch ({'MFMA tiles of 16 instances' if engine == duq.ENGINE_TILE else 'one workgroup per instance'}); "
                               f"inputs and outputs in HBM; value counts the instances that passed their "
                               f"outer test"
                               + ("; system constants estimated once (end_to_end_solves_per_s includes the "
                                  "estimate and the host copy of the outputs)" if workload == "mpc" else ""),
                   "B": B, "storage": precision},
        "plain_solves_per_s": round(plain_rate, 3),
        "speedup_vs_plain": round(value / plain_rate, 1),
        "roofline": roof,
        "end_to_end_solves_per_s": round(ok / e2e_s, 2),
        "kernel_solves_per_s": round(ok / (kern_ms * 1e-3), 1),
        "solve": {"instances_ok": ok, "instances_failed": B - ok,
                  "failed_status": sorted({int(r["status"]) for r in res if r["status"] != duq.DUQ_OK}),
                  "max_cert_subopt_rel": cert, "max_feas_abs": feas_rel,
                  "outer_mean": float(np.mean([r["outer_iters"] for r in res])),
                  "inner_mean": float(np.mean([r["inner_iters"] for r in res]))},
        "gen_seconds": round(gen_s, 1),
    }
    # every estimated lambda_min (the inner certificate's sigma) against the
    # true spectrum: the shared system once, each uneven instance
    if workload == "mpc":
        checks = [lam_min_is_lower_bound(sysm.H.astype(npdt), res0[0]["lam_min"])]
    else:
        checks = [lam_min_is_lower_bound(instance(i).Q, res[i]["lam_min"]) for i in range(B)]
    out["sigma_check"] = {"estimates_checked": len(checks), "not_a_lower_bound": len(checks) - int(sum(checks)),
                          "how": "Cholesky of Q - lam_min I on the host"}
    if with_cpu:
        from oracle import dfom
        from oracle.ipm import ipm_qp
        # accuracy against the oracle on a seeded sample: the interior-point
        # optimum f* and the oracle's own DFOM solution with the same constants
        rs = np.random.default_rng(7)
        m = oracle_sample or (6 if workload == "uneven" else 8)
        sel = np.sort(rs.choice(B, size=min(m, B), replace=False))
        Xh = X.cpu().numpy() if hasattr(X, "cpu") else X
        sub, feas_o, dx, fo_rel = [], [], [], []
        for i in sel:
            qp = instance(int(i))
            x = np.asarray(x_of(Xh, int(i)), float)
            _, fstar, _ = ipm_qp(qp.Q, qp.q, qp.G, qp.g, qp.lb, qp.ub)
            F = float(0.5 * x @ qp.Q @ x + qp.q @ x)
            sub.append(abs(F - fstar) / max(1.0, abs(fstar)))
            feas_o.append(float(np.linalg.norm(np.maximum(qp.G @ x + qp.g, 0.0))) / max(1.0, np.linalg.norm(qp.g)))
            ref = dfom.dfom_solve(qp, dfom.Options(method=method, output=output, eps_out=a.eps_out, eps_in=eps_in,
                                                   rho=a.rho, max_outer=a.batch_max_outer, lam_min=res[i]["lam_min"],
                                                   lam_max=res[i]["lam_max"], G_norm2=res[i]["G_norm2"]))
            dx.append(float(np.max(np.abs(x - ref.x))))
            fo_rel.append(abs(F - ref.F) / max(1.0, abs(ref.F)))
        out["vs_oracle"] = {"instances": [int(i) for i in sel], "max_subopt_rel_vs_ipm": max(sub),
                            "max_feas_rel": max(feas_o), "max_abs_x_minus_oracle_dfom": max(dx),
                            "max_rel_F_minus_oracle_dfom": max(fo_rel)}
        # the oracle's throughput on the host cores (a baseline, not a target)
        t = time.perf_counter()
        done = 0
        for i, c in zip(idx, consts):
            qp = instance(int(i))
            dfom.dfom_solve(qp, dfom.Options(method=method, output=output, eps_out=a.eps_out, eps_in=eps_in,
                                             rho=a.rho, max_outer=a.batch_max_outer, lam_min=c["lam_min"],
                                             lam_max=c["lam_max"], G_norm2=c["G_norm2"]))
            done += 1
            if time.perf_counter() - t > a.cpu_seconds:
                break
        cs = time.perf_counter() - t
        w_done = float(np.sum(ns[idx[:done]] ** 2 + ps[idx[:done]] * ns[idx[:done]]))
        out["cpu_baseline"] = {"value": round(B / (cs * w_all / w_done), 4), "unit": "solves/s",
                               "cores": len(os.sched_getaffinity(0)), "kind": "oracle",
                               "sample": f"{done} instances of the batch solved by the oracle in {cs:.1f} s, "
                                         f"scaled by matrix work to all {B}"}
    return out


def bench_serve(a):
    """--workload serve: the offered rate --rate for --duration seconds, or
    with --serve-protocol the capacity of one GPU: a saturation run (offered
    rate far above capacity for --sat-window seconds; the sustained rate is
    the completions over the span the server stayed busy, drain included),
    then a run of --duration seconds at each fraction in --load-fracs of that
    rate, whose latencies are the service's own when it keeps up (the drain
    time after the last arrival shows whether it did)."""
    if not a.serve_protocol:
        print(json.dumps(serve_run(a, a.rate, a.duration)), flush=True)
        return
    sat = serve_run(a, a.rate, a.sat_window)
    loads = []
    for frac in [float(f) for f in a.load_fracs.split(",")]:
        rate = round(frac * sat["value"], 1)
        r = serve_run(a, rate, a.duration)
        loads.append({"load_frac": frac, "offered_per_s": r["offered_per_s"], "solves_per_s": r["value"],
                      "drain_s_after_last_arrival": r["drain_s_after_last_arrival"], "latency_ms": r["latency_ms"],
                      "solve": r["solve"], "requests": r["config"]["requests"]})
        if len(loads) == 1:
            line = r
    line["saturation"] = {"offered_per_s": sat["offered_per_s"], "sustained_solves_per_s": sat["value"],
                          "completed_in_window_per_s": sat["completed_in_window_per_s"],
                          "drain_s_after_last_arrival": sat["drain_s_after_last_arrival"],
                          "window_s": a.sat_window, "requests": sat["config"]["requests"],
                          "latency_ms": sat["latency_ms"], "solve": sat["solve"]}
    line["loads"] = loads
    line["config"]["workload"] = (f"serving at fractions {a.load_fracs} of the sustained rate of a saturation run "
                                  f"({sat['value']:g}/s: all of {a.rate:g}/s offered for {a.sat_window:g} s, "
                                  f"completions over the busy span); the top-level figures are those of the first "
                                  f"fraction: " + line["config"]["workload"])
    print(json.dumps(line), flush=True)


def serve_run(a, rate, duration):
    """Serving loop: Poisson arrivals of a request mix, submitted from one host
    thread to duq_submit, collected with duq_poll.  Mix: `large_frac` dense QPs
    n=4096, p=2048 (config-1 generator; a pool of 8 (Q, G) made before the
    timed window, fresh q, g per request), the rest half uneven random QPs
    (n ~ U{20..512}, p = n//2) and half condensed MPC requests against 8
    registered systems (seeds 40..47, fresh x0).  Matrices stored FP32."""
    import threading

    import torch
    from paper_1504_05708_amd import duq, gen

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    duq.lib()
    method = duq.DFGM if a.method == "dfgm" else duq.DGM
    eps_in = a.eps_in if a.eps_in is not None else (1e-8 if method == duq.DFGM else 1e-6)
    opts = dict(method=method, output=duq.LAST if a.output == "last" else duq.AVG, eps_out=a.eps_out,
                eps_in=eps_in, rho=a.rho, max_outer=200000, serve_slice=a.slice)
    npdt = np.float32 if a.precision == "f32" else np.float64
    rng = np.random.default_rng(4)
    t0 = time.time()
    # arrivals and classes
    gaps = rng.exponential(1.0 / rate, int(rate * duration * 1.5) + 16)
    arr = np.cumsum(gaps)
    arr = arr[arr < duration]
    R = len(arr)
    u = rng.uniform(size=R)
    cls = np.where(u < a.large_frac, 2, np.where(u < a.large_frac + (1 - a.large_frac) / 2, 0, 1))
    n_unev = int(np.sum(cls == 0))
    workers = max(1, min(a.gen_workers, len(os.sched_getaffinity(0))))
    ub = gen.uneven_batch(B=max(n_unev, 1), seed=4, dtype=npdt, workers=workers)
    systems = [gen.mpc_system(seed=40 + j) for j in range(8)]
    n_large = int(np.sum(cls == 2))
    pool = []
    if n_large:
        for j in range(8):
            qp = gen.config1(n=4096, p=2048, seed=100 + j)
            pool.append((qp.Q.astype(npdt), qp.G.astype(npdt), qp.lb, qp.ub, qp.G))
    reqs = []
    iu = 0
    for r in range(R):
        if cls[r] == 0:
            qp = ub.instance(iu)
            iu += 1
            reqs.append(("uneven", dict(Q=qp.Q.astype(npdt), q=qp.q, G=qp.G.astype(npdt), g=qp.g, lb=qp.lb,
                                        ub=qp.ub)))
        elif cls[r] == 1:
            j = int(rng.integers(8))
            q, g = gen.mpc_linear_terms(systems[j], rng.uniform(-1.0, 1.0, 12))
            reqs.append(("mpc", dict(q=q, g=g, sys=j)))
        else:
            j = int(rng.integers(len(pool)))
            Q, G, lb, ubx, G64 = pool[j]
            q, g = gen.fresh_linear_terms(G64, rng)
            reqs.append(("large", dict(Q=Q, q=q, G=G, g=g, lb=lb, ub=ubx)))
    gen_s = time.time() - t0
    budget = 32 << 30
    srv = duq.Server(budget, **opts)
    sids = [srv.register_shared(sy.H.astype(npdt), sy.G.astype(npdt), sy.lb, sy.ub) for sy in systems]
    # warm-up: one request of each class, untimed
    for kind, d in reqs[:: max(1, R // 3)][:3]:
        t = srv.submit(q=d["q"], g=d["g"], shared_id=sids[d["sys"]]) if kind == "mpc" else srv.submit(**d)
        srv.wait(t, timeout=300)
    tickets = [None] * R
    sub_t = np.zeros(R)
    t_start = time.perf_counter()

    def submitter():
        for r, (kind, d) in enumerate(reqs):
            delay = arr[r] - (time.perf_counter() - t_start)
            if delay > 0:
                time.sleep(delay)
            sub_t[r] = time.perf_counter() - t_start
            if kind == "mpc":
                tickets[r] = srv.submit(q=d["q"], g=d["g"], shared_id=sids[d["sys"]])
            else:
                tickets[r] = srv.submit(**d)

    th = threading.Thread(target=submitter)
    th.start()
    results = [None] * R
    done_t = np.full(R, np.inf)
    pending = set(range(R))
    last_print = time.perf_counter()
    while pending:
        for r in list(pending):
            if tickets[r] is None:
                continue
            out = srv.poll(tickets[r])
            if out is not None:
                results[r] = out
                done_t[r] = time.perf_counter() - t_start
                pending.discard(r)
        now = time.perf_counter()
        if now - last_print > 10:
            print(f"[serve] t={now - t_start:.0f}s done {R - len(pending)}/{R}", file=sys.stderr, flush=True)
            last_print = now
        if now - t_start > duration + 240:
            break
        time.sleep(0.01)
    th.join()
    t_end = time.perf_counter()
    srv.close()
    # plain per-QP solver (duq_setup + duq_solve per request, same options) on a
    # sample of each class, weighted by the class counts of the stream
    plain_s = {}
    for k, m in (("uneven", 6), ("mpc", 12), ("large", 1)):
        idx = [i for i in range(R) if reqs[i][0] == k][:m]
        if not idx:
            continue
        sec = []
        for i in idx:
            d = reqs[i][1]
            o = {kk: v for kk, v in opts.items() if kk != "serve_slice"}
            if k == "mpc":
                sy = systems[d["sys"]]
                prob = (sy.H.astype(npdt), d["q"], sy.G.astype(npdt), d["g"], sy.lb, sy.ub)
                with duq.Solver(*prob, **o) as sv:   # the system's constants, as registered systems have
                    c = sv.constants()
                o.update(lam_min=c["lam_min"], lam_max=c["lam_max"], G_norm2=c["G_norm2"])
            else:
                prob = (d["Q"], d["q"], d["G"], d["g"], d["lb"], d["ub"])
            t = time.perf_counter()
            with duq.Solver(*prob, **o) as sv:
                sv.solve(check=False)
            sec.append(time.perf_counter() - t)
        plain_s[k] = float(np.mean(sec))
    done = [i for i in range(R) if results[i] is not None]
    lat = np.array([results[i][3]["time_ms"] for i in done])
    span = max(results[i][3]["time_ms"] * 1e-3 + sub_t[i] for i in done) if done else t_end - t_start
    ok = sum(results[i][0] == duq.DUQ_OK for i in done)
    by = {}
    for k in ("uneven", "mpc", "large"):
        ki = [i for i in done if reqs[i][0] == k]
        li = [results[i][3]["time_ms"] for i in ki]
        if li:
            by[k] = {"count": len(li), "ok": sum(results[i][0] == duq.DUQ_OK for i in ki),
                     "p50_ms": round(float(np.percentile(li, 50)), 3),
                     "p99_ms": round(float(np.percentile(li, 99)), 3),
                     "outer_mean": round(float(np.mean([results[i][3]["outer_iters"] for i in ki])), 1)}
    cert = max((results[i][3]["f"] - results[i][3]["lb_dual"]) / max(1.0, abs(results[i][3]["f"])) for i in done)
    line = {
        "metric": METRIC, "value": round(ok / span, 2), "unit": "solves/s", "n_gpus": 1, "steps": 1,
        "speedup_vs_plain": None,
        "warmup": 1, "ms_per_step": round(span * 1e3, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if a.precision == "f64" else "f32-storage/f64", "data": "synthetic",
        "config": {"workload": f"serving: Poisson arrivals {rate:g}/s for {duration:g} s (seed 4); "
                               f"{a.large_frac:.0%} dense n=4096 p=2048 (pool of 8, fresh q,g), rest half uneven "
                               f"n~U{{20..512}} and half MPC on 8 registered systems (seeds 40..47, fresh x0); "
                               f"matrices {a.precision}; {a.method.upper()}-{a.output} eps_out={a.eps_out:g} "
                               f"eps_in={eps_in:g}; {a.slice} outer iterations per round",
                   "requests": R, "hbm_budget_bytes": budget},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3),
                       "by_class": by},
        "solve": {"completed": len(done), "ok": ok, "failed": len(done) - ok, "max_cert_subopt_rel": cert,
                  "max_feas_abs": max(results[i][3]["feas"] for i in done)},
        "offered_per_s": round(R / duration, 1),
        # completions while requests still arrive: under overload, the rate the
        # GPU sustains; and how long the backlog took to drain afterwards
        "completed_in_window_per_s": round(float(np.sum(done_t <= duration)) / duration, 2),
        "drain_s_after_last_arrival": round(float(np.max(done_t[np.isfinite(done_t)])) - float(arr[-1]), 2)
        if done else None,
        "plain_solves_per_s": round(len(done) / sum(plain_s.get(reqs[i][0], 0.0) for i in done), 2),
        "plain_seconds_per_request": {k: round(v, 4) for k, v in plain_s.items()},
        "gen_seconds": round(gen_s, 1),
    }
    line["speedup_vs_plain"] = round(line["value"] / line["plain_solves_per_s"], 1)
    return line


# ----------------------------------------------------------------------------
# The paper's studies, reproduced qualitatively on synthetic QPs (the paper's
# own data and figures are not available): Sec. 3.1 / Fig. 1 (sensitivity to
# the inner accuracy) and Sec. 6.3 / Fig. 5 (outer iterations against n, last
# against averaged primal iterate).  Every solve runs on the GPU; the optimal
# value used for suboptimality comes from a tight GPU solve of the same QP.
# ----------------------------------------------------------------------------

def study_inner_accuracy(seeds=range(501, 509), n=60, p=30, eps_ins=(1e-1, 1e-2, 1e-3, 1e-4, 1e-6),
                         K=600, checkpoints=(50, 200, 600)):
    """Fig. 1: primal suboptimality |F(ubar^k) - F*|/|F*| and feasibility
    ||[G ubar^k + g]_+|| after k outer iterations of DGM and DFGM (last
    iterate) for several eps_in, on strongly convex random dense QPs; mean over
    the seeds."""
    from paper_1504_05708_amd import duq, gen
    qps = [gen.random_dense_qp(n, p, seed=s) for s in seeds]
    fstar = []
    for qp in qps:
        with duq.Solver(qp.Q, qp.q, qp.G, qp.g, qp.lb, qp.ub, method=duq.DFGM, eps_out=1e-9, eps_in=1e-13,
                        max_outer=200000, engine=duq.ENGINE_BLOCK) as s:
            fstar.append(s.solve()[2]["f"])
    table = []
    for method, name in ((duq.DGM, "DGM"), (duq.DFGM, "DFGM")):
        for ein in eps_ins:
            sub = np.zeros(len(checkpoints))
            feas = np.zeros(len(checkpoints))
            inner = 0
            for qp, fs in zip(qps, fstar):
                with duq.Solver(qp.Q, qp.q, qp.G, qp.g, qp.lb, qp.ub, method=method, eps_out=1e-13, eps_in=ein,
                                max_outer=K, trace_outer=K, engine=duq.ENGINE_BLOCK) as s:
                    _, _, r = s.solve(check=False)
                    S = s.trace(K)["scalars"]
                inner += r["inner_iters"]
                for j, k in enumerate(checkpoints):
                    sub[j] += abs(S[k - 1, 7] - fs) / max(1.0, abs(fs)) / len(qps)
                    feas[j] += S[k - 1, 8] / len(qps)
            table.append({"method": name, "eps_in": ein,
                          "subopt_rel": {str(k): float(v) for k, v in zip(checkpoints, sub)},
                          "feas": {str(k): float(v) for k, v in zip(checkpoints, feas)},
                          "inner_steps_per_qp": inner / len(qps)})
    return {"study": "inner_accuracy (Sec. 3.1, Fig. 1)",
            "workload": f"{len(qps)} random dense QPs n={n} p={p} (Q=A^T A/n+0.1I), seeds {min(seeds)}..{max(seeds)}; "
                        f"last primal iterate after k outer iterations; F* from a tight GPU solve",
            "rows": table}


def study_outer_vs_n(ns=(10, 50, 100, 200, 300, 400, 500), per_n=25, eps=1e-2, eps_in=1e-6, seed0=700):
    """Fig. 5: outer iterations to the outer test at eps, against n, for the
    last and the averaged primal iterate (DGM and DFGM), 25 random QPs per n
    solved as one batch on the GPU (p = n/2)."""
    from paper_1504_05708_amd import duq, gen
    rows = []
    for n in ns:
        qps = [gen.random_dense_qp(n, n // 2, seed=seed0 + 1000 * n + j) for j in range(per_n)]
        ub = gen.pack_uneven(qps)
        row = {"n": n}
        for method, mname in ((duq.DGM, "DGM"), (duq.DFGM, "DFGM")):
            for output, oname in ((duq.LAST, "LAST"), (duq.AVG, "AVG")):
                _, _, res = duq.solve_batch_uneven(ub, method=method, output=output, eps_out=eps, eps_in=eps_in,
                                                   max_outer=200000, check=False)
                outer = [r["outer_iters"] for r in res if r["status"] == duq.DUQ_OK]
                row[f"{mname}-{oname}"] = {"mean_outer": float(np.mean(outer)) if outer else None,
                                           "median_outer": float(np.median(outer)) if outer else None,
                                           "ok": len(outer)}
        rows.append(row)
    return {"study": "outer_vs_n (Sec. 6.3, Fig. 5)",
            "workload": f"{per_n} random dense QPs per n (Q=A^T A/n+0.1I, p=n/2, inequality rows), eps_out={eps:g}, "
                        f"eps_in={eps_in:g}; one uneven batch per n and method",
            "rows": rows}


def bench_studies(a):
    import torch
    from paper_1504_05708_amd import duq
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    duq.lib()
    for fn in (study_inner_accuracy, study_outer_vs_n):
        t = time.perf_counter()
        out = fn()
        out["seconds"] = round(time.perf_counter() - t, 1)
        print(json.dumps(out), flush=True)


def _release_device():
    # Free everything the run holds on the device before the interpreter's
    # own teardown, so that no library handle or cached block is released
    # after the HIP runtime (or a profiler attached to it) has shut down.
    import gc
    gc.collect()
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
    except Exception:
        pass


if __name__ == "__main__":
    main()
    _release_device()
