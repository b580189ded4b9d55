"""Benchmark: unaligned RKHS-subproblem solves per second on one MI355X.

Workload (default): the large unaligned case -- I = 1000 samples, J = 200
features, m_i ~ U{10..50} own times per sample (n ~ 30,700 design points,
q ~ 6.1e6 observations), Matern-3/2 kernel of length scale 0.1, rank r = 40,
lambda = 1e-4, rho = 1e-6, seed 0.  A step is one whole subproblem solve from
the observed values (per-solve setup, right-hand side, PCG / refinement, FP64
residual certificate) with every input already resident in HBM.

The headline form is the mixed-precision solver (BF16 MFMA inner solves in the
eigenbasis of K, FP64 refinement to relative residual 1e-7, i.e. K W within
1e-6); the plain FP64 PCG of the paper is timed beside it.

The "batched" field measures the batched form: 64 independent subproblems of
uneven size (n_b ~ U{500..8000}, r_b in {5, 10, 20, 40}, Gaussian kernels of
bandwidth ~U[0.05, 0.2), J_b = 20, lambda = 1e-4) solved by one persistent,
graph-captured launch in mixed precision, against the FP64 PCG solving the
same members one after another.  Both start from right-hand sides already in
HBM.  One JSON line goes to stdout.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0

# K and U_K are stored with row strides rounded up to 16 doubles: every row
# then starts on a 128-byte line, so a product's 16-element chunk of a row is
# one line (with the stride n = 30658, 245264 bytes, each chunk straddles two
# lines and the FP64 product fetched 1.24x its algorithmic bytes, not 1.01x).
KROW_ALIGN = 16
# Tiles of the batched solver written by `python -m paper_2603_25691_amd.tune batch`
# on MI355X (the defaults apply when the file is absent).
BATCH_TILES = os.path.join(ROOT, "paper_2603_25691_amd", "tiles_batch_mi355x.txt")
# HBM bytes per launch of the product kernels at the default workload (rows
# stored as above), from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs scaled
# by a calibration copy (profiles/products_n30658_r40_hbm_counters.md).  Keyed
# by kernel and shape; clear an entry whenever that kernel changes.
MEASURED_TRAFFIC = {("gemm_bf16_kernel<3, 4, 2, true>", 30658, 40): 1.9480e9,
                    ("gemm_f64_kernel<10, 4, 2, true, 1>", 30658, 40): 7.6937e9}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--I", type=int, default=1000, help="samples (1000 = full size)")
    ap.add_argument("--J", type=int, default=200)
    ap.add_argument("--precision", default="mixed_bf16",
                    choices=["mixed_bf16", "mixed_fp32", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run a plain device copy of this size (counter calibration)")
    ap.add_argument("--batch-count", type=int, default=64,
                    help="members of the batched workload (0: skip it)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--batch-only", action="store_true",
                    help="measure only the batched workload (prints its JSON object)")
    return ap.parse_args()


def bench_batch(a, torch, C):
    """The batched workload: one persistent graph launch for all members
    (mixed BF16) against the FP64 PCG over the members in turn."""
    from paper_2603_25691_amd.torch_api import BatchSolver, UISolver, upload
    from synth import batch_members

    t0 = time.time()
    probs, dps = [], []
    for bm in batch_members(seed=0, count=a.batch_count):
        p = bm.problem
        dps.append(upload(p, ldk_align=KROW_ALIGN))
        # keep only what the accuracy check needs on the host
        probs.append(p)
    torch.cuda.synchronize()
    ns = np.array([p.n for p in probs])
    rs = np.array([p.r for p in probs])
    log(f"batch: {len(probs)} members, n {ns.min()}..{ns.max()} (sum n^2 = {np.sum(ns**2.0):.3e}),"
        f" r {sorted(set(rs.tolist()))}; generated, uploaded, eig(K) in {time.time() - t0:.1f} s")
    tol = 1e-7
    t0 = time.time()
    table = BATCH_TILES if os.path.exists(BATCH_TILES) else None
    bs = BatchSolver(dps, [p.lam for p in probs], [p.rho for p in probs], tol, tile_table=table)
    rhs = bs.rhs()
    Ws = [torch.empty_like(b) for b in rhs]
    bs.bind(rhs, Ws)
    status, infos = bs.solve()
    torch.cuda.synchronize()
    log(f"batch: created + first solve in {time.time() - t0:.1f} s, status {status}")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(a.batch_steps):
        bs.solve(wait=False)
    ev1.record()
    torch.cuda.synchronize()
    ms_batch = ev0.elapsed_time(ev1) / a.batch_steps
    status, infos = bs.info()
    rounds, grid = bs.rounds()
    phase = bs.phase_ms()
    log("batch phases (ms, last launch): " + ", ".join(f"{k} {v:.2f}" for k, v in phase.items()))
    log(f"batch mixed: {ms_batch:.2f} ms per batch ({len(probs) * 1e3 / ms_batch:.1f} "
        f"subproblem solves/s), {rounds} rounds, grid {grid}, status {C.status_string(status)}")

    # FP64 PCG (paper form), members one after another
    tol64 = 1e-8
    solvers = [UISolver(dp, p.lam, p.rho, tol64, precision="fp64") for p, dp in zip(probs, dps)]
    for s_ in solvers:
        s_.setup()
    W64 = [torch.empty_like(b) for b in rhs]
    for s_, b, W in zip(solvers, rhs, W64):  # warm-up
        s_.solve(b, W)
    torch.cuda.synchronize()
    ev0.record()
    it64 = []
    for s_, b, W in zip(solvers, rhs, W64):
        _, info = s_.solve(b, W)
        it64.append(info.iters)
    ev1.record()
    torch.cuda.synchronize()
    ms64 = ev0.elapsed_time(ev1)
    log(f"batch fp64 (members in turn): {ms64:.1f} ms ({len(probs) * 1e3 / ms64:.1f} solves/s)")

    # accuracy: every member's mixed result against its FP64 result
    ekw = []
    for p, W, Wd in zip(probs, Ws, W64):
        Wh, Wdh = W.cpu().numpy(), Wd.cpu().numpy()
        KW = p.K @ Wdh
        ekw.append(float(np.linalg.norm(p.K @ Wh - KW) / np.linalg.norm(KW)))
    # algorithmic bytes of the n x n passes of one batched solve: per inner
    # iteration 2 BF16 passes over U_K; per refinement step but the last the
    # FP64 residual in the eigenbasis (2 passes over U_K; the last step goes
    # straight to the certificate when convergence is predicted, so this is a
    # lower bound); once per solve the rotation of b into the eigenbasis and of
    # the solution out of it (2 passes over U_K) and the FP64 certificate (2
    # passes over K).
    byts = 0.0
    for p, inf in zip(probs, infos):
        n2 = float(p.n) ** 2
        byts += inf.iters * 2 * 2 * n2 + (2 * max(inf.refine_steps - 1, 0) + 4) * 8 * n2
    gbps = byts / (ms_batch * 1e6)
    for s_ in solvers:
        s_.close()
    out = {
        "workload": (f"{len(probs)} subproblems, n_b~U{{500..8000}}, r_b in {{5,10,20,40}}, "
                     "RBF sigma_b~U[0.05,0.2), J_b=20, I_b=ceil(n_b/30), lambda=1e-4, "
                     "rho=1e-6, seed=0"),
        "members": len(probs), "sum_n2": float(np.sum(ns ** 2.0)),
        "tile_table": os.path.basename(table) if table else "defaults",
        "ms_per_batch": ms_batch, "solves_per_s": len(probs) * 1e3 / ms_batch,
        "status": C.status_string(status), "rounds": rounds, "grid": grid,
        "phase_ms": phase,
        "inner_iters_max": max(i.iters for i in infos),
        "refine_steps_max": max(i.refine_steps for i in infos),
        "relres_max": max(i.relres_true for i in infos),
        "fp64_ms_per_batch": ms64, "fp64_solves_per_s": len(probs) * 1e3 / ms64,
        "fp64_iters_max": max(it64),
        "mixed_vs_fp64_speedup": ms64 / ms_batch,
        "e_KW_vs_fp64_max": max(ekw),
        "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": gbps / HBM_PEAK_GBPS, "traffic": None,
                     "kernel": "batch_kernel (whole batched solve, n x n passes only)",
                     "algorithmic_bytes": byts},
    }
    bs.close()
    return out


def cpu_baseline(p, iters: int, budget_s: float = 20.0):
    """Time the oracle (numpy FP64) on the host on a bounded sample of the
    same workload: full-size two-step products and preconditioner applies."""
    import oracle as O

    try:
        from threadpoolctl import threadpool_info

        cores = max([i.get("num_threads", 0) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    V = O.gram_V(p.A, p.B)
    dV, UV = np.linalg.eigh(V)
    X = np.random.default_rng(1).standard_normal((p.n, p.r))
    # The preconditioner's cost does not depend on the eigenvector values; K
    # stands in for U_K here (a full host eigendecomposition at this n would
    # take tens of minutes and is one-time setup on both sides anyway).
    dK = np.ones(p.n)
    t_mv, t_pc, reps = 0.0, 0.0, 0
    t_start = time.perf_counter()
    while reps < 3 and time.perf_counter() - t_start < budget_s:
        t0 = time.perf_counter()
        O.matvec_twostep(p.K, Zhat, p.obs_t, p.lam, p.rho, X)
        t1 = time.perf_counter()
        O.precond_apply(p.K, dK, UV, dV, p.gamma, p.lam, p.rho, X)
        t2 = time.perf_counter()
        t_mv += t1 - t0
        t_pc += t2 - t1
        reps += 1
    t_mv /= reps
    t_pc /= reps
    per_solve = iters * (t_mv + t_pc)
    return {
        "value": 1.0 / per_solve,
        "unit": "solves/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{reps} full-size oracle two-step products ({t_mv:.2f} s each) and "
                   f"preconditioner applies ({t_pc:.2f} s each) on the host; per-solve time "
                   f"= {iters} PCG iterations (the FP64 run's count to the same accuracy) x "
                   f"(product + preconditioner) = {per_solve:.1f} s"),
    }


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    from paper_2603_25691_amd import cphifi as C
    from paper_2603_25691_amd.torch_api import UISolver, upload
    from synth import config_c3

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.batch_only:
        print(json.dumps(bench_batch(a, torch, C)), flush=True)
        return
    t0 = time.time()
    p = config_c3(I=a.I, J=a.J)
    log(f"generated n={p.n} q={p.q} r={p.r} in {time.time() - t0:.1f} s")
    t0 = time.time()
    dp = upload(p, ldk_align=KROW_ALIGN)
    torch.cuda.synchronize()
    log(f"uploaded + eig(K) on device in {time.time() - t0:.1f} s")
    n, r, q = p.n, p.r, p.q
    TK = C.FLAG_TIME_KERNELS

    if a.calib_copy_mb > 0:
        src = torch.empty(a.calib_copy_mb * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {a.calib_copy_mb} MiB done")

    # ---------------------------------------------------------------- matvec
    sf = UISolver(dp, p.lam, p.rho, p.tol, precision="fp64", check_every=1)
    X = torch.randn(n, r, dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    for _ in range(2):
        sf.apply(X, out=Y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    reps = 10
    e0.record()
    for _ in range(reps):
        sf.apply(X, out=Y)
    e1.record()
    torch.cuda.synchronize()
    mv_ms = e0.elapsed_time(e1) / reps
    mv_bytes = 2 * 8 * n * n + 16 * n * r + 8 * q
    log(f"matvec {mv_ms:.3f} ms = {mv_bytes / mv_ms / 1e6:.0f} GB/s")

    # ------------------------------------------------------------ FP64 PCG
    sf64 = UISolver(dp, p.lam, p.rho, p.tol, precision="fp64", flags=TK, check_every=1)
    W64, info = sf64.solve_subproblem()
    torch.cuda.synchronize()
    t = []
    g_ms, g_n = 0.0, 0
    for _ in range(a.fp64_steps):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        W64, info = sf64.solve_subproblem(W=W64)
        torch.cuda.synchronize()
        t.append(time.perf_counter() - s0)
        g_ms += info.gemm_ms
        g_n += info.gemm_launches
    fp64 = {"ms_per_solve": 1e3 * float(np.median(t)), "iters": info.iters,
            "relres_true": info.relres_true, "status": C.status_string(info.status),
            "solves_per_s": 1.0 / float(np.median(t)),
            "gemm_avg_ms": g_ms / max(g_n, 1), "gemm_launches_per_solve": g_n // max(1, len(t))}
    log(f"fp64 PCG: {fp64}")
    # The same FP64 PCG in the eigenbasis of K (x = U_K xbar, the rotation of
    # Section 3.3): two n x n passes per iteration instead of four; reported
    # beside the paper form as a second FP64 reference point.
    sfe = UISolver(dp, p.lam, p.rho, p.tol, precision="fp64", flags=C.FLAG_EIGENBASIS,
                   check_every=1)
    W64e, info_e = sfe.solve_subproblem()
    torch.cuda.synchronize()
    te = []
    for _ in range(a.fp64_steps):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        W64e, info_e = sfe.solve_subproblem(W=W64e)
        torch.cuda.synchronize()
        te.append(time.perf_counter() - s0)
    fp64_eig = {"ms_per_solve": 1e3 * float(np.median(te)), "iters": info_e.iters,
                "relres_true": info_e.relres_true, "status": C.status_string(info_e.status)}
    log(f"fp64 PCG in the eigenbasis: {fp64_eig}")
    del sfe, W64e
    fp64_bytes = 8 * n * n + 16 * n * r
    roof64 = {"bound": "hbm", "achieved": fp64_bytes / (fp64["gemm_avg_ms"] * 1e6),
              "peak": HBM_PEAK_GBPS, "unit": "GB/s"}
    roof64["frac"] = roof64["achieved"] / roof64["peak"]
    roof64["kernel"] = "gemm_f64_kernel<10, 4, 2, true, 1> (K X and U_K X products)"
    roof64["traffic"] = MEASURED_TRAFFIC.get((roof64["kernel"].split(" (")[0], n, r))

    # --------------------------------------------------- headline (mixed) form
    prec = a.precision
    tol = 1e-7 if prec != "fp64" else p.tol
    sm = UISolver(dp, p.lam, p.rho, tol, precision=prec, flags=TK, check_every=1)
    W, info = sm.solve_subproblem()
    for _ in range(max(0, a.warmup - 1)):
        W, info = sm.solve_subproblem(W=W)
    torch.cuda.synchronize()
    g_ms, g_n = 0.0, 0
    infos = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record()
    for _ in range(a.steps):
        W, info = sm.solve_subproblem(W=W)
        g_ms += info.gemm_ms
        g_n += info.gemm_launches
        infos.append(info.as_dict())
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_per_step = ev0.elapsed_time(ev1) / a.steps
    value = 1e3 / ms_per_step
    log(f"{prec}: {ms_per_step:.2f} ms/solve, {value:.2f} solves/s, wall {wall:.2f} s, "
        f"last {infos[-1]}")

    # the headline solve's inner operator: one eigenbasis apply at the plan's
    # precision (D_K U^T G(U D_K x) + lambda D_K x + rho x: two low-precision
    # passes over U_K and the gather), timed like the FP64 matvec
    mvl = None
    if prec != "fp64":
        xb = torch.randn(n, r, dtype=torch.float64, device="cuda")
        yb = torch.empty_like(xb)
        for _ in range(2):
            sm.apply_lowp(xb, out=yb)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            sm.apply_lowp(xb, out=yb)
        e1.record()
        torch.cuda.synchronize()
        mvl_ms = e0.elapsed_time(e1) / reps
        esz = 2 if prec == "mixed_bf16" else 4
        mvl_bytes = 2 * (esz * n * n + 16 * n * r) + 8 * q
        mvl = {"ms": mvl_ms, "GB_per_s": mvl_bytes / mvl_ms / 1e6,
               "frac_of_peak": mvl_bytes / mvl_ms / 1e6 / HBM_PEAK_GBPS, "bytes": mvl_bytes,
               "operator": "eigenbasis inner operator of the mixed solve (cphifi_ui_apply_lowp)"}
        log(f"inner-operator matvec {mvl_ms:.3f} ms = {mvl_bytes / mvl_ms / 1e6:.0f} GB/s")

    # ------------------------------------------------------------- accuracy
    Wh = W.cpu().numpy()
    W64h = W64.cpu().numpy()
    acc = {"relres_true": infos[-1]["relres_true"], "status": infos[-1]["status"]}
    KW64 = p.K @ W64h
    acc["e_KW_vs_fp64_gpu"] = float(np.linalg.norm(p.K @ Wh - KW64) / np.linalg.norm(KW64))
    if not a.no_oracle_check:
        import oracle as O

        Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
        t0 = time.time()
        acc["oracle_relres_certificate"] = O.relres(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho, Wh)
        log(f"oracle residual certificate {acc['oracle_relres_certificate']:.3e} "
            f"({time.time() - t0:.1f} s)")

    if prec == "mixed_bf16":
        lp_bytes = 2 * n * n + 16 * n * r
        kname = "gemm_bf16_kernel<3, 4, 2, true> (U_K-rounded products of the inner solve)"
    elif prec == "mixed_fp32":
        lp_bytes = 4 * n * n + 16 * n * r
        kname = "gemm_k4_kernel<float, NB=3, NN> (U_K-rounded products of the inner solve)"
    else:
        lp_bytes = fp64_bytes
        kname = roof64["kernel"]
    avg_ms = g_ms / max(g_n, 1)
    roof = {"bound": "hbm", "achieved": lp_bytes / (avg_ms * 1e6), "peak": HBM_PEAK_GBPS,
            "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = MEASURED_TRAFFIC.get((kname.split(" (")[0], n, r))
    roof["kernel"] = kname
    roof["avg_launch_ms"] = avg_ms
    roof["launches_per_solve"] = g_n / a.steps

    out = {
        "metric": "RKHS-subproblem solves/sec to 1e-6 rel err; matvec HBM GB/s; mixed vs FP64",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed_bf16": "bf16+f64", "mixed_fp32": "f32+f64", "fp64": "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": (f"unaligned RKHS subproblem: I={p.I} J={p.J} m_i~U{{10..50}} "
                                f"n={n} q={q} r={r} Matern-3/2(0.1) lambda={p.lam} "
                                f"rho={p.rho} seed=0"),
                   "form": prec, "n": n, "q": q, "r": r},
        "roofline": roof,
        "fp64": dict(fp64, roofline=roof64),
        "matvec": {"ms": mv_ms, "GB_per_s": mv_bytes / mv_ms / 1e6,
                   "frac_of_peak": mv_bytes / mv_ms / 1e6 / HBM_PEAK_GBPS,
                   "bytes": mv_bytes, "operator": "FP64 paper form (cphifi_ui_apply)"},
        "matvec_mixed": mvl,
        "mixed_vs_fp64_speedup": fp64["ms_per_solve"] / ms_per_step,
        "fp64_eigenbasis": dict(fp64_eig,
                                mixed_speedup=fp64_eig["ms_per_solve"] / ms_per_step),
        "accuracy": acc,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, fp64["iters"])
        log(f"cpu baseline {out['cpu_baseline']}")
    if a.batch_count > 0:
        del sf, sf64, sm, dp
        torch.cuda.empty_cache()
        out["batched"] = bench_batch(a, torch, C)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
