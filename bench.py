"""Benchmark: unaligned RKHS-subproblem solves per second on one MI355X.

Workload (default): the large unaligned case -- I = 1000 samples, J = 200
features, m_i ~ U{10..50} own times per sample (n ~ 30,700 design points,
q ~ 6.1e6 observations), Matern-3/2 kernel of length scale 0.1, rank r = 40,
lambda = 1e-4, rho = 1e-6, seed 0.  A step is one whole subproblem solve from
the observed values (per-solve setup, right-hand side, PCG / refinement, FP64
residual certificate) with every input already resident in HBM; each step is
timed with HIP events and `ms_per_step` is the median.

The headline form is the mixed-precision solver (BF16 MFMA inner solves in the
eigenbasis of K, FP64 refinement to a certified relative residual of 1e-7,
i.e. K W within 1e-6); the FP64 PCG of the paper is timed beside it at the same
residual target (and at the workload's own 1e-8).

Further fields: `matvec` (the FP64 two-step product of Section 4.4.1),
`small` (I = 20, J = 10, r = 5: latency per solve, with the oracle's dense
and least-squares solves timed on the host), `aligned` (n = 200 grid, I = 500,
J = 100, q = 1e7, r = 10/20/40: FP64 and both mixed precisions, the aligned
solvers of Section 3, the oracle's Kronecker Cholesky and decoupled solves
timed on the host), `paper_shapes` (the shapes of the paper's unaligned
experiments, its PCG setting, against the oracle's PCG) and `batched`
(64 subproblems of uneven size in one persistent, graph-captured launch,
against the FP64 PCG over the same members).  One JSON line goes to stdout.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
FP64_PEAK_TFLOPS = 78.6

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
MEASURED_TRAFFIC = {("gemm_bf16_kernel<3, 4, 2, true>", 30658, 40): 1.9539e9,
                    ("gemm_f64_kernel<10, 4, 2, true, 1>", 30658, 40): 7.6591e9}
# HBM bytes per launch of the batched kernel on the 64-member workload, from the
# same two counters (profiles/c5_batch64_hbm_counters.md); clear on a change.
BATCH_TRAFFIC = 2.314e11
F64_KERNEL = "gemm_f64_kernel<10, 4, 2, true, 1>"
BF16_KERNEL = "gemm_bf16_kernel<3, 4, 2, true>"
# relative residual the mixed solves are refined to (e_KW within 1e-6), and
# the FP64 runs compared with them at the same target
MIXED_TOL = 1e-7
BATCH_TOL = 5e-8


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
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run a plain device copy of this size (counter calibration)")
    ap.add_argument("--batch-count", type=int, default=64,
                    help="members of the batched workload (0: skip it)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--batch-only", action="store_true",
                    help="measure only the batched workload (prints its JSON object)")
    ap.add_argument("--small-only", action="store_true",
                    help="run only the small workload and print its JSON (profiling)")
    ap.add_argument("--no-small", action="store_true", help="skip the small workload")
    ap.add_argument("--no-aligned", action="store_true", help="skip the aligned workload")
    ap.add_argument("--no-paper-shapes", action="store_true",
                    help="skip the paper-shaped stand-ins")
    ap.add_argument("--eig-dir", default="",
                    help="read the batch members' eigenpairs from this directory "
                         "(written by --save-eig) instead of computing them")
    ap.add_argument("--save-eig", default="", help="write the batch members' eigenpairs here")
    return ap.parse_args()


def cpu_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info

        cores = max([i.get("num_threads", 0) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    return model, cores


def host_median(fn, reps: int = 3, budget_s: float = 20.0):
    """Median wall time of fn() on the host (at most `reps` runs, fewer when
    the budget is spent); returns (seconds, last result)."""
    t, out = [], None
    t0 = time.perf_counter()
    while len(t) < reps and (not t or time.perf_counter() - t0 < budget_s):
        s0 = time.perf_counter()
        out = fn()
        t.append(time.perf_counter() - s0)
    return float(np.median(t)), out


class StepTimer:
    """HIP events around each step on the current stream; median of the steps."""

    def __init__(self, torch):
        self.torch = torch
        self.ev = []

    def run(self, fn, steps: int):
        torch = self.torch
        pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(steps)]
        out = None
        for e0, e1 in pairs:
            e0.record()
            out = fn()
            e1.record()
        torch.cuda.synchronize()
        ms = [e0.elapsed_time(e1) for e0, e1 in pairs]
        return float(np.median(ms)), float(np.mean(ms)), out


def achievable_read(torch, C, gib: int = 4, reps: int = 10):
    """The achievable HBM read rate: the library's streaming-read kernel over a
    `gib` GiB buffer (16-byte loads), best median over a few grid sizes."""
    nbytes = gib * 2 ** 30
    buf = torch.zeros(nbytes // 8, dtype=torch.float64, device="cuda")
    part = torch.empty(65536, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    timer = StepTimer(torch)
    best = None
    for blocks in (1024, 2048, 4096, 8192, 16384):
        def run():
            C.cphifi_stream_read(buf.data_ptr(), nbytes, blocks, part.data_ptr(), st)
        run()
        torch.cuda.synchronize()
        ms, _, _ = timer.run(run, reps)
        gbps = nbytes / ms / 1e6
        if best is None or gbps > best["GB_per_s"]:
            best = {"GB_per_s": gbps, "ms": ms, "blocks": blocks, "bytes": nbytes,
                    "frac_of_peak": gbps / HBM_PEAK_GBPS}
    del buf, part
    torch.cuda.empty_cache()
    best["kernel"] = "stream_read_kernel (cphifi_stream_read)"
    return best


def roofline_hbm(kernel, bytes_per_launch, avg_ms, launches, n, r):
    ach = bytes_per_launch / (avg_ms * 1e6)
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBPS,
            "traffic": MEASURED_TRAFFIC.get((kernel, n, r)), "kernel": kernel,
            "algorithmic_bytes": bytes_per_launch, "avg_launch_ms": avg_ms,
            "launches_per_solve": launches, "ms_per_solve": avg_ms * launches}


# --------------------------------------------------------------- small (C1)
def bench_small(torch, C, steps: int):
    """I = 20, J = 10, m_i ~ U{5..15}, Gaussian 0.1, r = 5, lambda = 1e-3: a
    latency-bound solve (K is 0.3 MB).  GPU time per solve (events, median)
    for the FP64 PCG to relres 1e-10 and the mixed form to 1e-7, against the
    oracle's dense Cholesky and least-squares solves on the host."""
    import oracle as O
    from paper_2603_25691_amd.torch_api import UISolver, upload
    from synth import config_c1

    p = config_c1()
    dp = upload(p)
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    t_dense, Wo = host_median(lambda: O.solve_dense(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho))
    t_brute, _ = host_median(lambda: O.solve_lstsq(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho))
    out = {"workload": f"unaligned RKHS subproblem: I=20 J=10 m_i~U{{5..15}} n={p.n} "
                       f"q={p.q} r=5 RBF(0.1) lambda=1e-3 rho=1e-6 seed=0",
           "n": p.n, "q": p.q, "r": p.r,
           "oracle_dense_ms": 1e3 * t_dense, "oracle_lstsq_ms": 1e3 * t_brute}
    timer = StepTimer(torch)
    # fp64: the default at this size, one persistent launch of co-resident
    # workgroups (CPHIFI_FLAG_PERSISTENT); fp64_graph: replays of a captured
    # graph of PCG iterations (CPHIFI_FLAG_NO_PERSISTENT); fp64_launches: the
    # launch-by-launch loop (and CPHIFI_FLAG_NO_GRAPH)
    legs = (("fp64", "fp64", 1e-10, 0),
            ("fp64_graph", "fp64", 1e-10, C.FLAG_NO_PERSISTENT),
            ("fp64_launches", "fp64", 1e-10, C.FLAG_NO_PERSISTENT | C.FLAG_NO_GRAPH),
            ("mixed_bf16", "mixed_bf16", MIXED_TOL, 0))
    for label, prec, tol, flags in legs:
        s = UISolver(dp, p.lam, p.rho, tol, precision=prec, flags=flags)
        W, info = s.solve_subproblem()
        med, mean, (W, info) = timer.run(lambda: s.solve_subproblem(W=W), steps)
        out[label] = {"us_per_solve": 1e3 * med, "us_mean": 1e3 * mean,
                     "solves_per_s": 1e3 / med, "iters": info.iters,
                     "refine_steps": info.refine_steps, "relres_true": info.relres_true,
                     "status": C.status_string(info.status),
                     "e_KW_vs_oracle_dense": O.e_kw(p.K, W.cpu().numpy(), Wo),
                     "tol": tol}
        s.close()
    out["gpu_vs_oracle_dense"] = out["oracle_dense_ms"] / (out["fp64"]["us_per_solve"] / 1e3)
    log(f"small: fp64 {out['fp64']['us_per_solve']:.0f} us (persistent launch; graph "
        f"{out['fp64_graph']['us_per_solve']:.0f} us, launch loop "
        f"{out['fp64_launches']['us_per_solve']:.0f} us), mixed "
        f"{out['mixed_bf16']['us_per_solve']:.0f} us per solve; oracle dense "
        f"{out['oracle_dense_ms']:.1f} ms, lstsq {out['oracle_lstsq_ms']:.1f} ms")
    return out


# ---------------------------------------------------------- aligned (C2, C4)
def bench_aligned(torch, C, steps: int):
    """Aligned case: n = 200 uniform grid, I = 500, J = 100 (q = 1e7), Gaussian
    0.05, lambda = 1e-4, r = 10 / 20 / 40.  With every entry observed the
    preconditioner is exact (gamma = 1), PCG takes one iteration, and the time
    goes to the gather-scatter over 1e7 observations.  FP64 and both mixed
    precisions (K products in BF16 / FP32), e_KW against the oracle's decoupled
    rho-solve; the oracle's Kronecker Cholesky and decoupled solve on the host."""
    import oracle as O
    from paper_2603_25691_amd.torch_api import AlignedSolver, UISolver, upload
    from synth import config_c2

    res = {"workload": "aligned RKHS subproblem: n=200 grid, I=500 J=100 q=1e7 RBF(0.05) "
                       "lambda=1e-4 rho=1e-6 seed=0", "ranks": {}}
    timer = StepTimer(torch)
    for r in (10, 20, 40):
        p = config_c2(r=r)
        dp = upload(p)
        Bm = O.mttkrp_full(p.y.reshape(p.n, p.I, p.J), p.A, p.B)
        KB = p.K @ Bm
        V = O.gram_V(p.A, p.B)

        def dec():
            dK, UK = O.kernel_eig(p.K)
            dV, UV = np.linalg.eigh(V)
            return O.solve_aligned_rho_decoupled(UK, dK, UV, dV, KB, p.lam, p.rho)

        t_dec, Wdec = host_median(dec)
        t_kron, Wk = host_median(lambda: O.solve_aligned_rho_kron(p.K, V, KB, p.lam, p.rho),
                                 reps=1)
        t_mttkrp, _ = host_median(lambda: O.mttkrp_full(p.y.reshape(p.n, p.I, p.J), p.A, p.B))
        row = {"oracle_mttkrp_ms": 1e3 * t_mttkrp, "oracle_decoupled_ms": 1e3 * t_dec,
               "oracle_kron_cholesky_ms": 1e3 * t_kron,
               "e_KW_kron_vs_decoupled": O.e_kw(p.K, Wk, Wdec)}
        # fp64_structured: the same solve with the K products on c = K(0,:)
        # (Toeplitz K of the uniform grid) and the fiber-collapsed gather
        # (every (time, sample) pair observed at all J features)
        structured = C.FLAG_TOEPLITZ_K | C.FLAG_FIBER_COLLAPSE
        for label, prec, tol, flags in (("fp64", "fp64", 1e-10, 0),
                                        ("fp64_structured", "fp64", 1e-10, structured),
                                        ("mixed_bf16", "mixed_bf16", MIXED_TOL, 0),
                                        ("mixed_fp32", "mixed_fp32", MIXED_TOL, 0)):
            s = UISolver(dp, p.lam, p.rho, tol, precision=prec, flags=flags)
            W, info = s.solve_subproblem()
            med, mean, (W, info) = timer.run(lambda: s.solve_subproblem(W=W), steps)
            row[label] = {"ms_per_solve": med, "iters": info.iters,
                         "refine_steps": info.refine_steps, "relres_true": info.relres_true,
                         "status": C.status_string(info.status),
                         "e_KW_vs_oracle_decoupled": O.e_kw(p.K, W.cpu().numpy(), Wdec)}
            s.close()
        # Section 3's own solvers on the GPU (rho = 0 system, right-hand side B):
        # the MTTKRP from the observed values, then the decoupled direct solve or
        # PCG on the transformed system; e_KW against the oracle's decoupled solve
        dK0, UK0 = O.kernel_eig(p.K)
        dV0, UV0 = np.linalg.eigh(V)
        W0 = O.solve_decoupled(UK0, dK0, UV0, dV0, Bm, p.lam)
        s = UISolver(dp, p.lam, p.rho, 1e-10)
        Bd = s.mttkrp()
        for meth, tol in (("decoupled", 0.0), ("pcg", 1e-10)):
            al = AlignedSolver(dp, p.lam, method=meth, tol=tol)
            Wa, ia = al.solve(s.mttkrp(out=Bd))

            def step_al():
                s.mttkrp(out=Bd)
                return al.solve(Bd, W=Wa)

            med, _, (Wa, ia) = timer.run(step_al, steps)
            row[f"aligned_{meth}"] = {"ms_per_solve": med, "iters": ia.iters,
                                      "relres_true": ia.relres_true,
                                      "status": C.status_string(ia.status),
                                      "e_KW_vs_oracle_decoupled_rho0":
                                          O.e_kw(p.K, Wa.cpu().numpy(), W0)}
            al.close()
        s.close()
        row["gpu_fp64_vs_oracle_mttkrp_plus_decoupled"] = (
            (t_mttkrp + t_dec) * 1e3 / row["fp64"]["ms_per_solve"])
        res["ranks"][str(r)] = row
        log(f"aligned r={r}: fp64 {row['fp64']['ms_per_solve']:.2f} ms "
            f"(e_KW {row['fp64']['e_KW_vs_oracle_decoupled']:.1e}; structured "
            f"{row['fp64_structured']['ms_per_solve']:.3f} ms), bf16 "
            f"{row['mixed_bf16']['ms_per_solve']:.2f} ms, fp32 "
            f"{row['mixed_fp32']['ms_per_solve']:.2f} ms; decoupled "
            f"{row['aligned_decoupled']['ms_per_solve']:.2f} ms, aligned PCG "
            f"{row['aligned_pcg']['ms_per_solve']:.2f} ms ({row['aligned_pcg']['iters']} its); "
            f"oracle mttkrp {1e3 * t_mttkrp:.0f} ms "
            f"decoupled {1e3 * t_dec:.0f} ms kron {1e3 * t_kron:.0f} ms")
        del dp
        torch.cuda.empty_cache()
    return res


# ------------------------------------------------------ paper shapes (C6)
def bench_paper_shapes(torch, C, steps: int):
    """Shape-only stand-ins of the paper's unaligned experiments (Section 5.2):
    vortex 199 x 449 x 151 and Miranda 256 x 256 x 269 tensors, all modes RKHS
    on integer grids (Gaussian bandwidths 4/4/3 and 1/1/2), q = 50,000 entries
    uniformly without replacement, lambda = 0.1, rho = 1e-6; the last mode's
    subproblem.  The paper's PCG setting (tol 1e-6, at most 75 iterations) in
    FP64 on the GPU against the oracle's PCG (the same algorithm on the host),
    per rank r."""
    import oracle as O
    from paper_2603_25691_amd.torch_api import UISolver, upload
    from synth import make_paper_standin

    model, cores = cpu_info()
    out = {"workload": "paper-shaped stand-ins (vortex 199x449x151, Miranda 256x256x269): "
                       "q=50000 uniform entries, Gaussian RKHS modes, lambda=0.1 rho=1e-6, "
                       "PCG tol 1e-6 maxit 75 (the paper's setting)",
           "host": f"{cores} threads ({model})", "cases": {}}
    timer = StepTimer(torch)
    for name, dims, sig in (("vortex", (199, 449, 151), (4.0, 4.0, 3.0)),
                            ("miranda", (256, 256, 269), (1.0, 1.0, 2.0))):
        for r in (5, 25, 50):
            p = make_paper_standin(shape=dims, sigmas=sig, r=r)
            dp = upload(p)
            Zhat, V = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j), O.gram_V(p.A, p.B)
            eig = O.kernel_eig(p.K)
            t_pcg, ref = host_median(lambda: O.solve_pcg(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho,
                                                         p.gamma, V, 1e-6, 75, eigK=eig))
            row = {"n": p.n, "r": r, "oracle_pcg_ms": 1e3 * t_pcg, "oracle_iters": ref.iters}
            for prec, tol in (("fp64", 1e-6), ("mixed_bf16", 1e-6)):
                s = UISolver(dp, p.lam, p.rho, tol, precision=prec, maxit=75)
                W, info = s.solve_subproblem()
                med, _, (W, info) = timer.run(lambda: s.solve_subproblem(W=W), steps)
                row[prec] = {"ms_per_solve": med, "iters": info.iters,
                             "relres_true": info.relres_true,
                             "status": C.status_string(info.status),
                             "e_KW_vs_oracle_pcg": O.e_kw(p.K, W.cpu().numpy(), ref.X)}
                s.close()
            row["gpu_fp64_vs_oracle_pcg"] = row["oracle_pcg_ms"] / row["fp64"]["ms_per_solve"]
            out["cases"][f"{name}-r{r}"] = row
            log(f"paper shape {name} r={r}: fp64 {row['fp64']['ms_per_solve']:.2f} ms "
                f"({row['fp64']['iters']} its), mixed {row['mixed_bf16']['ms_per_solve']:.2f} ms; "
                f"oracle PCG {row['oracle_pcg_ms']:.0f} ms ({ref.iters} its)")
            del dp
        out["als"] = out.get("als", {})
        out["als"][name] = bench_als(torch, C, dims, sig)
    # samples x features x time: two finite modes (CP-ALS rows) and one RKHS mode
    out["als"]["finite-finite-rkhs"] = bench_als(torch, C, (200, 50, 300), (1.0, 1.0, 3.0),
                                                 finite=(True, True, False), q=100000)
    return out


def bench_als(torch, C, dims, sig, r: int = 10, outer: int = 3, finite=(False, False, False),
              q: int = 50000):
    """The alternating optimisation on one stand-in (all three modes, the
    paper's subproblem setting, warm starts): GPU time per outer iteration and
    the oracle's (O-pcg blocks; row solves for finite modes) for one outer
    iteration on the host; error histories side by side."""
    import time
    import oracle as O
    from paper_2603_25691_amd.torch_api import AlsSolver, kernel_eig
    from synth import make_als_problem

    p = make_als_problem(shape=dims, sigmas=sig, r=r, seed=1, q=q, finite=finite)
    Ks = [None if K is None else torch.from_numpy(K).cuda() for K in p.Ks]
    eig = [(None, None) if K is None else kernel_eig(K) for K in Ks]
    coords = torch.from_numpy(p.coords).cuda()
    y = torch.from_numpy(p.y).cuda()
    W0 = [torch.from_numpy(W).cuda() for W in p.W0s]
    res = {"shape": list(dims), "r": r, "outer": outer, "q": q,
           "finite_modes": [k for k in range(3) if finite[k]]}
    for prec in ("fp64", "mixed_bf16"):
        s = AlsSolver(Ks, [u for u, _ in eig], [d for _, d in eig], coords, y, r, p.lams,
                      p.rho, p.tol, 0.0, outer, maxit=p.maxit, precision=prec, n=list(dims))
        s.run(W0)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, info, errors = s.run(W0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[prec] = {"ms_per_outer": 1e3 * dt / info.outer, "errors": errors,
                     "inner_iters": info.inner_iters, "capped": info.capped}
        s.close()
    eigs = [None if K is None else O.kernel_eig(K) for K in p.Ks]
    t_or, ref = host_median(lambda: O.cp_hifi_als(p.Ks, p.coords, p.y, p.W0s, p.lams, p.rho,
                                                  max_outer=1, als_tol=0.0, solver="pcg",
                                                  tol=p.tol, maxit=p.maxit, eigs=eigs),
                            reps=1)
    res["oracle_ms_per_outer"] = 1e3 * t_or
    res["oracle_errors_first_outer"] = ref.errors
    res["gpu_fp64_vs_oracle"] = res["oracle_ms_per_outer"] / res["fp64"]["ms_per_outer"]
    log(f"ALS {dims} r={r}: fp64 {res['fp64']['ms_per_outer']:.1f} ms / outer iteration, "
        f"mixed {res['mixed_bf16']['ms_per_outer']:.1f} ms; oracle {1e3 * t_or:.0f} ms; "
        f"errors {['%.4f' % e for e in res['fp64']['errors']]}")
    return res


# ------------------------------------------------------------- batched (C5)
def bench_batch(a, torch, C):
    """The batched workload: one persistent graph launch for all members
    (mixed BF16) against the FP64 PCG over the members in turn, both refined
    to the same relative residual."""
    from paper_2603_25691_amd.torch_api import BatchSolver, UISolver, upload
    from synth import batch_members

    t0 = time.time()
    probs, dps = [], []
    for b, bm in enumerate(batch_members(seed=0, count=a.batch_count)):
        p = bm.problem
        eig = None
        if a.eig_dir:
            z = np.load(os.path.join(a.eig_dir, f"eig{b}.npz"), allow_pickle=False)
            eig = (z["UK"], z["dK"])
        dp = upload(p, ldk_align=KROW_ALIGN, eig=eig)
        if a.save_eig:
            os.makedirs(a.save_eig, exist_ok=True)
            np.savez(os.path.join(a.save_eig, f"eig{b}.npz"),
                     UK=dp.UK[:, :p.n].cpu().numpy(), dK=dp.dK.cpu().numpy())
        dps.append(dp)
        probs.append(p)
        if (b + 1) % 8 == 0:
            log(f"batch: {b + 1} members uploaded with eig(K) ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    ns = np.array([p.n for p in probs])
    rs = np.array([p.r for p in probs])
    log(f"batch: {len(probs)} members, n {ns.min()}..{ns.max()} (sum n^2 = {np.sum(ns**2.0):.3e}),"
        f" r {sorted(set(rs.tolist()))}; generated, uploaded, eig(K) in {time.time() - t0:.1f} s")
    tol = BATCH_TOL
    t0 = time.time()
    table = BATCH_TILES if os.path.exists(BATCH_TILES) else None
    bs = BatchSolver(dps, [p.lam for p in probs], [p.rho for p in probs], tol, tile_table=table)
    # the right-hand sides b = K B of the FP64 baseline (the batched solve
    # starts from the observed values and forms its own, inside the launch)
    rhs = bs.rhs()
    Ws = [torch.empty_like(b) for b in rhs]
    bs.bind(bs.ys(), Ws)
    status, infos = bs.solve()
    torch.cuda.synchronize()
    log(f"batch: created + first solve in {time.time() - t0:.1f} s, status {status}")
    timer = StepTimer(torch)
    ms_batch, ms_mean, _ = timer.run(lambda: bs.solve(wait=False), a.batch_steps)
    status, infos = bs.info()
    rounds, grid = bs.rounds()
    phase = bs.phase_ms()
    log("batch phases (ms, last launch): " + ", ".join(f"{k} {v:.2f}" for k, v in phase.items()))
    log(f"batch mixed: {ms_batch:.2f} ms per batch ({len(probs) * 1e3 / ms_batch:.1f} "
        f"subproblem solves/s), {rounds} rounds, grid {grid}, status {C.status_string(status)}")

    # FP64 PCG (paper form), members one after another, to the same target,
    # each a whole subproblem from its observed values as in the batched launch
    solvers = [UISolver(dp, p.lam, p.rho, tol, precision="fp64") for p, dp in zip(probs, dps)]
    W64 = [torch.empty_like(b) for b in rhs]

    def fp64_all():
        its = []
        for s_, W in zip(solvers, W64):
            _, info = s_.solve_subproblem(W=W)
            its.append(info.iters)
        return its

    fp64_all()  # warm-up
    ms64, _, it64 = timer.run(fp64_all, 2)
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
        "tol": tol,
        "ms_per_batch": ms_batch, "ms_per_batch_mean": ms_mean,
        "solves_per_s": len(probs) * 1e3 / ms_batch,
        "status": C.status_string(status), "rounds": rounds, "grid": grid,
        "phase_ms": phase,
        "inner_iters_max": max(i.iters for i in infos),
        "refine_steps_max": max(i.refine_steps for i in infos),
        "relres_max": max(i.relres_true for i in infos),
        "fp64_tol": tol,
        "fp64_ms_per_batch": ms64, "fp64_solves_per_s": len(probs) * 1e3 / ms64,
        "fp64_iters_max": max(it64),
        "mixed_vs_fp64_speedup": ms64 / ms_batch,
        "e_KW_vs_fp64_max": max(ekw),
        "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": gbps / HBM_PEAK_GBPS,
                     "traffic": BATCH_TRAFFIC if len(probs) == 64 else None,
                     "kernel": "batch_kernel (whole batched solve, n x n passes only)",
                     "algorithmic_bytes": byts},
    }
    bs.close()
    return out


# ------------------------------------------------------------ CPU baseline
def cpu_baseline(p, iters: int, budget_s: float = 25.0):
    """The oracle's PCG (Section 4.4: two-step product, eq. fx preconditioner,
    numpy FP64) run on the host at the full size for a bounded number of
    iterations, projected to a whole solve: right-hand side + `iters`
    iterations (the FP64 GPU run's count to the same residual).  The host
    eigendecomposition of K at this n would take tens of minutes (one-time
    setup on both sides, excluded as on the GPU), so K stands in for U_K in the
    preconditioner; its cost does not depend on the eigenvector values."""
    import oracle as O

    model, cores = cpu_info()
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    V = O.gram_V(p.A, p.B)
    dV, UV = np.linalg.eigh(V)
    dK = np.ones(p.n)
    t0 = time.perf_counter()
    rhs = O.rhs_matrix(p.K, O.mttkrp_observed(p.y, Zhat, p.obs_t, p.n))
    t_rhs = time.perf_counter() - t0
    counted = {"it": 0}

    def A(X):
        counted["it"] += 1
        return O.matvec_twostep(p.K, Zhat, p.obs_t, p.lam, p.rho, X)

    def M(X):
        return O.precond_apply(p.K, dK, UV, dV, p.gamma, p.lam, p.rho, X)

    k = 1
    t0 = time.perf_counter()
    O.pcg(A, M, rhs, 1e-30, k)
    t_one = time.perf_counter() - t0
    k = max(1, min(4, int(budget_s / max(t_one, 1e-3))))
    t0 = time.perf_counter()
    res = O.pcg(A, M, rhs, 1e-30, k)
    t_k = time.perf_counter() - t0
    # pcg does one preconditioner apply before the loop and one per iteration
    per_it = t_k / max(res.iters, 1)
    per_solve = t_rhs + iters * per_it
    return {
        "value": 1.0 / per_solve,
        "unit": "solves/s",
        "cores": cores,
        "kind": "oracle",
        "projected": True,
        "cpu_model": model,
        "sample": (f"{res.iters} iterations of the oracle's PCG at full size "
                   f"({per_it:.2f} s each, products, gather-scatter and eq. fx apply) and its "
                   f"right-hand side ({t_rhs:.2f} s) on {cores} host threads ({model}); "
                   f"projected to one solve = right-hand side + {iters} iterations (the FP64 "
                   f"GPU run's count to the same residual) = {per_solve:.1f} s"),
    }


# ---------------------------------------------------------------- headline
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
    if a.small_only:
        print(json.dumps(bench_small(torch, C, max(a.steps, 10))), flush=True)
        return
    if a.batch_only:
        if a.calib_copy_mb > 0:
            src = torch.empty(a.calib_copy_mb * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
            src.fill_(1.0)
            torch.empty_like(src).copy_(src)
            torch.cuda.synchronize()
            log(f"calibration copy of {a.calib_copy_mb} MiB done")
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
    timer = StepTimer(torch)

    if a.calib_copy_mb > 0:
        src = torch.empty(a.calib_copy_mb * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {a.calib_copy_mb} MiB done")

    read_bw = achievable_read(torch, C)
    log(f"achievable HBM read {read_bw['GB_per_s']:.0f} GB/s ({read_bw['blocks']} workgroups)")

    # ---------------------------------------------------------------- matvec
    sf = UISolver(dp, p.lam, p.rho, p.tol, precision="fp64", check_every=1)
    X = torch.randn(n, r, dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    for _ in range(2):
        sf.apply(X, out=Y)
    torch.cuda.synchronize()
    mv_ms, _, _ = timer.run(lambda: sf.apply(X, out=Y), 10)
    mv_bytes = 2 * 8 * n * n + 16 * n * r + 8 * q
    log(f"matvec {mv_ms:.3f} ms = {mv_bytes / mv_ms / 1e6:.0f} GB/s")
    # the same operator with the fiber-collapsed gather (every time point of
    # this workload is one complete fiber: its sample at all J features)
    sfc = UISolver(dp, p.lam, p.rho, p.tol, precision="fp64", check_every=1,
                   flags=C.FLAG_FIBER_COLLAPSE)
    Yc = torch.empty_like(X)
    for _ in range(2):
        sfc.apply(X, out=Yc)
    torch.cuda.synchronize()
    mvc_ms, _, _ = timer.run(lambda: sfc.apply(X, out=Yc), 10)
    mvc_diff = float((Yc - Y).norm() / Y.norm())
    sfc.close()
    log(f"matvec with the fiber-collapsed gather {mvc_ms:.3f} ms (rel. diff {mvc_diff:.1e})")

    # ------------------------------------------------------------ FP64 PCG
    def fp64_run(tol, flags=0, with_w=None):
        s = UISolver(dp, p.lam, p.rho, tol, precision="fp64", flags=flags, check_every=1)
        W, info = s.solve_subproblem(W=with_w)
        torch.cuda.synchronize()
        t, g_ms, g_n = [], 0.0, 0
        for _ in range(a.fp64_steps):
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            W, info = s.solve_subproblem(W=W)
            torch.cuda.synchronize()
            t.append(time.perf_counter() - s0)
            g_ms += info.gemm_ms
            g_n += info.gemm_launches
        s.close()
        ms = 1e3 * float(np.median(t))
        return W, {"ms_per_solve": ms, "solves_per_s": 1e3 / ms, "tol": tol,
                   "iters": info.iters, "relres_true": info.relres_true,
                   "status": C.status_string(info.status),
                   "gemm_avg_ms": g_ms / max(g_n, 1),
                   "gemm_launches_per_solve": g_n // max(1, len(t))}

    # the paper-form FP64 PCG at the mixed form's residual target (the
    # baseline of the mixed-vs-FP64 ratio) and at the workload's own 1e-8
    W64, fp64 = fp64_run(MIXED_TOL, flags=TK)
    log(f"fp64 PCG (tol {MIXED_TOL:g}): {fp64}")
    W64c, fp64_cfg = fp64_run(p.tol, flags=TK)
    log(f"fp64 PCG (tol {p.tol:g}): {fp64_cfg}")
    # the same FP64 PCG in the eigenbasis of K (x = U_K xbar, the rotation of
    # Section 3.3): two n x n passes per iteration instead of four
    _, fp64_eig = fp64_run(MIXED_TOL, flags=C.FLAG_EIGENBASIS)
    log(f"fp64 PCG in the eigenbasis (tol {MIXED_TOL:g}): {fp64_eig}")
    # a tight FP64 solution: the reference both are measured against
    sT = UISolver(dp, p.lam, p.rho, 1e-10, precision="fp64", check_every=1)
    WT, infoT = sT.solve_subproblem()
    torch.cuda.synchronize()
    sT.close()
    fp64_bytes = 8 * n * n + 16 * n * r

    # --------------------------------------------------- headline (mixed) form
    prec = a.precision
    tol = MIXED_TOL if prec != "fp64" else p.tol
    sm = UISolver(dp, p.lam, p.rho, tol, precision=prec, flags=TK, check_every=1)
    W, info = sm.solve_subproblem()
    for _ in range(max(0, a.warmup - 1)):
        W, info = sm.solve_subproblem(W=W)
    torch.cuda.synchronize()
    rec = {"g_ms": 0.0, "g_n": 0, "infos": []}

    def step():
        Wn, inf = sm.solve_subproblem(W=W)
        rec["g_ms"] += inf.gemm_ms
        rec["g_n"] += inf.gemm_launches
        rec["infos"].append(inf.as_dict())
        return Wn

    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ms_per_step, ms_mean, W = timer.run(step, a.steps)
    wall = time.perf_counter() - wall0
    value = 1e3 / ms_per_step
    infos = rec["infos"]
    log(f"{prec}: {ms_per_step:.2f} ms/solve (median; mean {ms_mean:.2f}), {value:.2f} "
        f"solves/s, wall {wall:.2f} s, last {infos[-1]}")
    lp_avg = rec["g_ms"] / max(rec["g_n"], 1)
    lp_launches = rec["g_n"] / a.steps

    # the FP64 products inside the same mixed solve (rotations, FP64
    # residuals, certificate), timed in extra solves of their own
    f64_avg, f64_launches = None, None
    if prec != "fp64":
        s64 = UISolver(dp, p.lam, p.rho, tol, precision=prec, flags=TK | C.FLAG_TIME_FP64,
                       check_every=1)
        Wx, ix = s64.solve_subproblem()
        g_ms, g_n = 0.0, 0
        for _ in range(3):
            Wx, ix = s64.solve_subproblem(W=Wx)
            g_ms += ix.gemm_ms
            g_n += ix.gemm_launches
        s64.close()
        del Wx
        f64_avg, f64_launches = g_ms / max(g_n, 1), g_n / 3

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
        mvl_ms, _, _ = timer.run(lambda: sm.apply_lowp(xb, out=yb), 10)
        esz = 2 if prec == "mixed_bf16" else 4
        mvl_bytes = 2 * (esz * n * n + 16 * n * r) + 8 * q
        mvl = {"ms": mvl_ms, "GB_per_s": mvl_bytes / mvl_ms / 1e6,
               "frac_of_peak": mvl_bytes / mvl_ms / 1e6 / HBM_PEAK_GBPS, "bytes": mvl_bytes,
               "operator": "eigenbasis inner operator of the mixed solve (cphifi_ui_apply_lowp)"}
        log(f"inner-operator matvec {mvl_ms:.3f} ms = {mvl_bytes / mvl_ms / 1e6:.0f} GB/s")

    # ------------------------------------------------------------- accuracy
    Wh, WTh = W.cpu().numpy(), WT.cpu().numpy()
    KWT = p.K @ WTh

    def ekw_t(Wx):
        return float(np.linalg.norm(p.K @ Wx - KWT) / np.linalg.norm(KWT))

    acc = {"relres_true": infos[-1]["relres_true"], "status": infos[-1]["status"],
           "reference": f"FP64 GPU PCG to relres 1e-10 (certified {infoT.relres_true:.2e})",
           "e_KW_mixed": ekw_t(Wh), "e_KW_fp64_same_target": ekw_t(W64.cpu().numpy()),
           "e_KW_fp64_tol_1e-8": ekw_t(W64c.cpu().numpy())}
    if not a.no_oracle_check:
        import oracle as O

        Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
        t0 = time.time()
        acc["oracle_relres_certificate"] = O.relres(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho, Wh)
        log(f"oracle residual certificate {acc['oracle_relres_certificate']:.3e} "
            f"({time.time() - t0:.1f} s)")
    log(f"accuracy: {acc}")

    if prec == "mixed_bf16":
        lp_bytes, kname = 2 * n * n + 16 * n * r, BF16_KERNEL
    elif prec == "mixed_fp32":
        lp_bytes, kname = 4 * n * n + 16 * n * r, "gemm_k4_kernel<float, 3, 2, 4, false, 4>"
    else:
        lp_bytes, kname = fp64_bytes, F64_KERNEL
    roof_lp = roofline_hbm(kname, lp_bytes, lp_avg, lp_launches, n, r)
    roofs = [roof_lp]
    if f64_avg is not None:
        roofs.append(roofline_hbm(F64_KERNEL, fp64_bytes, f64_avg, f64_launches, n, r))
    # the kernel that takes most of the timed solve is the headline roofline
    roofs.sort(key=lambda x: -x["ms_per_solve"])
    for rf in roofs:
        rf["frac_of_achievable_read"] = rf["achieved"] / read_bw["GB_per_s"]
    roof = dict(roofs[0], share_of_solve=roofs[0]["ms_per_solve"] / ms_per_step)
    # at r = 40 the FP64 product also sits at the FP64 MFMA ridge: flops per launch
    if roof["kernel"] == F64_KERNEL:
        fl = 2.0 * n * n * r
        roof["mfma_tflops"] = fl / (roof["avg_launch_ms"] * 1e9)
        roof["mfma_frac_fp64_peak"] = roof["mfma_tflops"] / FP64_PEAK_TFLOPS
    fp64_roof = roofline_hbm(F64_KERNEL, fp64_bytes, fp64["gemm_avg_ms"],
                             fp64["gemm_launches_per_solve"], n, r)

    out = {
        "metric": "RKHS-subproblem solves/sec to 1e-6 rel err; matvec HBM GB/s; mixed vs FP64",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_mean": ms_mean,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed_bf16": "bf16+f64", "mixed_fp32": "f32+f64", "fp64": "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": (f"unaligned RKHS subproblem: I={p.I} J={p.J} m_i~U{{10..50}} "
                                f"n={n} q={q} r={r} Matern-3/2(0.1) lambda={p.lam} "
                                f"rho={p.rho} seed=0"),
                   "form": prec, "n": n, "q": q, "r": r, "tol": tol},
        "roofline": roof,
        "roofline_second": roofs[1] if len(roofs) > 1 else None,
        "fp64": dict(fp64, roofline=fp64_roof),
        "fp64_tol_1e-8": fp64_cfg,
        "matvec": {"ms": mv_ms, "GB_per_s": mv_bytes / mv_ms / 1e6,
                   "frac_of_peak": mv_bytes / mv_ms / 1e6 / HBM_PEAK_GBPS,
                   "frac_of_achievable_read": mv_bytes / mv_ms / 1e6 / read_bw["GB_per_s"],
                   "bytes": mv_bytes, "operator": "FP64 paper form (cphifi_ui_apply)"},
        "hbm_read_achievable": read_bw,
        "matvec_fiber_collapse": {"ms": mvc_ms, "rel_diff_vs_matvec": mvc_diff,
                                  "operator": "FP64 paper form, FLAG_FIBER_COLLAPSE"},
        "matvec_mixed": mvl,
        "mixed_vs_fp64_speedup": fp64["ms_per_solve"] / ms_per_step,
        "fp64_eigenbasis": dict(fp64_eig,
                                mixed_speedup=fp64_eig["ms_per_solve"] / ms_per_step),
        "accuracy": acc,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, fp64["iters"])
        log(f"cpu baseline {out['cpu_baseline']}")
    del sf, sm, dp, W, W64, W64c, WT
    torch.cuda.empty_cache()
    if not a.no_small:
        out["small"] = bench_small(torch, C, max(a.steps, 10))
    if not a.no_aligned:
        out["aligned"] = bench_aligned(torch, C, max(3, min(a.steps, 10)))
    if not a.no_paper_shapes:
        out["paper_shapes"] = bench_paper_shapes(torch, C, max(3, min(a.steps, 10)))
    if a.batch_count > 0:
        out["batched"] = bench_batch(a, torch, C)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
