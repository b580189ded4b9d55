"""Tile autotuner for the n x n by n x r product kernels.

  python -m paper_2603_25691_amd.tune sweep --n 500 2000 8000 30658 --r 5 10 20 40 \
      --elt fp64 bf16 --out tiles.txt
  python -m paper_2603_25691_amd.tune measure --n 30658 --r 40 --elt bf16 --reps 4 \
      --calib-mb 1024
  python -m paper_2603_25691_amd.tune batch --count 64 \
      --out paper_2603_25691_amd/tiles_batch_mi355x.txt

`sweep` times every (mw, s, ksplit) tile of cphifi_product for each size and
writes the fastest per (element type, orientation, r, n) to a plain-text table
that plans read when CPHIFI_TILE_TABLE names it.  Table line format:

    <elt> <trans> <r_lo> <r_hi> <n_lo> <n_hi> <mw> <s> <ksplit>

with elt in {f64, f32, bf16}; the first line whose ranges contain (r, n) wins.

`batch` tunes the tiles of the persistent batched solver on the synthetic
batched workload itself (members of uneven n and r): inside one launch the
members' product items share the grid, so the best split-K depth there is not
the one of a product launched alone.  For each candidate -- a target k-range
length per work item and the BF16 rows per wave -- it writes a table, times
batched solves with it, and keeps the fastest table.

`measure` runs the chosen product `reps` times after a plain device copy of
known size, so a hardware-counter run (e.g. rocprofv3 --pmc FETCH_SIZE) can scale
the product's HBM bytes by what the counter reads for the copy.
"""

from __future__ import annotations

import argparse
import json
import sys

import torch

from . import cphifi as C
from .torch_api import bf16_tiles, product

TILES = {"fp64": [(1, 4), (1, 8), (2, 4), (2, 8), (4, 2), (4, 4)],
         "fp32": [(1, 4), (1, 8), (2, 4), (2, 8), (4, 4)],
         "bf16": [(1, 4), (2, 2), (2, 4), (4, 2)]}
TAG = {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}
# the solver's BF16 copies of U_K are tiled, so that is the layout timed
PRODUCT_ELT = {"fp64": "fp64", "fp32": "fp32", "bf16": "bf16_tiled"}
ESIZE = {"fp64": 8, "fp32": 4, "bf16": 2}


def _operand(elt: str, n: int, gen: torch.Generator, ld_align: int = 1) -> torch.Tensor:
    U = torch.rand(n, n, dtype=torch.float64, device="cuda", generator=gen)
    if elt in ("fp64", "fp32"):
        if elt == "fp32":
            U = U.float()
        ld = (n + ld_align - 1) // ld_align * ld_align
        if ld == n:
            return U
        Up = torch.zeros(n, ld, dtype=U.dtype, device="cuda")
        Up[:, :n] = U
        return Up[:, :n]  # row stride ld
    ld = (n + 255) // 256 * 256
    Ub = torch.zeros(n, ld, dtype=torch.bfloat16, device="cuda")
    Ub[:, :n] = U.to(torch.bfloat16)
    return bf16_tiles(Ub)


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def sweep(ns, rs, elts, out_path: str, reps: int = 5, ld_align: int = 1) -> None:
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    lines = []
    for elt in elts:
        transes = (False,) if elt == "bf16" else (False, True)
        for n in sorted(ns):
            U = _operand(elt, n, gen, ld_align)
            for r in sorted(rs):
                X = torch.rand(n, r, dtype=torch.float64, device="cuda", generator=gen)
                Y = torch.empty_like(X)
                ws = torch.empty(C.cphifi_product_workspace_bytes(n, r, C.ELT_BF16) + 256,
                                 dtype=torch.uint8, device="cuda")
                for trans in transes:
                    best = None
                    for tile in TILES[elt]:
                        for ks in (0, 1, 2, 4, 8):
                            ms = _time(lambda: product(U, X, PRODUCT_ELT[elt], trans, tile,
                                                       ks, out=Y, workspace=ws), reps)
                            rec = {"elt": elt, "trans": trans, "n": n, "r": r, "tile": tile,
                                   "ksplit": ks, "ms": ms,
                                   "GBps": (ESIZE[elt] * n * n + 16 * n * r) / ms / 1e6}
                            print(json.dumps(rec), flush=True)
                            if best is None or ms < best["ms"]:
                                best = rec
                    lines.append((elt, trans, n, r, best))
            del U
            torch.cuda.empty_cache()
    # ranges: each measured n covers up to the next measured n; each r up to the next r
    ns_s, rs_s = sorted(ns), sorted(rs)
    with open(out_path, "w") as f:
        f.write("# elt trans r_lo r_hi n_lo n_hi mw s ksplit  (tile table, MI355X)\n")
        for elt, trans, n, r, b in lines:
            i, k = ns_s.index(n), rs_s.index(r)
            n_lo = 1 if i == 0 else ns_s[i - 1] + 1
            n_hi = n if i + 1 < len(ns_s) else 1 << 31
            r_lo = 1 if k == 0 else rs_s[k - 1] + 1
            r_hi = r if k + 1 < len(rs_s) else 64
            f.write(f"{TAG[elt]} {int(trans)} {r_lo} {r_hi} {n_lo} {n_hi} {b['tile'][0]} "
                    f"{b['tile'][1]} {b['ksplit']}\n")
    print(f"wrote {out_path}", file=sys.stderr)


def measure(n: int, r: int, elts, reps: int, calib_mb: int, trans: bool = False,
            ld_align: int = 1) -> None:
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    if calib_mb > 0:
        src = torch.ones(calib_mb * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": calib_mb * 2 ** 20}), flush=True)
    for elt in elts:
        U = _operand(elt, n, gen, ld_align)
        X = torch.rand(n, r, dtype=torch.float64, device="cuda", generator=gen)
        Y = torch.empty_like(X)
        ws = torch.empty(C.cphifi_product_workspace_bytes(n, r, C.ELT_BF16) + 256,
                         dtype=torch.uint8, device="cuda")
        ms = _time(lambda: product(U, X, PRODUCT_ELT[elt], trans and elt != "bf16", (0, 0), 0,
                                   out=Y, workspace=ws), reps)
        print(json.dumps({"elt": elt, "n": n, "r": r, "ms": ms, "reps": reps,
                          "trans": bool(trans and elt != "bf16"), "ld": U.stride(0),
                          "algorithmic_bytes": ESIZE[elt] * n * n + 16 * n * r}), flush=True)
        del U
        torch.cuda.empty_cache()


BATCH_KRANGE = (768, 1024, 1536, 2048, 3072, 4096)
BATCH_BF16_MW = (2, 4)
BATCH_BIN = 512  # n bins of the batch table


def _batch_table(path: str, krange: int, bf_mw: int, n_max: int) -> None:
    """Split-K depth ~ n / krange per bin of n (midpoint), BF16 rows per wave
    bf_mw; the FP64 tiles of the batched kernel are fixed, only their depth
    comes from the table."""
    with open(path, "w") as f:
        f.write(f"# batched solver tiles (MI355X): k-range ~{krange}, bf16 mw {bf_mw}\n")
        f.write("# elt trans r_lo r_hi n_lo n_hi mw s ksplit\n")
        for lo in range(1, n_max + 1, BATCH_BIN):
            hi = lo + BATCH_BIN - 1
            ks = max(1, min(16, round((lo + hi) / 2 / krange)))
            f.write(f"bf16 0 1 64 {lo} {hi} {bf_mw} 2 {ks}\n")
            f.write(f"f64 0 1 64 {lo} {hi} 2 4 {ks}\n")
            f.write(f"f64 1 1 64 {lo} {hi} 2 4 {ks}\n")


def batch(count: int, seed: int, out_path: str, reps: int = 3) -> None:
    import os
    import tempfile

    from synth import batch_members

    from .torch_api import BatchSolver, upload

    probs, dps = [], []
    for bm in batch_members(seed=seed, count=count):
        probs.append(bm.problem)
        dps.append(upload(bm.problem, ldk_align=8))
    torch.cuda.synchronize()
    n_max = (max(p.n for p in probs) + BATCH_BIN - 1) // BATCH_BIN * BATCH_BIN
    tmp = tempfile.mkdtemp(prefix="cphifi_tune_")
    best = None
    for kr in BATCH_KRANGE:
        for mw in BATCH_BF16_MW:
            # a fresh file name per candidate: plans cache tables by path
            path = os.path.join(tmp, f"batch_k{kr}_mw{mw}.txt")
            _batch_table(path, kr, mw, n_max)
            bs = BatchSolver(dps, [p.lam for p in probs], [p.rho for p in probs], probs[0].tol,
                             tile_table=path)
            try:
                # the batched solve starts from the observed values
                Ws = [torch.empty(p.n, p.r, dtype=torch.float64, device=p.K.device)
                      for p in dps]
                bs.bind(bs.ys(), Ws)
                status, _ = bs.solve()
                ms = _time(lambda: bs.solve(wait=False), reps)
                status, infos = bs.info()
            finally:
                bs.close()
            rec = {"krange": kr, "bf16_mw": mw, "ms_per_batch": ms,
                   "status": C.status_string(status),
                   "relres_max": max(i.relres_true for i in infos)}
            print(json.dumps(rec), flush=True)
            if status == C.OK and (best is None or ms < best[0]):
                best = (ms, kr, mw)
    if best is None:
        raise SystemExit("no candidate solved the batch")
    _batch_table(out_path, best[1], best[2], max(n_max, 1 << 15))
    print(f"wrote {out_path} (k-range {best[1]}, bf16 mw {best[2]}, {best[0]:.2f} ms)",
          file=sys.stderr)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("sweep")
    s.add_argument("--n", type=int, nargs="+", required=True)
    s.add_argument("--r", type=int, nargs="+", required=True)
    s.add_argument("--elt", nargs="+", default=["fp64", "bf16"])
    s.add_argument("--out", default="tiles.txt")
    s.add_argument("--reps", type=int, default=5)
    s.add_argument("--ld-align", type=int, default=1,
                   help="FP64 / FP32 operand row stride rounded up to a multiple of this")
    m = sub.add_parser("measure")
    m.add_argument("--n", type=int, required=True)
    m.add_argument("--r", type=int, required=True)
    m.add_argument("--elt", nargs="+", default=["bf16", "fp64"])
    m.add_argument("--reps", type=int, default=4)
    m.add_argument("--calib-mb", type=int, default=1024)
    m.add_argument("--ld-align", type=int, default=1,
                   help="FP64 / FP32 operand row stride rounded up to a multiple of this")
    m.add_argument("--trans", action="store_true",
                   help="the transposed product (FP64 / FP32 only)")
    b = sub.add_parser("batch")
    b.add_argument("--count", type=int, default=64)
    b.add_argument("--seed", type=int, default=0)
    b.add_argument("--reps", type=int, default=3)
    b.add_argument("--out", default="tiles_batch.txt")
    a = ap.parse_args(argv)
    if a.cmd == "sweep":
        sweep(a.n, a.r, a.elt, a.out, a.reps, ld_align=a.ld_align)
    elif a.cmd == "batch":
        batch(a.count, a.seed, a.out, a.reps)
    else:
        measure(a.n, a.r, a.elt, a.reps, a.calib_mb, trans=a.trans, ld_align=a.ld_align)


if __name__ == "__main__":
    main()
