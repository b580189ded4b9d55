"""ctypes binding of libcphifi.so (the C ABI in include/cphifi.h).

Functions keep the C names and take plain integers for device pointers and the
HIP stream.  Nothing here computes: every step of the solve runs in the
library's HIP kernels.  The library must be built in-tree
(``python -m paper_2603_25691_amd.build``); importing this module raises if it
is missing, and there is no fallback path.
"""

from __future__ import annotations

import ctypes as C
import os
import re
from typing import Optional

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcphifi.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "cphifi.h")

# ------------------------------------------------------------ constants
OK = 0
INVALID_ARG = 1
HIP_ERROR = 2
UNSUPPORTED = 3
BREAKDOWN = 4
NUMERIC = 5
NOT_CONVERGED = 6

FP64 = 0
MIXED_FP32 = 1
MIXED_BF16 = 2

FLAG_WARM_START = 1
FLAG_VALIDATE = 2
FLAG_TIME_KERNELS = 4
FLAG_NO_PRECOND = 8
FLAG_EIGENBASIS = 16
FLAG_NO_UKT_COPY = 32
FLAG_TIME_FP64 = 64
FLAG_PERSISTENT = 128
FLAG_TOEPLITZ_K = 256
FLAG_FIBER_COLLAPSE = 512
FLAG_NO_GRAPH = 1024
FLAG_NO_PERSISTENT = 2048
FLAG_FP64_RESIDUALS = 4096

PRECISIONS = {"fp64": FP64, "mixed_fp32": MIXED_FP32, "mixed_bf16": MIXED_BF16}


class cphifi_ui_desc(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("r", C.c_int64), ("q", C.c_int64), ("I", C.c_int64),
        ("J", C.c_int64), ("ldk", C.c_int64),
        ("lambda_", C.c_double), ("rho", C.c_double), ("gamma", C.c_double),
        ("tol", C.c_double), ("inner_tol", C.c_double),
        ("precision", C.c_int32), ("flags", C.c_int32), ("maxit", C.c_int32),
        ("max_refine", C.c_int32), ("check_every", C.c_int32), ("reserved", C.c_int32),
    ]


class cphifi_ui_inputs(C.Structure):
    _fields_ = [(name, C.c_void_p) for name in
                ("K", "UK", "dK", "obs_ptr", "obs_i", "obs_j", "A", "B", "Zhat", "V")]


class cphifi_solve_info(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("iters", C.c_int32), ("refine_steps", C.c_int32),
        ("gemm_launches", C.c_int32), ("relres_true", C.c_double),
        ("relres_recursive", C.c_double), ("gemm_ms", C.c_double),
        ("history", C.c_void_p),
    ]

    def as_dict(self):
        return {
            "status": status_string(self.status), "iters": self.iters,
            "refine_steps": self.refine_steps, "relres_true": self.relres_true,
            "relres_recursive": self.relres_recursive, "gemm_ms": self.gemm_ms,
            "gemm_launches": self.gemm_launches,
        }


ALIGNED_DECOUPLED = 0
ALIGNED_PCG = 1
ALIGNED_METHODS = {"decoupled": ALIGNED_DECOUPLED, "pcg": ALIGNED_PCG}


class cphifi_aligned_desc(C.Structure):
    _fields_ = [("n", C.c_int64), ("r", C.c_int64), ("ldk", C.c_int64),
                ("lambda_", C.c_double), ("tol", C.c_double),
                ("method", C.c_int32), ("maxit", C.c_int32)]


class cphifi_aligned_inputs(C.Structure):
    _fields_ = [(name, C.c_void_p) for name in ("UK", "dK", "Bm", "V", "A", "B")] + \
               [("I", C.c_int64), ("J", C.c_int64)]


class cphifi_als_desc(C.Structure):
    _fields_ = [("n", C.c_int64 * 3), ("q", C.c_int64), ("r", C.c_int64),
                ("lambda_", C.c_double * 3), ("rho", C.c_double), ("tol", C.c_double),
                ("als_tol", C.c_double), ("precision", C.c_int32), ("flags", C.c_int32),
                ("maxit", C.c_int32), ("max_outer", C.c_int32), ("finite", C.c_int32 * 3),
                ("reserved", C.c_int32)]


class cphifi_als_inputs(C.Structure):
    _fields_ = [("K", C.c_void_p * 3), ("UK", C.c_void_p * 3), ("dK", C.c_void_p * 3),
                ("coords", C.c_void_p), ("y", C.c_void_p)]


class cphifi_als_info(C.Structure):
    _fields_ = [("outer", C.c_int32), ("converged", C.c_int32), ("inner_iters", C.c_int32),
                ("capped", C.c_int32), ("rel_error", C.c_double), ("errors", C.c_void_p)]

    def as_dict(self):
        return {"outer": self.outer, "converged": bool(self.converged),
                "inner_iters": self.inner_iters, "capped": self.capped,
                "rel_error": self.rel_error}


class CphifiError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {status_string(status)}: {detail}")
        self.status = status


def _single_hip_runtime() -> None:
    """torch ships its own libamdhip64 under the same SONAME as ROCm's.  Loading
    torch first makes the dynamic linker resolve this library's HIP runtime to
    torch's copy, so device memory from torch and kernels launched here live in
    one runtime.  (Loading this library first would give the process two HIP
    runtimes, and the second one to initialise sees no device.)"""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def _load() -> C.CDLL:
    _single_hip_runtime()
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2603_25691_amd.build` "
            "(the HIP library is the only implementation; there is no fallback)")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "cphifi_ui_workspace_bytes": (C.c_int, [C.POINTER(cphifi_ui_desc), C.POINTER(C.c_size_t)]),
        "cphifi_ui_plan_create": (C.c_int, [C.POINTER(P), C.POINTER(cphifi_ui_desc),
                                            C.POINTER(cphifi_ui_inputs), P, C.c_size_t, P]),
        "cphifi_ui_setup": (C.c_int, [P]),
        "cphifi_ui_rhs": (C.c_int, [P, P, P]),
        "cphifi_ui_mttkrp": (C.c_int, [P, P, P]),
        "cphifi_ui_apply": (C.c_int, [P, P, P]),
        "cphifi_ui_precond": (C.c_int, [P, P, P]),
        "cphifi_ui_apply_lowp": (C.c_int, [P, P, P]),
        "cphifi_ui_solve": (C.c_int, [P, P, P, C.POINTER(cphifi_solve_info)]),
        "cphifi_ui_solve_subproblem": (C.c_int, [P, P, P, C.POINTER(cphifi_solve_info)]),
        "cphifi_ui_plan_destroy": (C.c_int, [P]),
        "cphifi_kernel_eig": (C.c_int, [C.c_int64, P, C.c_int64, P, P, P]),
        "cphifi_kernel_eig_jacobi": (C.c_int, [C.c_int64, P, C.c_int64, P, P, C.c_double, C.c_int,
                                               C.POINTER(C.c_int), P]),
        "cphifi_aligned_workspace_bytes": (C.c_int, [C.POINTER(cphifi_aligned_desc),
                                                     C.POINTER(C.c_size_t)]),
        "cphifi_aligned_solve": (C.c_int, [C.POINTER(cphifi_aligned_desc),
                                           C.POINTER(cphifi_aligned_inputs), P, P, C.c_size_t,
                                           P, C.POINTER(cphifi_solve_info)]),
        "cphifi_als_workspace_bytes": (C.c_int, [C.POINTER(cphifi_als_desc),
                                                 C.POINTER(C.c_size_t)]),
        "cphifi_als_create": (C.c_int, [C.POINTER(P), C.POINTER(cphifi_als_desc),
                                        C.POINTER(cphifi_als_inputs), P, C.c_size_t, P]),
        "cphifi_als_run": (C.c_int, [P, C.POINTER(P), C.POINTER(P), C.POINTER(cphifi_als_info)]),
        "cphifi_als_destroy": (C.c_int, [P]),
        "cphifi_product_workspace_bytes": (C.c_int, [C.c_int64, C.c_int64, C.c_int,
                                                     C.POINTER(C.c_size_t)]),
        "cphifi_product_tile_ok": (C.c_int, [C.c_int, C.c_int, C.c_int]),
        "cphifi_stream_read": (C.c_int, [P, C.c_int64, C.c_int32, P, P]),
        "cphifi_product_static_max_bytes": (C.c_size_t, []),
        "cphifi_product_static": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                            C.c_int64, P, C.c_int64, P, C.c_int64, P, P, P]),
        "cphifi_product": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64, P,
                                     C.c_int64, P, C.c_int64, P, P, P, C.c_size_t, P]),
        "cphifi_batch_workspace_bytes": (C.c_int, [C.c_int, C.POINTER(cphifi_ui_desc),
                                                   C.POINTER(C.c_size_t)]),
        "cphifi_batch_create": (C.c_int, [C.POINTER(P), C.c_int, C.POINTER(cphifi_ui_desc),
                                          C.POINTER(cphifi_ui_inputs), P, C.c_size_t, P,
                                          C.c_char_p]),
        "cphifi_batch_plan": (C.c_int, [P, C.c_int, C.POINTER(P)]),
        "cphifi_batch_rhs": (C.c_int, [P, C.POINTER(P), C.POINTER(P)]),
        "cphifi_batch_bind": (C.c_int, [P, C.POINTER(P), C.POINTER(P)]),
        "cphifi_batch_solve": (C.c_int, [P, C.POINTER(P), C.POINTER(P),
                                         C.POINTER(cphifi_solve_info)]),
        "cphifi_batch_info": (C.c_int, [P, C.POINTER(cphifi_solve_info)]),
        "cphifi_batch_graph": (C.c_int, [P, C.POINTER(P)]),
        "cphifi_batch_rounds": (C.c_int, [P, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "cphifi_batch_phase_ms": (C.c_int, [P, C.POINTER(C.c_double)]),
        "cphifi_batch_destroy": (C.c_int, [P]),
        "cphifi_status_string": (C.c_char_p, [C.c_int]),
        "cphifi_last_error": (C.c_char_p, []),
        "cphifi_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def lib() -> C.CDLL:
    return _lib


def declared_functions(header: str = HEADER_PATH):
    """Names of the functions include/cphifi.h declares."""
    text = open(header).read()
    return sorted(set(re.findall(r"CPHIFI_API\s+[\w\s\*]+?\b(cphifi_\w+)\s*\(", text)))


def status_string(status: int) -> str:
    return _lib.cphifi_status_string(int(status)).decode()


def last_error() -> str:
    return _lib.cphifi_last_error().decode()


def version() -> str:
    return _lib.cphifi_version().decode()


def _check(status: int, where: str, soft_ok: bool = False) -> int:
    if status == OK or (soft_ok and status == NOT_CONVERGED):
        return status
    raise CphifiError(status, where, last_error())


def cphifi_ui_workspace_bytes(desc: cphifi_ui_desc) -> int:
    out = C.c_size_t(0)
    _check(_lib.cphifi_ui_workspace_bytes(C.byref(desc), C.byref(out)),
           "cphifi_ui_workspace_bytes")
    return int(out.value)


def cphifi_ui_plan_create(desc: cphifi_ui_desc, inputs: cphifi_ui_inputs, workspace: int,
                          workspace_bytes: int, stream: int) -> int:
    plan = C.c_void_p(0)
    _check(_lib.cphifi_ui_plan_create(C.byref(plan), C.byref(desc), C.byref(inputs),
                                      C.c_void_p(workspace), C.c_size_t(workspace_bytes),
                                      C.c_void_p(stream)), "cphifi_ui_plan_create")
    return int(plan.value)


def cphifi_ui_setup(plan: int) -> None:
    _check(_lib.cphifi_ui_setup(C.c_void_p(plan)), "cphifi_ui_setup")


def cphifi_ui_rhs(plan: int, y: int, b: int) -> None:
    _check(_lib.cphifi_ui_rhs(C.c_void_p(plan), C.c_void_p(y), C.c_void_p(b)), "cphifi_ui_rhs")


def cphifi_ui_mttkrp(plan: int, y: int, Bm: int) -> None:
    _check(_lib.cphifi_ui_mttkrp(C.c_void_p(plan), C.c_void_p(y), C.c_void_p(Bm)),
           "cphifi_ui_mttkrp")


def cphifi_ui_apply(plan: int, x: int, y: int) -> None:
    _check(_lib.cphifi_ui_apply(C.c_void_p(plan), C.c_void_p(x), C.c_void_p(y)),
           "cphifi_ui_apply")


def cphifi_ui_precond(plan: int, x: int, z: int) -> None:
    _check(_lib.cphifi_ui_precond(C.c_void_p(plan), C.c_void_p(x), C.c_void_p(z)),
           "cphifi_ui_precond")


def cphifi_ui_apply_lowp(plan: int, xbar: int, ybar: int) -> None:
    _check(_lib.cphifi_ui_apply_lowp(C.c_void_p(plan), C.c_void_p(xbar), C.c_void_p(ybar)),
           "cphifi_ui_apply_lowp")


def cphifi_ui_solve(plan: int, b: int, W: int, history=None) -> cphifi_solve_info:
    info = cphifi_solve_info()
    if history is not None:
        info.history = history.ctypes.data
    st = _lib.cphifi_ui_solve(C.c_void_p(plan), C.c_void_p(b), C.c_void_p(W), C.byref(info))
    _check(st, "cphifi_ui_solve", soft_ok=True)
    return info


def cphifi_ui_solve_subproblem(plan: int, y: int, W: int, history=None) -> cphifi_solve_info:
    info = cphifi_solve_info()
    if history is not None:
        info.history = history.ctypes.data
    st = _lib.cphifi_ui_solve_subproblem(C.c_void_p(plan), C.c_void_p(y), C.c_void_p(W),
                                         C.byref(info))
    _check(st, "cphifi_ui_solve_subproblem", soft_ok=True)
    return info


def cphifi_ui_plan_destroy(plan: int) -> None:
    _check(_lib.cphifi_ui_plan_destroy(C.c_void_p(plan)), "cphifi_ui_plan_destroy")


def cphifi_kernel_eig(n: int, K: int, ldk: int, UK: int, dK: int, stream: int) -> None:
    _check(_lib.cphifi_kernel_eig(C.c_int64(n), C.c_void_p(K), C.c_int64(ldk), C.c_void_p(UK),
                                  C.c_void_p(dK), C.c_void_p(stream)), "cphifi_kernel_eig")


def cphifi_kernel_eig_jacobi(n: int, K: int, ldk: int, UK: int, dK: int, tol: float,
                             max_sweeps: int, stream: int) -> int:
    sweeps = C.c_int(0)
    _check(_lib.cphifi_kernel_eig_jacobi(n, C.c_void_p(K), ldk, C.c_void_p(UK), C.c_void_p(dK),
                                         tol, max_sweeps, C.byref(sweeps), C.c_void_p(stream)),
           "cphifi_kernel_eig_jacobi")
    return int(sweeps.value)


def make_desc(n: int, r: int, q: int, I: int = 0, J: int = 0, lam: float = 1e-3,
              rho: float = 1e-6, gamma: float = 0.0, tol: float = 1e-10,
              precision: int = FP64, flags: int = 0, maxit: int = 0, max_refine: int = 0,
              inner_tol: float = 0.0, check_every: int = 0, ldk: int = 0) -> cphifi_ui_desc:
    d = cphifi_ui_desc()
    d.n, d.r, d.q, d.I, d.J, d.ldk = n, r, q, I, J, ldk
    d.lambda_, d.rho, d.gamma, d.tol, d.inner_tol = lam, rho, gamma, tol, inner_tol
    d.precision, d.flags, d.maxit, d.max_refine = precision, flags, maxit, max_refine
    d.check_every = check_every
    return d


def make_inputs(**ptrs: Optional[int]) -> cphifi_ui_inputs:
    inp = cphifi_ui_inputs()
    for k, v in ptrs.items():
        setattr(inp, k, None if v is None else int(v))
    return inp


def make_aligned_desc(n: int, r: int, lam: float, method: int, tol: float = 0.0,
                      maxit: int = 0, ldk: int = 0) -> cphifi_aligned_desc:
    d = cphifi_aligned_desc()
    d.n, d.r, d.ldk, d.lambda_, d.tol, d.method, d.maxit = n, r, ldk, lam, tol, method, maxit
    return d


def cphifi_aligned_workspace_bytes(desc: cphifi_aligned_desc) -> int:
    out = C.c_size_t(0)
    _check(_lib.cphifi_aligned_workspace_bytes(C.byref(desc), C.byref(out)),
           "cphifi_aligned_workspace_bytes")
    return int(out.value)


def cphifi_aligned_solve(desc: cphifi_aligned_desc, inputs: cphifi_aligned_inputs, W: int,
                         workspace: int, workspace_bytes: int, stream: int) -> cphifi_solve_info:
    info = cphifi_solve_info()
    st = _lib.cphifi_aligned_solve(C.byref(desc), C.byref(inputs), C.c_void_p(W),
                                   C.c_void_p(workspace), C.c_size_t(workspace_bytes),
                                   C.c_void_p(stream), C.byref(info))
    _check(st, "cphifi_aligned_solve", soft_ok=True)
    return info


def make_als_desc(n, q: int, r: int, lams, rho: float, tol: float, als_tol: float,
                  max_outer: int, maxit: int = 0, precision: int = 0,
                  flags: int = 0, finite=(False, False, False)) -> cphifi_als_desc:
    d = cphifi_als_desc()
    for k in range(3):
        d.n[k], d.lambda_[k], d.finite[k] = int(n[k]), float(lams[k]), int(bool(finite[k]))
    d.q, d.r, d.rho, d.tol, d.als_tol = q, r, rho, tol, als_tol
    d.precision, d.flags, d.maxit, d.max_outer = precision, flags, maxit, max_outer
    return d


def cphifi_als_workspace_bytes(desc: cphifi_als_desc) -> int:
    out = C.c_size_t(0)
    _check(_lib.cphifi_als_workspace_bytes(C.byref(desc), C.byref(out)),
           "cphifi_als_workspace_bytes")
    return int(out.value)


def cphifi_als_create(desc: cphifi_als_desc, inputs: cphifi_als_inputs, workspace: int,
                      workspace_bytes: int, stream: int) -> int:
    h = C.c_void_p()
    _check(_lib.cphifi_als_create(C.byref(h), C.byref(desc), C.byref(inputs),
                                  C.c_void_p(workspace), C.c_size_t(workspace_bytes),
                                  C.c_void_p(stream)), "cphifi_als_create")
    return h.value


def cphifi_als_run(handle: int, W_ptrs, F_ptrs=None, errors_ptr: int = 0) -> cphifi_als_info:
    info = cphifi_als_info()
    info.errors = errors_ptr or None
    W = (C.c_void_p * 3)(*[int(p) for p in W_ptrs])
    F = None if F_ptrs is None else (C.c_void_p * 3)(*[int(p) for p in F_ptrs])
    _check(_lib.cphifi_als_run(C.c_void_p(handle), W, F, C.byref(info)), "cphifi_als_run")
    return info


def cphifi_als_destroy(handle: int) -> None:
    if handle:
        _check(_lib.cphifi_als_destroy(C.c_void_p(handle)), "cphifi_als_destroy")


ELT_F64 = 0
ELT_F32 = 1
ELT_BF16 = 2
ELT_BF16_TILED = 3  # BF16 U in the 16 x 64 tile layout of the solver's copies


def cphifi_product_workspace_bytes(n: int, r: int, elt: int) -> int:
    out = C.c_size_t(0)
    _check(_lib.cphifi_product_workspace_bytes(n, r, elt, C.byref(out)),
           "cphifi_product_workspace_bytes")
    return int(out.value)


def cphifi_product_tile_ok(elt: int, mw: int, s: int) -> bool:
    return bool(_lib.cphifi_product_tile_ok(elt, mw, s))


def cphifi_product(elt: int, trans: int, mw: int, s: int, ksplit: int, n: int, U: int, ldu: int,
                   X: int, r: int, xscale: Optional[int], Y: int, workspace: int,
                   workspace_bytes: int, stream: int) -> None:
    _check(_lib.cphifi_product(elt, trans, mw, s, ksplit, n, C.c_void_p(U), ldu, C.c_void_p(X),
                               r, C.c_void_p(xscale) if xscale else None, C.c_void_p(Y),
                               C.c_void_p(workspace), C.c_size_t(workspace_bytes),
                               C.c_void_p(stream)), "cphifi_product")


def cphifi_stream_read(buf: int, nbytes: int, blocks: int, partial: int, stream: int = 0) -> None:
    _check(_lib.cphifi_stream_read(C.c_void_p(buf), nbytes, blocks, C.c_void_p(partial),
                                   C.c_void_p(stream)), "cphifi_stream_read")


def cphifi_product_static_max_bytes() -> int:
    return int(_lib.cphifi_product_static_max_bytes())


def cphifi_product_static(elt: int, trans: int, mw: int, s: int, ksplit: int, n: int, U: int,
                          ldu: int, X: int, r: int, xscale: Optional[int], Y: int,
                          stream: int) -> None:
    _check(_lib.cphifi_product_static(elt, trans, mw, s, ksplit, n, C.c_void_p(U), ldu,
                                      C.c_void_p(X), r,
                                      C.c_void_p(xscale) if xscale else None, C.c_void_p(Y),
                                      C.c_void_p(stream)), "cphifi_product_static")


# ------------------------------------------------------------- batched solver
def _ptr_array(ptrs):
    arr = (C.c_void_p * len(ptrs))()
    for i, v in enumerate(ptrs):
        arr[i] = int(v)
    return arr


def cphifi_batch_workspace_bytes(descs) -> int:
    arr = (cphifi_ui_desc * len(descs))(*descs)
    out = C.c_size_t(0)
    _check(_lib.cphifi_batch_workspace_bytes(len(descs), arr, C.byref(out)),
           "cphifi_batch_workspace_bytes")
    return int(out.value)


def cphifi_batch_create(descs, inputs, workspace: int, workspace_bytes: int, stream: int,
                        tile_table: Optional[str] = None) -> int:
    darr = (cphifi_ui_desc * len(descs))(*descs)
    iarr = (cphifi_ui_inputs * len(inputs))(*inputs)
    bt = C.c_void_p(0)
    _check(_lib.cphifi_batch_create(C.byref(bt), len(descs), darr, iarr, C.c_void_p(workspace),
                                    C.c_size_t(workspace_bytes), C.c_void_p(stream),
                                    tile_table.encode() if tile_table else None),
           "cphifi_batch_create")
    return int(bt.value)


def cphifi_batch_plan(batch: int, member: int) -> int:
    out = C.c_void_p(0)
    _check(_lib.cphifi_batch_plan(C.c_void_p(batch), member, C.byref(out)), "cphifi_batch_plan")
    return int(out.value)


def cphifi_batch_rhs(batch: int, y_ptrs, b_ptrs) -> None:
    _check(_lib.cphifi_batch_rhs(C.c_void_p(batch), _ptr_array(y_ptrs), _ptr_array(b_ptrs)),
           "cphifi_batch_rhs")


def cphifi_batch_bind(batch: int, y_ptrs, W_ptrs) -> None:
    _check(_lib.cphifi_batch_bind(C.c_void_p(batch), _ptr_array(y_ptrs), _ptr_array(W_ptrs)),
           "cphifi_batch_bind")


def cphifi_batch_solve(batch: int, count: int, y_ptrs=None, W_ptrs=None, wait: bool = True):
    """Returns (status, [cphifi_solve_info]) when wait, else None (async launch)."""
    infos = (cphifi_solve_info * count)() if wait else None
    st = _lib.cphifi_batch_solve(C.c_void_p(batch),
                                 _ptr_array(y_ptrs) if y_ptrs is not None else None,
                                 _ptr_array(W_ptrs) if W_ptrs is not None else None, infos)
    if not wait:
        _check(st, "cphifi_batch_solve")
        return None
    if st not in (OK, NOT_CONVERGED, NUMERIC, BREAKDOWN):
        raise CphifiError(st, "cphifi_batch_solve", last_error())
    return st, list(infos)


def cphifi_batch_info(batch: int, count: int):
    infos = (cphifi_solve_info * count)()
    st = _lib.cphifi_batch_info(C.c_void_p(batch), infos)
    if st not in (OK, NOT_CONVERGED, NUMERIC, BREAKDOWN):
        raise CphifiError(st, "cphifi_batch_info", last_error())
    return st, list(infos)


def cphifi_batch_graph(batch: int) -> int:
    out = C.c_void_p(0)
    _check(_lib.cphifi_batch_graph(C.c_void_p(batch), C.byref(out)), "cphifi_batch_graph")
    return int(out.value)


def cphifi_batch_rounds(batch: int):
    rounds, grid = C.c_int(0), C.c_int(0)
    _check(_lib.cphifi_batch_rounds(C.c_void_p(batch), C.byref(rounds), C.byref(grid)),
           "cphifi_batch_rounds")
    return int(rounds.value), int(grid.value)


def cphifi_batch_destroy(batch: int) -> None:
    _check(_lib.cphifi_batch_destroy(C.c_void_p(batch)), "cphifi_batch_destroy")


BATCH_PHASES = ("products_a", "gather", "rows_split", "products_b", "finish",
                "update_precond", "precond_refine", "control", "round_setup")


def cphifi_batch_phase_ms(batch: int) -> dict:
    arr = (C.c_double * 9)()
    _check(_lib.cphifi_batch_phase_ms(C.c_void_p(batch), arr), "cphifi_batch_phase_ms")
    return dict(zip(BATCH_PHASES, list(arr)))
