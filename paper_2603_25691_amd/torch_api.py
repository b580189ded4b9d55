"""Torch-tensor convenience layer over the C ABI (argument marshalling only).

torch supplies device memory and the current HIP stream; every computation is
a call into libcphifi.so.  Inputs must already be CUDA (HIP) tensors of the
documented dtype and layout; nothing is converted or computed here.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import torch

from . import cphifi as _c


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _need(t: torch.Tensor, dtype, shape, name: str):
    if not t.is_cuda or t.dtype != dtype or tuple(t.shape) != tuple(shape) or \
            not t.is_contiguous():
        raise ValueError(f"{name}: expected contiguous device {dtype} of shape {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


def kernel_eig(K: torch.Tensor, method: str = "divide_conquer", tol: float = 1e-14,
               max_sweeps: int = 30):
    """One-time eigendecomposition of K on the device (library call).

    K: (n, ldk) storage with ldk >= n (row stride ldk).  Returns (UK, dK) with
    UK of the same storage shape holding eigenvector k in row k (the LAPACK
    column-major order the ABI expects) and dK ascending.  method:
    "divide_conquer" (cphifi_kernel_eig) or "jacobi" (cphifi_kernel_eig_jacobi;
    the sweep count is kept in kernel_eig.last_sweeps).
    """
    n, ldk = K.shape[0], K.shape[1]
    if ldk < n:
        raise ValueError("K: row stride below n")
    _need(K, torch.float64, (n, ldk), "K")
    UK = torch.empty_like(K)
    dK = torch.empty(n, dtype=torch.float64, device=K.device)
    if method == "jacobi":
        kernel_eig.last_sweeps = _c.cphifi_kernel_eig_jacobi(
            n, K.data_ptr(), ldk, UK.data_ptr(), dK.data_ptr(), tol, max_sweeps, _stream())
    elif method == "divide_conquer":
        _c.cphifi_kernel_eig(n, K.data_ptr(), ldk, UK.data_ptr(), dK.data_ptr(), _stream())
    else:
        raise ValueError(f"unknown eigensolver {method!r}")
    return UK, dK


def _ldk(prob) -> int:
    return prob.K.shape[1]


@dataclass
class DeviceProblem:
    n: int
    r: int
    q: int
    I: int
    J: int
    K: torch.Tensor
    UK: torch.Tensor
    dK: torch.Tensor
    obs_ptr: torch.Tensor
    obs_i: torch.Tensor
    obs_j: torch.Tensor
    y: torch.Tensor
    A: Optional[torch.Tensor] = None
    B: Optional[torch.Tensor] = None
    Zhat: Optional[torch.Tensor] = None
    V: Optional[torch.Tensor] = None


class UISolver:
    """A plan plus its workspace; methods mirror the C ABI calls."""

    def __init__(self, prob: DeviceProblem, lam: float, rho: float, tol: float,
                 precision: str = "fp64", gamma: float = 0.0, flags: int = 0, maxit: int = 0,
                 max_refine: int = 0, inner_tol: float = 0.0, check_every: int = 0):
        self.prob = prob
        n, r, q = prob.n, prob.r, prob.q
        _need(prob.K, torch.float64, (n, _ldk(prob)), "K")
        _need(prob.UK, torch.float64, (n, _ldk(prob)), "UK")
        _need(prob.dK, torch.float64, (n,), "dK")
        _need(prob.obs_ptr, torch.int32, (n + 1,), "obs_ptr")
        _need(prob.y, torch.float64, (q,), "y")
        if prob.Zhat is None:
            _need(prob.A, torch.float64, (prob.I, r), "A")
            _need(prob.B, torch.float64, (prob.J, r), "B")
            _need(prob.obs_i, torch.int32, (q,), "obs_i")
            _need(prob.obs_j, torch.int32, (q,), "obs_j")
        else:
            _need(prob.Zhat, torch.float64, (q, r), "Zhat")
        if prob.V is not None:
            _need(prob.V, torch.float64, (r, r), "V")
        self.desc = _c.make_desc(n, r, q, prob.I, prob.J, lam, rho, gamma, tol,
                                 _c.PRECISIONS[precision], flags, maxit, max_refine, inner_tol,
                                 check_every, ldk=_ldk(prob))
        self.inputs = _c.make_inputs(K=_ptr(prob.K), UK=_ptr(prob.UK), dK=_ptr(prob.dK),
                                     obs_ptr=_ptr(prob.obs_ptr), obs_i=_ptr(prob.obs_i),
                                     obs_j=_ptr(prob.obs_j), A=_ptr(prob.A), B=_ptr(prob.B),
                                     Zhat=_ptr(prob.Zhat), V=_ptr(prob.V))
        self.ws_bytes = _c.cphifi_ui_workspace_bytes(self.desc)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8,
                                     device=prob.K.device)
        base = self.workspace.data_ptr()
        self._ws = (base + 255) // 256 * 256
        self.plan = _c.cphifi_ui_plan_create(self.desc, self.inputs, self._ws, self.ws_bytes,
                                             _stream())

    def _vec(self):
        return torch.empty(self.prob.n, self.prob.r, dtype=torch.float64,
                           device=self.prob.K.device)

    def setup(self):
        _c.cphifi_ui_setup(self.plan)

    def rhs(self, y: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None):
        y = self.prob.y if y is None else y
        out = self._vec() if out is None else out
        _c.cphifi_ui_rhs(self.plan, y.data_ptr(), out.data_ptr())
        return out

    def mttkrp(self, y: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None):
        y = self.prob.y if y is None else y
        out = self._vec() if out is None else out
        _c.cphifi_ui_mttkrp(self.plan, y.data_ptr(), out.data_ptr())
        return out

    def apply(self, x: torch.Tensor, out: Optional[torch.Tensor] = None):
        out = self._vec() if out is None else out
        _c.cphifi_ui_apply(self.plan, x.data_ptr(), out.data_ptr())
        return out

    def precond(self, x: torch.Tensor, out: Optional[torch.Tensor] = None):
        out = self._vec() if out is None else out
        _c.cphifi_ui_precond(self.plan, x.data_ptr(), out.data_ptr())
        return out

    def apply_lowp(self, xbar: torch.Tensor, out: Optional[torch.Tensor] = None):
        out = self._vec() if out is None else out
        _c.cphifi_ui_apply_lowp(self.plan, xbar.data_ptr(), out.data_ptr())
        return out

    def solve(self, b: torch.Tensor, W: Optional[torch.Tensor] = None, history=None):
        W = self._vec() if W is None else W
        info = _c.cphifi_ui_solve(self.plan, b.data_ptr(), W.data_ptr(), history)
        return W, info

    def solve_subproblem(self, y: Optional[torch.Tensor] = None,
                         W: Optional[torch.Tensor] = None, history=None):
        y = self.prob.y if y is None else y
        W = self._vec() if W is None else W
        info = _c.cphifi_ui_solve_subproblem(self.plan, y.data_ptr(), W.data_ptr(), history)
        return W, info

    def close(self):
        if getattr(self, "plan", 0):
            _c.cphifi_ui_plan_destroy(self.plan)
            self.plan = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AlignedSolver:
    """The aligned subproblem of Section 3 (cphifi_aligned_solve): the
    decoupled direct solve or PCG on the transformed system, from U_K, d_K of
    prob and a right-hand side Bm = T Z (n x r).  V = Z^T Z is formed on the
    device from prob's factors when with_factors, else passed from the
    host-side Gram given as V (a device tensor) or computed by the caller."""

    def __init__(self, prob: DeviceProblem, lam: float, method: str = "decoupled",
                 tol: float = 0.0, maxit: int = 0, V: Optional[torch.Tensor] = None,
                 with_factors: bool = True):
        self.prob = prob
        n, r = prob.n, prob.r
        _need(prob.UK, torch.float64, (n, _ldk(prob)), "UK")
        _need(prob.dK, torch.float64, (n,), "dK")
        if V is not None:
            _need(V, torch.float64, (r, r), "V")
            with_factors = False
        self.V = V
        self.desc = _c.make_aligned_desc(n, r, lam, _c.ALIGNED_METHODS[method], tol, maxit,
                                         ldk=_ldk(prob))
        self.inputs = _c.cphifi_aligned_inputs()
        self.inputs.UK, self.inputs.dK = prob.UK.data_ptr(), prob.dK.data_ptr()
        if V is not None:
            self.inputs.V = V.data_ptr()
        else:
            _need(prob.A, torch.float64, (prob.I, r), "A")
            _need(prob.B, torch.float64, (prob.J, r), "B")
            self.inputs.A, self.inputs.B = prob.A.data_ptr(), prob.B.data_ptr()
            self.inputs.I, self.inputs.J = prob.I, prob.J
        self.ws_bytes = _c.cphifi_aligned_workspace_bytes(self.desc)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8,
                                     device=prob.UK.device)
        self._ws = (self.workspace.data_ptr() + 255) // 256 * 256

    def solve(self, Bm: torch.Tensor, W: Optional[torch.Tensor] = None):
        n, r = self.prob.n, self.prob.r
        _need(Bm, torch.float64, (n, r), "Bm")
        W = torch.empty(n, r, dtype=torch.float64, device=Bm.device) if W is None else W
        self.inputs.Bm = Bm.data_ptr()
        info = _c.cphifi_aligned_solve(self.desc, self.inputs, W.data_ptr(), self._ws,
                                       self.ws_bytes, _stream())
        return W, info

    def close(self):
        self.workspace = None


class BatchSolver:
    """Many subproblems solved by one persistent, graph-captured launch
    (cphifi_batch_*).  probs: DeviceProblems in the implicit (A, B) form;
    per-member parameters are given as scalars or lists."""

    def __init__(self, probs, lam, rho, tol, inner_tol: float = 0.0, maxit: int = 0,
                 max_refine: int = 0, flags: int = 0, tile_table: Optional[str] = None):
        self.probs = list(probs)
        m = len(self.probs)

        def per(v):
            return list(v) if isinstance(v, (list, tuple)) else [v] * m
        lam, rho, tol, inner_tol = per(lam), per(rho), per(tol), per(inner_tol)
        maxit, max_refine, flags = per(maxit), per(max_refine), per(flags)
        self.descs, self.inputs = [], []
        for k, pr in enumerate(self.probs):
            n, r, q = pr.n, pr.r, pr.q
            _need(pr.K, torch.float64, (n, _ldk(pr)), "K")
            _need(pr.UK, torch.float64, (n, _ldk(pr)), "UK")
            _need(pr.dK, torch.float64, (n,), "dK")
            _need(pr.obs_ptr, torch.int32, (n + 1,), "obs_ptr")
            _need(pr.A, torch.float64, (pr.I, r), "A")
            _need(pr.B, torch.float64, (pr.J, r), "B")
            _need(pr.obs_i, torch.int32, (q,), "obs_i")
            _need(pr.obs_j, torch.int32, (q,), "obs_j")
            self.descs.append(_c.make_desc(n, r, q, pr.I, pr.J, lam[k], rho[k], 0.0, tol[k],
                                           _c.MIXED_BF16, flags[k], maxit[k], max_refine[k],
                                           inner_tol[k], ldk=_ldk(pr)))
            self.inputs.append(_c.make_inputs(K=_ptr(pr.K), UK=_ptr(pr.UK), dK=_ptr(pr.dK),
                                              obs_ptr=_ptr(pr.obs_ptr), obs_i=_ptr(pr.obs_i),
                                              obs_j=_ptr(pr.obs_j), A=_ptr(pr.A),
                                              B=_ptr(pr.B)))
        self.ws_bytes = _c.cphifi_batch_workspace_bytes(self.descs)
        dev = self.probs[0].K.device
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        self._ws = (self.workspace.data_ptr() + 255) // 256 * 256
        self.batch = _c.cphifi_batch_create(self.descs, self.inputs, self._ws, self.ws_bytes,
                                            _stream(), tile_table)

    def plan(self, k: int) -> int:
        return _c.cphifi_batch_plan(self.batch, k)

    def rhs(self):
        bs = [torch.empty(p.n, p.r, dtype=torch.float64, device=p.K.device) for p in self.probs]
        _c.cphifi_batch_rhs(self.batch, [p.y.data_ptr() for p in self.probs],
                            [b.data_ptr() for b in bs])
        return bs

    def ys(self):
        """The members' observed values (the batched solve starts from them)."""
        return [p.y for p in self.probs]

    def _check_bound(self, ys, Ws):
        # the C ABI takes raw pointers: the shapes are checked here
        if len(ys) != len(self.probs) or len(Ws) != len(self.probs):
            raise ValueError("one observed-value vector and one W per member")
        for k, (pr, y, W) in enumerate(zip(self.probs, ys, Ws)):
            _need(y, torch.float64, (pr.q,), f"y[{k}]")
            _need(W, torch.float64, (pr.n, pr.r), f"W[{k}]")

    def bind(self, ys, Ws):
        """Bind each member's observed values ys[k] (device, q_k doubles) and
        its output Ws[k] (n_k x r_k)."""
        self._check_bound(ys, Ws)
        _c.cphifi_batch_bind(self.batch, [y.data_ptr() for y in ys], [W.data_ptr() for W in Ws])

    def solve(self, ys=None, Ws=None, wait: bool = True):
        """Solve every member from its observed values ys (device q_i doubles)
        into Ws (n_i x r_i).  Returns (status, infos) when wait, else None."""
        if ys is not None and Ws is not None:
            self._check_bound(ys, Ws)
        return _c.cphifi_batch_solve(self.batch, len(self.probs),
                                     None if ys is None else [y.data_ptr() for y in ys],
                                     None if Ws is None else [W.data_ptr() for W in Ws], wait)

    def info(self):
        return _c.cphifi_batch_info(self.batch, len(self.probs))

    def graph(self) -> int:
        return _c.cphifi_batch_graph(self.batch)

    def rounds(self):
        return _c.cphifi_batch_rounds(self.batch)

    def phase_ms(self):
        return _c.cphifi_batch_phase_ms(self.batch)

    def close(self):
        if getattr(self, "batch", 0):
            _c.cphifi_batch_destroy(self.batch)
            self.batch = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def upload(p, device="cuda", explicit=None, eig=None, ldk_align: int = 1) -> DeviceProblem:
    """Copy a synth.Problem's arrays to the device (host-to-device copies only).

    explicit: optional (Zhat, V) host arrays for the explicit per-observation
    form; otherwise the implicit (A, B) form is used.  eig: optional host
    (UK, dK) in the ABI's layout; by default the library computes the
    eigendecomposition of K on the device.  ldk_align: K and U_K are stored
    with row stride round_up(n, ldk_align) (an even stride keeps every row
    16-byte aligned for the FP64 products' vector loads).
    """
    import numpy as np

    def dev(a, dtype):
        return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dtype)

    ldk = (p.n + ldk_align - 1) // ldk_align * ldk_align
    if ldk == p.n:
        K = dev(p.K, torch.float64)
    else:
        K = torch.zeros(p.n, ldk, dtype=torch.float64, device=device)
        K[:, :p.n] = dev(p.K, torch.float64)
    if eig is not None:
        if ldk != p.n:
            raise ValueError("eig= takes the unpadded layout")
        UK = dev(eig[0], torch.float64)
        dK = dev(eig[1], torch.float64)
    else:
        UK, dK = kernel_eig(K)
    obs_ptr = dev(p.obs_ptr, torch.int32)
    obs_i = dev(p.obs_i, torch.int32)
    obs_j = dev(p.obs_j, torch.int32)
    y = dev(p.y, torch.float64)
    if explicit is not None:
        return DeviceProblem(p.n, p.r, p.q, p.I, p.J, K, UK, dK, obs_ptr, obs_i, obs_j, y,
                             Zhat=dev(explicit[0], torch.float64),
                             V=dev(explicit[1], torch.float64))
    A = dev(p.A, torch.float64)
    B = dev(p.B, torch.float64)
    return DeviceProblem(p.n, p.r, p.q, p.I, p.J, K, UK, dK, obs_ptr, obs_i, obs_j, y, A=A, B=B)


def bf16_tiles(Ub: torch.Tensor) -> torch.Tensor:
    """The 16 x 64 tile layout of a row-major bfloat16 matrix (n rows, row
    stride a multiple of 64, zero-padded columns): 16-row x 64-column tiles,
    each row-major, the column tiles of a row block consecutive.  Returned as a
    (round_up(n, 16), ld) tensor whose storage is that layout (so its stride(0)
    is the ldu the product takes); the padding rows are zero."""
    n, ld = Ub.shape
    if ld % 64 != 0:
        raise ValueError("bf16_tiles: the row stride must be a multiple of 64")
    rows = (n + 15) // 16 * 16
    P = torch.zeros(rows, ld, dtype=Ub.dtype, device=Ub.device)
    P[:n] = Ub
    return P.view(rows // 16, 16, ld // 64, 64).permute(0, 2, 1, 3).contiguous().view(rows, ld)


def product(U: torch.Tensor, X: torch.Tensor, elt: str = "fp64", trans: bool = False,
            tile=(0, 0), ksplit: int = 0, xscale: Optional[torch.Tensor] = None,
            out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None):
    """Y = op(U) diag(xscale) X through cphifi_product (U already in the element
    type's storage: float64, float32, bfloat16 zero-padded to a row stride
    that is a multiple of 8 and >= round_up(n, 128), or for "bf16_tiled" the
    output of bf16_tiles)."""
    e = {"fp64": _c.ELT_F64, "fp32": _c.ELT_F32, "bf16": _c.ELT_BF16,
         "bf16_tiled": _c.ELT_BF16_TILED}[elt]
    n, r = X.shape
    mw, s = tile
    if mw == 0:  # the solver's default tiles
        if e in (_c.ELT_BF16, _c.ELT_BF16_TILED):
            mw, s = 4, 2
        elif e == _c.ELT_F64:
            g4 = 2 * ((r + 7) // 8)
            if trans:
                mw, s = (4, 2) if g4 <= 10 else (2, 4) if g4 <= 14 else (1, 8)
            else:
                mw, s = (4, 4) if r <= 48 else (2, 4)
        else:
            mw, s = (4, 4) if trans or (n >= 4096 and r <= 48) else (2, 4)
    ws_bytes = _c.cphifi_product_workspace_bytes(n, r, e)
    if workspace is None or workspace.numel() < ws_bytes + 256:
        workspace = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=X.device)
    base = (workspace.data_ptr() + 255) // 256 * 256
    out = torch.empty(n, r, dtype=torch.float64, device=X.device) if out is None else out
    _c.cphifi_product(e, int(trans), mw, s, ksplit, n, U.data_ptr(), U.stride(0), X.data_ptr(),
                      r, None if xscale is None else xscale.data_ptr(), out.data_ptr(), base,
                      ws_bytes, _stream())
    return out


class AlsSolver:
    """CP-HIFI alternating optimisation over three RKHS modes (cphifi_als_*).

    Ks, UKs, dKs: per mode the kernel matrix (n_k x n_k), its eigenvectors (as
    kernel_eig returns them) and eigenvalues, device float64, or None for a
    finite-dimensional mode (then n[k] gives its size); coords: (q, 3) device
    int32; y: (q,) device float64."""

    def __init__(self, Ks, UKs, dKs, coords: torch.Tensor, y: torch.Tensor, r: int, lams,
                 rho: float, tol: float, als_tol: float, max_outer: int, maxit: int = 0,
                 precision: str = "fp64", flags: int = 0, n=None):
        finite = [K is None for K in Ks]
        n = [int(Ks[k].shape[0]) if not finite[k] else int(n[k]) for k in range(3)]
        for k in range(3):
            if finite[k]:
                continue
            _need(Ks[k], torch.float64, (n[k], n[k]), f"K[{k}]")
            _need(UKs[k], torch.float64, (n[k], n[k]), f"UK[{k}]")
            _need(dKs[k], torch.float64, (n[k],), f"dK[{k}]")
        q = int(y.shape[0])
        _need(coords, torch.int32, (q, 3), "coords")
        _need(y, torch.float64, (q,), "y")
        self.n, self.r, self.max_outer = n, r, max_outer
        self._keep = (list(Ks), list(UKs), list(dKs), coords, y)
        self.desc = _c.make_als_desc(n, q, r, lams, rho, tol, als_tol, max_outer, maxit,
                                     _c.PRECISIONS[precision], flags, finite)
        self.inputs = _c.cphifi_als_inputs()
        for k in range(3):
            if not finite[k]:
                self.inputs.K[k], self.inputs.UK[k] = Ks[k].data_ptr(), UKs[k].data_ptr()
                self.inputs.dK[k] = dKs[k].data_ptr()
        self.inputs.coords, self.inputs.y = coords.data_ptr(), y.data_ptr()
        self.ws_bytes = _c.cphifi_als_workspace_bytes(self.desc)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=y.device)
        ws = (self.workspace.data_ptr() + 255) // 256 * 256
        self.handle = _c.cphifi_als_create(self.desc, self.inputs, ws, self.ws_bytes,
                                           _stream())

    def run(self, W0s):
        """Returns (Ws, Fs, info, errors): the final weights and factors (device),
        the run's info and the relative error before / after each outer iteration."""
        Ws = []
        for k in range(3):
            _need(W0s[k], torch.float64, (self.n[k], self.r), f"W0[{k}]")
            Ws.append(W0s[k].clone())
        Fs = [torch.empty_like(W) for W in Ws]
        errors = (ctypes.c_double * (self.max_outer + 1))()
        info = _c.cphifi_als_run(self.handle, [W.data_ptr() for W in Ws],
                                 [F.data_ptr() for F in Fs], ctypes.addressof(errors))
        return Ws, Fs, info, list(errors)[: info.outer + 1]

    def close(self):
        _c.cphifi_als_destroy(self.handle)
        self.handle = None
        self.workspace = None
