"""CP-HIFI alternating optimisation on the host (Section 2, eq.
cp-hifi-subproblem; the outer loop of the experiments of Section 5).

TEST INFRASTRUCTURE ONLY, like the rest of this package: imported by tests,
never by the library.

The tensor is 3-way.  An infinite-dimensional mode k (every mode of the
paper's vortex and Miranda experiments) has its own kernel matrix K_k and its
factor is A_k = K_k W_k (Section 2); with the other two factors fixed, W_k
solves the unaligned subproblem of eq. unaligned-infinite-1: its observations
are grouped by their mode-k index, and the Khatri-Rao row of an observation is
the Hadamard product of the other two factors' rows at its indices.  A
finite-dimensional mode (K_k given as None) has no regulariser (Section 2), so
its block is CP-ALS with missing data: each row a_i of A_k = W_k solves the
least-squares problem over its observations, with the shift rho I added to
the normal equations (a row with few observations stays definite).  One outer
iteration updates modes 0, 1, 2 in turn; the loop ends when the relative error
on the observed entries changes by less than ``als_tol`` between two outer
iterations, or after ``max_outer`` of them (Section 5: 50 and 1e-6).

Functions with no independent pin: none (tests/test_oracle_als_pins.py checks the
model values by loops, the monotone decrease of the full objective under exact
block updates, and the stationarity of each block right after its update).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np

from .cphifi_oracle import (gram_V, kernel_eig, khatri_rao_rows, solve_dense,  # noqa: F401
                            solve_pcg)

__all__ = ["cp_values", "als_rel_error", "als_objective", "finite_mode_update", "mode_view",
           "AlsResult", "cp_hifi_als"]


def cp_values(factors: Sequence[np.ndarray], coords: np.ndarray) -> np.ndarray:
    """Model entries at the observed coordinates: sum over c of the product over
    modes k of A_k(i_k, c) (the CP model of Section 2)."""
    prod = np.ones((coords.shape[0], factors[0].shape[1]))
    for k, A in enumerate(factors):
        prod = prod * A[coords[:, k]]
    return prod.sum(axis=1)


def als_rel_error(factors: Sequence[np.ndarray], coords: np.ndarray, y: np.ndarray) -> float:
    """||y - model||_Omega / ||y||_Omega (the error the outer loop monitors)."""
    return float(np.linalg.norm(y - cp_values(factors, coords)) / np.linalg.norm(y))


def als_objective(Ks: Sequence[np.ndarray], Ws: Sequence[np.ndarray], coords: np.ndarray,
                  y: np.ndarray, lams: Sequence[float], rho: float) -> float:
    """The function the block updates decrease: the misfit on the observed
    entries plus, per mode, lam_k tr(W_k^T K_k W_k) + rho ||W_k||_F^2 (the
    regulariser of Section 2 and the shift of Section 4.1); a finite mode
    (K None) contributes rho ||W_k||_F^2 only."""
    factors = [W if K is None else K @ W for K, W in zip(Ks, Ws)]
    misfit = float(np.sum((y - cp_values(factors, coords)) ** 2))
    reg = sum((0.0 if K is None else lam * float(np.trace(W.T @ K @ W)))
              + rho * float(np.sum(W * W)) for K, W, lam in zip(Ks, Ws, lams))
    return misfit + reg


def finite_mode_update(coords: np.ndarray, y: np.ndarray, factors: Sequence[np.ndarray],
                       k: int, n_k: int, rho: float) -> np.ndarray:
    """CP-ALS block of a finite mode with missing data: for every row i,
    (Z_i^T Z_i + rho I) a_i = Z_i^T y_i with Z_i the Khatri-Rao rows of the
    observations whose mode-k index is i."""
    t, i, j, a, b = mode_view(coords, k)
    Z = khatri_rao_rows(factors[a], factors[b], i, j)
    r = Z.shape[1]
    W = np.zeros((n_k, r))
    for row in range(n_k):
        sel = t == row
        Zi, yi = Z[sel], y[sel]
        W[row] = np.linalg.solve(Zi.T @ Zi + rho * np.eye(r), Zi.T @ yi)
    return W


def mode_view(coords: np.ndarray, k: int):
    """Mode k's subproblem indices: (t, i, j, a, b) with t the mode-k index of
    every observation and i, j its indices in the other modes a < b."""
    a, b = [m for m in range(coords.shape[1]) if m != k]
    return coords[:, k], coords[:, a], coords[:, b], a, b


@dataclass
class AlsResult:
    Ws: List[np.ndarray]
    factors: List[np.ndarray]
    errors: List[float]                      # relative error before / after each outer iteration
    outer: int                               # outer iterations run
    inner_iters: List[List[int]] = field(default_factory=list)  # PCG iterations per mode update
    objectives: List[float] = field(default_factory=list)       # after every block update


def cp_hifi_als(Ks: Sequence[np.ndarray], coords: np.ndarray, y: np.ndarray,
                W0s: Sequence[np.ndarray], lams: Sequence[float], rho: float,
                max_outer: int = 50, als_tol: float = 1e-6, solver: str = "dense",
                tol: float = 1e-6, maxit: int = 75, eigs: Optional[Sequence] = None,
                track_objective: bool = False,
                on_block: Optional[Callable[[int, int, List[np.ndarray]], None]] = None
                ) -> AlsResult:
    """CP-HIFI alternating optimisation with every mode infinite-dimensional.

    solver="dense": each block update is the exact minimiser (O-dense).
    solver="pcg": the method of Section 4.4 (O-pcg) with relative-residual
    tolerance ``tol``, at most ``maxit`` iterations, warm-started from the
    block's current W (as the outer loop of Section 5 runs it).
    on_block(outer, k, Ws), when given, sees the weights after every block
    update.
    """
    d = len(Ks)
    if d != 3 or coords.shape[1] != 3:
        raise ValueError("3-way tensors only")
    Ws = [np.array(W, dtype=np.float64, copy=True) for W in W0s]
    factors = [W if K is None else K @ W for K, W in zip(Ks, Ws)]
    errors = [als_rel_error(factors, coords, y)]
    if eigs is None and solver == "pcg":
        eigs = [None if K is None else kernel_eig(K) for K in Ks]
    q = coords.shape[0]
    inner: List[List[int]] = []
    objs: List[float] = []
    outer = 0
    for _ in range(max_outer):
        its = []
        for k in range(d):
            t, i, j, a, b = mode_view(coords, k)
            Zhat = khatri_rao_rows(factors[a], factors[b], i, j)
            if Ks[k] is None:
                Ws[k] = finite_mode_update(coords, y, factors, k, Ws[k].shape[0], rho)
                its.append(0)
            elif solver == "dense":
                Ws[k] = solve_dense(Ks[k], Zhat, t, y, lams[k], rho)
                its.append(0)
            elif solver == "pcg":
                n_k, n_a, n_b = Ks[k].shape[0], Ws[a].shape[0], Ws[b].shape[0]
                gamma = q / (n_k * n_a * n_b)
                V = gram_V(factors[a], factors[b])
                res = solve_pcg(Ks[k], Zhat, t, y, lams[k], rho, gamma, V, tol, maxit,
                                eigK=eigs[k], X0=Ws[k])
                Ws[k] = res.X
                its.append(res.iters)
            else:
                raise ValueError(f"unknown solver {solver!r}")
            factors[k] = Ws[k] if Ks[k] is None else Ks[k] @ Ws[k]
            if on_block is not None:
                on_block(outer, k, Ws)
            if track_objective:
                objs.append(als_objective(Ks, Ws, coords, y, lams, rho))
        inner.append(its)
        outer += 1
        errors.append(als_rel_error(factors, coords, y))
        if abs(errors[-2] - errors[-1]) < als_tol:
            break
    return AlsResult(Ws, factors, errors, outer, inner, objs)
