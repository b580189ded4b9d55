"""Plain, slow, FP64 reference for the unaligned RKHS-mode CP-HIFI subproblem.

TEST INFRASTRUCTURE ONLY -- imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library.  Everything here is numpy /
scipy in float64 and follows the paper (Brust & Kolda, "Fast and Accurate
CP-HIFI Tensor Decompositions Exploiting Kronecker Structure") step by step.

Conventions
-----------
* ``W``, ``X``, ``B`` ... are logical n x r matrices (numpy arrays of shape
  (n, r)).  ``vec`` is the column-major vectorisation used throughout the paper
  (Appendix A, Kronecker identities): entry ``l*n + s`` of vec(X) is X[s, l].
* An observation l has time index ``obs_t[l]`` (the infinite mode's index
  i_k in the paper), and the indices ``obs_i[l]``, ``obs_j[l]`` of the two other
  modes.  ``Zhat`` is the q x r matrix of per-observation Khatri-Rao rows.

Readings of the paper used here (all listed with reasons in the design notes):
* rho is the extra Tikhonov shift of Section 4.1 (symmetric rho-regularised
  system); the objective it belongs to is the data misfit plus
  lambda * tr(W^T K W) plus rho * ||W||_F^2.
* gamma = q / (n I J) (density of the observed tensor, Section 4.4.2).
* V = Z^T Z with Z the Khatri-Rao product of the *full* other-mode factors
  (Section 4.4.2 reuses the aligned definition of Section 3), not the Gram of the
  observed rows.
* Eigenvalues of the psd K returned slightly negative by LAPACK are clamped to
  zero before the preconditioner's diagonal is formed.
* PCG is the standard preconditioned conjugate-gradient recurrence; it stops on
  the recursively updated residual ||r_k|| <= tol * ||b||.

Functions with no independent pin: none (every function below is exercised by
a pin in tests/test_oracle_pins.py).
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla

__all__ = [
    "vec", "unvec", "khatri_rao_rows", "khatri_rao", "forward_matrix",
    "mttkrp_observed", "mttkrp_full", "rhs_matrix", "system_matrix", "objective", "solve_dense",
    "solve_dense_with_error",
    "solve_lstsq", "gram_V", "matvec_twostep", "precond_matrix", "precond_diag",
    "precond_apply", "kernel_eig", "pcg", "PcgResult", "solve_pcg",
    "solve_aligned_full", "solve_decoupled", "solve_aligned_rho_kron",
    "solve_aligned_rho_kron_with_error", "solve_aligned_rho_decoupled",
    "aligned_matvec", "aligned_diag_precond", "solve_aligned_pcg",
    "e_kw", "e_fit", "e_w", "relres", "problem_arrays",
]


# ---------------------------------------------------------------------------
# Vectorisation and Khatri-Rao rows
# ---------------------------------------------------------------------------

def vec(X: np.ndarray) -> np.ndarray:
    """Column-major vec (Appendix A, eq. kronecker-identity)."""
    return np.asarray(X).reshape(-1, order="F")


def unvec(x: np.ndarray, n: int, r: int) -> np.ndarray:
    """Inverse of :func:`vec` for an n x r matrix."""
    return np.asarray(x).reshape((n, r), order="F")


def khatri_rao_rows(A: np.ndarray, B: np.ndarray, obs_i: np.ndarray,
                    obs_j: np.ndarray) -> np.ndarray:
    """Per-observation Khatri-Rao rows, eq. (zhat) for a 3-way tensor.

    Zhat(l, :) is the Hadamard product of the other modes' factor rows that
    observation l touches: A(i_l, :) * B(j_l, :).
    """
    return A[obs_i] * B[obs_j]


def khatri_rao(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Column-wise Kronecker (Khatri-Rao) product Z = B kr A, of size (J I) x r."""
    I, r = A.shape
    J = B.shape[0]
    return (B[:, None, :] * A[None, :, :]).reshape(J * I, r)


# ---------------------------------------------------------------------------
# The explicit system (Section 4.1 / 4.2)
# ---------------------------------------------------------------------------

def forward_matrix(K: np.ndarray, Zhat: np.ndarray, obs_t: np.ndarray) -> np.ndarray:
    """F of eq. (F): row l is Zhat(l,:) kron Khat(l,:), with Khat(l,:) = K(t_l,:).

    The row-wise Kronecker product puts Zhat(l, c) * K(t_l, s) in column
    c*n + s, matching the column-major vec of the n x r unknown.
    """
    q, r = Zhat.shape
    n = K.shape[0]
    Khat = K[obs_t]                                   # eq. (khat)
    return (Zhat[:, :, None] * Khat[:, None, :]).reshape(q, r * n)


def _segment_sum(idx: np.ndarray, vals: np.ndarray, n: int) -> np.ndarray:
    """out[s, :] = sum of vals[l, :] over l with idx[l] == s (column by column)."""
    out = np.zeros((n, vals.shape[1]))
    for c in range(vals.shape[1]):
        out[:, c] = np.bincount(idx, weights=vals[:, c], minlength=n)
    return out


def mttkrp_observed(y: np.ndarray, Zhat: np.ndarray, obs_t: np.ndarray,
                    n: int) -> np.ndarray:
    """B = T Z with T zero outside Omega (Section 4): B(s,:) = sum_{l: t_l=s} y_l Zhat(l,:)."""
    return _segment_sum(obs_t, y[:, None] * Zhat, n)


def mttkrp_full(Y: np.ndarray, A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """MTTKRP of a fully observed tensor (the aligned case of Section 3):
    B(s,:) = sum_{i,j} Y[s,i,j] A(i,:) * B(j,:), i.e. the mode-1 unfolding of
    Y times the Khatri-Rao product of the other two factors.  Y has shape
    (n, I, J); the contraction over j is one matrix product, the sum over i a
    weighted sum of rows."""
    n, I, J = Y.shape
    T = (Y.reshape(n * I, J) @ B).reshape(n, I, -1)   # T[s,i,:] = sum_j Y[s,i,j] B(j,:)
    return np.sum(T * A[None, :, :], axis=1)


def rhs_matrix(K: np.ndarray, Bm: np.ndarray) -> np.ndarray:
    """Right-hand side of eq. (unaligned-infinite-1): unvec(vec(K B)) = K B."""
    return K @ Bm


def system_matrix(F: np.ndarray, K: np.ndarray, lam: float, rho: float) -> np.ndarray:
    """Left-hand matrix of eq. (unaligned-infinite-1): F^T F + lam (I_r kron K) + rho I."""
    nr = F.shape[1]
    n = K.shape[0]
    r = nr // n
    return F.T @ F + lam * np.kron(np.eye(r), K) + rho * np.eye(nr)


def objective(K: np.ndarray, A: np.ndarray, B: np.ndarray, obs_t: np.ndarray,
              obs_i: np.ndarray, obs_j: np.ndarray, y: np.ndarray, lam: float,
              rho: float, W: np.ndarray) -> float:
    """The subproblem objective evaluated directly (Section 2, eq.
    unaligned-infinite-with-k, plus the rho shift of Section 4.1):

        sum_l (y_l - sum_c (K W)(t_l, c) A(i_l, c) B(j_l, c))^2
          + lam * tr(W^T K W) + rho * ||W||_F^2
    """
    KW = K @ W
    pred = np.sum(KW[obs_t] * A[obs_i] * B[obs_j], axis=1)
    misfit = np.sum((y - pred) ** 2)
    return float(misfit + lam * np.trace(W.T @ K @ W) + rho * np.sum(W * W))


def solve_dense(K: np.ndarray, Zhat: np.ndarray, obs_t: np.ndarray, y: np.ndarray,
                lam: float, rho: float) -> np.ndarray:
    """O-dense: form F, F^T F + lam(I kron K) + rho I and F^T y; Cholesky solve.

    Section 4.2 (symmetric direct solve).  Returns W (n x r).
    """
    n = K.shape[0]
    r = Zhat.shape[1]
    F = forward_matrix(K, Zhat, obs_t)
    H = system_matrix(F, K, lam, rho)
    rhs = F.T @ y
    c = sla.cho_factor(H, lower=True)
    return unvec(sla.cho_solve(c, rhs), n, r)


def solve_dense_with_error(K: np.ndarray, Zhat: np.ndarray, obs_t: np.ndarray,
                           y: np.ndarray, lam: float, rho: float):
    """O-dense plus an estimate of its own forward error in K W.

    Returns (W, delta) where W is the Cholesky solution of :func:`solve_dense`
    and delta = ||K D||_F / ||K W||_F for the FP64 iterative-refinement
    correction D = unvec(H^{-1}(F^T y - H w)).  For ill-conditioned instances
    delta is what limits any comparison against W."""
    n = K.shape[0]
    r = Zhat.shape[1]
    F = forward_matrix(K, Zhat, obs_t)
    H = system_matrix(F, K, lam, rho)
    rhs = F.T @ y
    c = sla.cho_factor(H, lower=True)
    w = sla.cho_solve(c, rhs)
    dw = sla.cho_solve(c, rhs - H @ w)
    W = unvec(w, n, r)
    delta = float(np.linalg.norm(K @ unvec(dw, n, r)) / np.linalg.norm(K @ W))
    return W, delta


def solve_lstsq(K: np.ndarray, Zhat: np.ndarray, obs_t: np.ndarray, y: np.ndarray,
                lam: float, rho: float) -> np.ndarray:
    """O-brute: minimise the objective as one stacked least-squares problem.

        || [F; sqrt(lam) (I_r kron K^{1/2}); sqrt(rho) I] w - [y; 0; 0] ||^2

    solved by an SVD-based least-squares routine, with K^{1/2} from the
    eigendecomposition of K (negative rounding eigenvalues clamped to zero).
    A different algorithm for the same minimiser as :func:`solve_dense`.
    """
    n = K.shape[0]
    r = Zhat.shape[1]
    F = forward_matrix(K, Zhat, obs_t)
    d, U = np.linalg.eigh(K)
    Khalf = (U * np.sqrt(np.maximum(d, 0.0))) @ U.T
    top = F
    mid = np.sqrt(lam) * np.kron(np.eye(r), Khalf)
    bot = np.sqrt(rho) * np.eye(n * r)
    G = np.vstack([top, mid, bot])
    rhs = np.concatenate([y, np.zeros(n * r), np.zeros(n * r)])
    w, *_ = sla.lstsq(G, rhs, lapack_driver="gelsd")
    return unvec(w, n, r)


# ---------------------------------------------------------------------------
# Matrix-free pieces of the PCG method (Section 4.4)
# ---------------------------------------------------------------------------

def gram_V(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """V := Z^T Z with Z the Khatri-Rao product of the other-mode factors
    (Section 3, reused by the preconditioner of Section 4.4.2)."""
    Z = khatri_rao(A, B)
    return Z.T @ Z


def matvec_twostep(K: np.ndarray, Zhat: np.ndarray, obs_t: np.ndarray, lam: float,
                   rho: float, X: np.ndarray) -> np.ndarray:
    """y = (F^T F + lam (I kron K) + rho I) x by the two-step product of Section 4.4.1.

    Xhat = K X; xbar_l = Xhat(t_l,:) . Zhat(l,:) (eq. vl);
    Yhat1(s,:) = sum_{l: t_l = s} xbar_l Zhat(l,:) (eq. yhat1);
    Y = K Yhat1 + lam Xhat + rho X.
    """
    Xhat = K @ X
    xbar = np.sum(Xhat[obs_t] * Zhat, axis=1)
    Yhat1 = _segment_sum(obs_t, xbar[:, None] * Zhat, X.shape[0])
    return K @ Yhat1 + lam * Xhat + rho * X


def precond_matrix(K: np.ndarray, V: np.ndarray, gamma: float, lam: float,
                   rho: float) -> np.ndarray:
    """Dense preconditioner of eq. (precon): gamma (V kron K^2) + lam (I kron K) + rho I."""
    n = K.shape[0]
    r = V.shape[0]
    return (gamma * np.kron(V, K @ K) + lam * np.kron(np.eye(r), K)
            + rho * np.eye(n * r))


def kernel_eig(K: np.ndarray):
    """eq. (eigK): K = U_K D_K U_K^T; eigenvalues clamped to be nonnegative."""
    d, U = np.linalg.eigh(K)
    return np.maximum(d, 0.0), U


def precond_diag(dK: np.ndarray, dV: np.ndarray, gamma: float, lam: float,
                 rho: float) -> np.ndarray:
    """D = unvec(1 / diag(gamma (D_V kron D_K^2) + lam (I kron D_K) + rho I)), n x r.

    Entry (s, c) of the diagonal is gamma dV_c dK_s^2 + lam dK_s + rho
    (Section 4.4.2)."""
    return 1.0 / (gamma * (dK[:, None] ** 2) * dV[None, :] + lam * dK[:, None] + rho)


def precond_apply(UK: np.ndarray, dK: np.ndarray, UV: np.ndarray, dV: np.ndarray,
                  gamma: float, lam: float, rho: float, X: np.ndarray) -> np.ndarray:
    """M^{-1} x of eq. (fx): U_K ((U_K^T X U_V) had D) U_V^T."""
    D = precond_diag(np.maximum(dK, 0.0), dV, gamma, lam, rho)
    return UK @ (((UK.T @ X) @ UV) * D) @ UV.T


@dataclass
class PcgResult:
    X: np.ndarray
    iters: int
    relres_hist: List[float]
    converged: bool


def _fro(X: np.ndarray, Y: np.ndarray) -> float:
    return float(np.sum(X * Y))


def pcg(apply_A: Callable[[np.ndarray], np.ndarray],
        apply_Minv: Callable[[np.ndarray], np.ndarray], Bm: np.ndarray, tol: float,
        maxit: int, X0: Optional[np.ndarray] = None) -> PcgResult:
    """Standard preconditioned conjugate gradients on n x r unknowns.

    The method of Section 4.4 applies textbook PCG (the Golub-Van Loan form)
    with the matrix-free product and eq. (fx); the inner product is the
    Frobenius one, i.e. the Euclidean inner product of the vec'ed unknowns.
    Stops when ||r_k|| <= tol ||b|| on the recursively updated residual.
    """
    X = np.zeros_like(Bm) if X0 is None else X0.copy()
    R = Bm - apply_A(X) if X0 is not None else Bm.copy()
    bnorm = np.sqrt(_fro(Bm, Bm))
    hist = [np.sqrt(_fro(R, R)) / bnorm if bnorm > 0 else 0.0]
    if bnorm == 0.0 or hist[0] <= tol:
        return PcgResult(X, 0, hist, True)
    Z = apply_Minv(R)
    P = Z.copy()
    rz = _fro(R, Z)
    for k in range(1, maxit + 1):
        Q = apply_A(P)
        alpha = rz / _fro(P, Q)
        X = X + alpha * P
        R = R - alpha * Q
        rel = np.sqrt(_fro(R, R)) / bnorm
        hist.append(rel)
        if rel <= tol:
            return PcgResult(X, k, hist, True)
        Z = apply_Minv(R)
        rz_new = _fro(R, Z)
        beta = rz_new / rz
        rz = rz_new
        P = Z + beta * P
    return PcgResult(X, maxit, hist, False)


def solve_pcg(K: np.ndarray, Zhat: np.ndarray, obs_t: np.ndarray, y: np.ndarray,
              lam: float, rho: float, gamma: float, V: np.ndarray, tol: float,
              maxit: int, eigK=None, X0: Optional[np.ndarray] = None,
              precondition: bool = True) -> PcgResult:
    """O-pcg: the method of Section 4.4 on the host.

    Right-hand side K B with B the observed MTTKRP, the two-step product, and
    the eq. (fx) preconditioner built from the eigendecompositions of K and V.
    ``precondition=False`` runs plain CG (the paper's "cg" comparison).
    """
    n = K.shape[0]
    Bm = mttkrp_observed(y, Zhat, obs_t, n)
    rhs = rhs_matrix(K, Bm)
    if eigK is None:
        eigK = kernel_eig(K)
    dK, UK = eigK
    dV, UV = np.linalg.eigh(V)

    def A_op(X):
        return matvec_twostep(K, Zhat, obs_t, lam, rho, X)

    if precondition:
        def M_op(X):
            return precond_apply(UK, dK, UV, dV, gamma, lam, rho, X)
    else:
        def M_op(X):
            return X.copy()
    return pcg(A_op, M_op, rhs, tol, maxit, X0)


# ---------------------------------------------------------------------------
# Aligned subproblem (Section 3)
# ---------------------------------------------------------------------------

def solve_aligned_full(K: np.ndarray, V: np.ndarray, Bm: np.ndarray,
                       lam: float) -> np.ndarray:
    """Section 3.1: Cholesky of (V kron K + lam I) vec(W) = vec(B) (eq. aligned-solve)."""
    n = K.shape[0]
    r = V.shape[0]
    H = np.kron(V, K) + lam * np.eye(n * r)
    c = sla.cho_factor(H, lower=True)
    return unvec(sla.cho_solve(c, vec(Bm)), n, r)


def solve_decoupled(UK: np.ndarray, dK: np.ndarray, UV: np.ndarray, dV: np.ndarray,
                    Bm: np.ndarray, lam: float) -> np.ndarray:
    """Section 3.2, eq. (W-decoupled): W = U_K ((U_K^T B U_V) had D) U_V^T,
    D(s, c) = 1 / (dV_c dK_s + lam)."""
    D = 1.0 / (dK[:, None] * dV[None, :] + lam)
    return UK @ (((UK.T @ Bm) @ UV) * D) @ UV.T


def solve_aligned_rho_kron(K: np.ndarray, V: np.ndarray, KB: np.ndarray, lam: float,
                           rho: float) -> np.ndarray:
    """O-kron: for a full observation set F^T F = V kron K^2, so the system of
    eq. (unaligned-infinite-1) is (V kron K^2 + lam I kron K + rho I) w = vec(K B);
    solved by Cholesky.  Valid only when every entry is observed."""
    n = K.shape[0]
    r = V.shape[0]
    H = np.kron(V, K @ K) + lam * np.kron(np.eye(r), K) + rho * np.eye(n * r)
    c = sla.cho_factor(H, lower=True)
    return unvec(sla.cho_solve(c, vec(KB)), n, r)


def solve_aligned_rho_kron_with_error(K: np.ndarray, V: np.ndarray, KB: np.ndarray,
                                      lam: float, rho: float):
    """O-kron plus an estimate of its own forward error in K W: (W, delta) with
    delta = ||K D|| / ||K W|| for the FP64 iterative-refinement correction
    D = unvec(H^{-1}(vec(K B) - H w)), H = V kron K^2 + lam I kron K + rho I."""
    n = K.shape[0]
    r = V.shape[0]
    H = np.kron(V, K @ K) + lam * np.kron(np.eye(r), K) + rho * np.eye(n * r)
    c = sla.cho_factor(H, lower=True)
    rhs = vec(KB)
    w = sla.cho_solve(c, rhs)
    dw = sla.cho_solve(c, rhs - H @ w)
    W = unvec(w, n, r)
    delta = float(np.linalg.norm(K @ unvec(dw, n, r)) / np.linalg.norm(K @ W))
    return W, delta


def solve_aligned_rho_decoupled(UK: np.ndarray, dK: np.ndarray, UV: np.ndarray,
                                dV: np.ndarray, KB: np.ndarray, lam: float,
                                rho: float) -> np.ndarray:
    """O-dec for the rho-system of a fully observed tensor: with
    F^T F = V kron K^2 the system matrix is diagonalised by U_V kron U_K (the
    step of Section 3.2 that gives eq. W-decoupled, applied to the system of
    eq. unaligned-infinite-1), so
    W = U_K ((U_K^T (K B) U_V) / (dK^2 dV^T + lam dK 1^T + rho)) U_V^T
    entrywise in the eigenbasis."""
    D = dK[:, None] ** 2 * dV[None, :] + lam * dK[:, None] + rho
    return UK @ (((UK.T @ KB) @ UV) / D) @ UV.T


def aligned_matvec(dK: np.ndarray, V: np.ndarray, lam: float, X: np.ndarray) -> np.ndarray:
    """eq. (pcg-matvec-ai): (V kron D_K + lam I) x = vec(D_K X V + lam X), X n x r."""
    return dK[:, None] * (X @ V) + lam * X


def aligned_diag_precond(dK: np.ndarray, V: np.ndarray, lam: float) -> np.ndarray:
    """Inverse diagonal of eq. (precond-ai): 1 / (diag(V)_c dK_s + lam), n x r."""
    return 1.0 / (np.diag(V)[None, :] * dK[:, None] + lam)


def solve_aligned_pcg(UK: np.ndarray, dK: np.ndarray, V: np.ndarray, Bm: np.ndarray,
                      lam: float, tol: float, maxit: int) -> PcgResult:
    """Section 3.3: PCG on (V kron D_K + lam I) vec(Wbar) = vec(U_K^T B), then W = U_K Wbar."""
    Bbar = UK.T @ Bm
    Dinv = aligned_diag_precond(dK, V, lam)
    res = pcg(lambda X: aligned_matvec(dK, V, lam, X), lambda X: Dinv * X, Bbar, tol,
              maxit)
    return PcgResult(UK @ res.X, res.iters, res.relres_hist, res.converged)


# ---------------------------------------------------------------------------
# Error measures
# ---------------------------------------------------------------------------

def e_kw(K: np.ndarray, W: np.ndarray, Wref: np.ndarray) -> float:
    """||K (W - Wref)||_F / ||K Wref||_F -- error of the RKHS factor K W."""
    return float(np.linalg.norm(K @ (W - Wref)) / np.linalg.norm(K @ Wref))


def e_fit(K: np.ndarray, Zhat: np.ndarray, obs_t: np.ndarray, W: np.ndarray,
          Wref: np.ndarray) -> float:
    """||F (w - wref)|| / ||F wref|| -- error of the fitted values at Omega."""
    KD = K @ (W - Wref)
    KR = K @ Wref
    num = np.sum(KD[obs_t] * Zhat, axis=1)
    den = np.sum(KR[obs_t] * Zhat, axis=1)
    return float(np.linalg.norm(num) / np.linalg.norm(den))


def e_w(W: np.ndarray, Wref: np.ndarray) -> float:
    return float(np.linalg.norm(W - Wref) / np.linalg.norm(Wref))


def relres(K: np.ndarray, Zhat: np.ndarray, obs_t: np.ndarray, y: np.ndarray,
           lam: float, rho: float, W: np.ndarray) -> float:
    """Residual certificate ||K B - A(W)||_F / ||K B||_F with the two-step product."""
    n = K.shape[0]
    rhs = rhs_matrix(K, mttkrp_observed(y, Zhat, obs_t, n))
    R = rhs - matvec_twostep(K, Zhat, obs_t, lam, rho, W)
    return float(np.linalg.norm(R) / np.linalg.norm(rhs))


def problem_arrays(p):
    """Convenience: (K, Zhat, obs_t, y, lam, rho, gamma, V) for a synth.Problem."""
    Zhat = khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    return p.K, Zhat, p.obs_t, p.y, p.lam, p.rho, p.gamma, gram_V(p.A, p.B)
