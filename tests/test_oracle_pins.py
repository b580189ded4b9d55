"""Pins of the CPU oracle against facts other than its own formulas.

Each test checks an oracle function against something the paper or the
mathematics fixes independently: the model as literally defined (loops), the
objective's stationarity, a different algorithm for the same minimiser,
Kronecker identities, textbook special cases and library routines.
"""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import oracle as O
from synth import config_c1, make_aligned, make_small


def _tiny(seed=3, n=6, I=3, J=2, r=2, q=20, lam=0.1, rho=1e-2, sigma=0.3):
    return make_small(seed, n=n, I=I, J=J, r=r, q=q, kernel="rbf", kernel_param=sigma,
                      lam=lam, rho=rho)


# ---------------------------------------------------------------- vec / F ----

def test_kronecker_vec_identity():
    """Appendix A: vec(A X C) = (C^T kron A) vec(X) with column-major vec."""
    rng = np.random.default_rng(0)
    A = rng.standard_normal((4, 3))
    X = rng.standard_normal((3, 5))
    C = rng.standard_normal((5, 2))
    lhs = O.vec(A @ X @ C)
    rhs = np.kron(C.T, A) @ O.vec(X)
    assert np.allclose(lhs, rhs, rtol=1e-13, atol=1e-13)
    assert np.array_equal(O.unvec(O.vec(X), 3, 5), X)


def test_forward_matrix_is_the_model_at_observed_entries():
    """F vec(W) must equal the CP model with time factor K W, evaluated entry by
    entry with plain loops (eq. unaligned-infinite-with-k, eq. F)."""
    p = _tiny()
    rng = np.random.default_rng(1)
    W = rng.standard_normal((p.n, p.r))
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    F = O.forward_matrix(p.K, Zhat, p.obs_t)
    got = F @ O.vec(W)
    want = []
    for l in range(p.q):
        acc = 0.0
        for c in range(p.r):
            kw = 0.0
            for s in range(p.n):
                kw += p.K[p.obs_t[l], s] * W[s, c]
            acc += kw * p.A[p.obs_i[l], c] * p.B[p.obs_j[l], c]
        want.append(acc)
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13)


def test_objective_matches_loops():
    p = _tiny()
    W = np.random.default_rng(2).standard_normal((p.n, p.r))
    got = O.objective(p.K, p.A, p.B, p.obs_t, p.obs_i, p.obs_j, p.y, p.lam, p.rho, W)
    KW = [[sum(p.K[a, s] * W[s, c] for s in range(p.n)) for c in range(p.r)]
          for a in range(p.n)]
    mis = 0.0
    for l in range(p.q):
        pred = sum(KW[p.obs_t[l]][c] * p.A[p.obs_i[l], c] * p.B[p.obs_j[l], c]
                   for c in range(p.r))
        mis += (p.y[l] - pred) ** 2
    reg = sum(W[a, c] * KW[a][c] for a in range(p.n) for c in range(p.r))
    shift = sum(W[a, c] ** 2 for a in range(p.n) for c in range(p.r))
    assert got == pytest.approx(mis + p.lam * reg + p.rho * shift, rel=1e-13)


def test_khatri_rao_gram_is_hadamard_of_grams():
    """V = Z^T Z = (A^T A) had (B^T B) for a Khatri-Rao Z; with every entry observed
    the observed-row Gram Zhat^T Zhat equals V."""
    rng = np.random.default_rng(4)
    A = rng.standard_normal((7, 3))
    B = rng.standard_normal((5, 3))
    V = O.gram_V(A, B)
    assert np.allclose(V, (A.T @ A) * (B.T @ B), rtol=1e-13)
    ii, jj = np.meshgrid(np.arange(7), np.arange(5), indexing="ij")
    Zh = O.khatri_rao_rows(A, B, ii.ravel(), jj.ravel())
    assert np.allclose(Zh.T @ Zh, V, rtol=1e-13)


# ------------------------------------------------------ normal equations ----

def test_dense_solution_is_stationary_point_of_objective():
    """The Cholesky solution must be a stationary point of the objective as
    written: f(W+E) - f(W-E) = 2 <grad f(W), E> = 0 for any E."""
    p = _tiny(q=25)
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    W = O.solve_dense(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho)
    rng = np.random.default_rng(5)
    f = lambda X: O.objective(p.K, p.A, p.B, p.obs_t, p.obs_i, p.obs_j, p.y,
                              p.lam, p.rho, X)
    for _ in range(4):
        E = rng.standard_normal(W.shape)
        E *= np.sqrt(f(W)) / np.linalg.norm(E)
        fp, fm, f0 = f(W + E), f(W - E), f(W)
        curv = fp + fm - 2 * f0
        assert curv > 0
        assert abs(fp - fm) <= 1e-9 * curv
    # a perturbed solution is not stationary (sanity of the test itself)
    W2 = W + 1e-3 * rng.standard_normal(W.shape)
    E = rng.standard_normal(W.shape)
    assert abs(f(W2 + E) - f(W2 - E)) > 1e-6 * (f(W2 + E) + f(W2 - E) - 2 * f(W2))


def test_lstsq_and_cholesky_agree():
    """Two different algorithms for the same minimiser agree in K W and fitted values."""
    p = _tiny(n=8, I=3, J=3, r=3, q=40, lam=1e-3, rho=1e-6, seed=11)
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    Wd = O.solve_dense(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho)
    Wl = O.solve_lstsq(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho)
    assert O.e_kw(p.K, Wl, Wd) < 1e-10
    assert O.e_fit(p.K, Zhat, p.obs_t, Wl, Wd) < 1e-10


def test_dense_error_estimate_tracks_conditioning():
    """The refinement-based error estimate is at rounding level for a well-
    conditioned system and grows with cond(H) (rho -> 0 makes H singular)."""
    p = _tiny(q=25, lam=1e-1, rho=1e-1)
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    W, d_good = O.solve_dense_with_error(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho)
    assert np.array_equal(W, O.solve_dense(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho))
    assert 0 <= d_good < 1e-14
    q = make_small(41, n=40, I=4, J=4, r=3, q=200, kernel_param=0.3, lam=1e-6, rho=1e-12)
    Zq = O.khatri_rao_rows(q.A, q.B, q.obs_i, q.obs_j)
    _, d_bad = O.solve_dense_with_error(q.K, Zq, q.obs_t, q.y, q.lam, q.rho)
    assert d_bad > 100 * d_good
    assert d_bad < 1e-3


def test_rhs_is_F_transpose_y():
    """F^T y = vec(K B) with B the observed MTTKRP (Section 4, eq. unaligned-infinite-1)."""
    p = _tiny(seed=7, q=30)
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    F = O.forward_matrix(p.K, Zhat, p.obs_t)
    Bm = O.mttkrp_observed(p.y, Zhat, p.obs_t, p.n)
    assert np.allclose(F.T @ p.y, O.vec(O.rhs_matrix(p.K, Bm)), rtol=1e-13, atol=1e-13)


# ------------------------------------------------------- two-step product ----

def test_twostep_product_equals_dense_system():
    """Section 4.4.1: the two-step product equals the explicit matrix times x."""
    p = _tiny(n=9, I=4, J=3, r=3, q=50, seed=8)
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    H = O.system_matrix(O.forward_matrix(p.K, Zhat, p.obs_t), p.K, p.lam, p.rho)
    X = np.random.default_rng(9).standard_normal((p.n, p.r))
    got = O.matvec_twostep(p.K, Zhat, p.obs_t, p.lam, p.rho, X)
    want = O.unvec(H @ O.vec(X), p.n, p.r)
    assert np.linalg.norm(got - want) <= 1e-14 * np.linalg.norm(want) * 10


def test_operator_symmetric_positive_definite():
    p = config_c1()
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    rng = np.random.default_rng(10)
    X = rng.standard_normal((p.n, p.r))
    Y = rng.standard_normal((p.n, p.r))
    AX = O.matvec_twostep(p.K, Zhat, p.obs_t, p.lam, p.rho, X)
    AY = O.matvec_twostep(p.K, Zhat, p.obs_t, p.lam, p.rho, Y)
    lhs, rhs = np.sum(AX * Y), np.sum(X * AY)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(AX) * np.linalg.norm(Y)
    assert np.sum(X * AX) >= p.rho * np.sum(X * X)


# ---------------------------------------------------------- preconditioner ----

def test_precond_apply_inverts_dense_preconditioner():
    """eq. (fx) is the inverse of eq. (precon) built with Kronecker products."""
    p = _tiny(n=7, I=3, J=4, r=3, q=30, seed=12)
    V = O.gram_V(p.A, p.B)
    M = O.precond_matrix(p.K, V, p.gamma, p.lam, p.rho)
    dK, UK = O.kernel_eig(p.K)
    dV, UV = np.linalg.eigh(V)
    X = np.random.default_rng(13).standard_normal((p.n, p.r))
    MX = O.unvec(M @ O.vec(X), p.n, p.r)
    back = O.precond_apply(UK, dK, UV, dV, p.gamma, p.lam, p.rho, MX)
    assert np.linalg.norm(back - X) <= 1e-8 * np.linalg.norm(X)
    # and against a direct dense solve with M
    Y = np.random.default_rng(14).standard_normal((p.n, p.r))
    direct = O.unvec(np.linalg.solve(M, O.vec(Y)), p.n, p.r)
    got = O.precond_apply(UK, dK, UV, dV, p.gamma, p.lam, p.rho, Y)
    assert np.linalg.norm(got - direct) <= 1e-8 * np.linalg.norm(direct)


def _aligned_tiny(seed=15, n=6, I=3, J=2, r=2, sigma=0.2, lam=0.05, rho=1e-3):
    return make_aligned(seed, I=I, J=J, n=n, r=r, sigma=sigma, lam=lam, rho=rho,
                        tol=1e-12)


def test_aligned_preconditioner_is_exact_and_pcg_takes_one_iteration():
    """With every entry observed, S S^T = I, gamma = 1 and M equals the system
    matrix, so PCG converges in a single iteration."""
    p = _aligned_tiny()
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    V = O.gram_V(p.A, p.B)
    H = O.system_matrix(O.forward_matrix(p.K, Zhat, p.obs_t), p.K, p.lam, p.rho)
    M = O.precond_matrix(p.K, V, 1.0, p.lam, p.rho)
    assert p.gamma == 1.0
    assert np.linalg.norm(H - M) <= 1e-13 * np.linalg.norm(H)
    res = O.solve_pcg(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho, p.gamma, V, 1e-10, 50)
    assert res.iters == 1


# ---------------------------------------------------------------- aligned ----

def test_aligned_full_solution_is_stationary():
    """Section 3: the solution of (V kron K + lam I) w = vec(B) minimises
    ||T - K W Z^T||_F^2 + lam tr(W^T K W) (rho = 0 objective), K nonsingular."""
    p = _aligned_tiny(n=5, sigma=0.15, lam=0.1)
    V = O.gram_V(p.A, p.B)
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    Bm = O.mttkrp_observed(p.y, Zhat, p.obs_t, p.n)
    W = O.solve_aligned_full(p.K, V, Bm, p.lam)
    f = lambda X: O.objective(p.K, p.A, p.B, p.obs_t, p.obs_i, p.obs_j, p.y, p.lam,
                              0.0, X)
    rng = np.random.default_rng(16)
    for _ in range(3):
        E = rng.standard_normal(W.shape)
        fp, fm, f0 = f(W + E), f(W - E), f(W)
        assert abs(fp - fm) <= 1e-9 * (fp + fm - 2 * f0)


def test_decoupled_equals_full_aligned_solve():
    """eq. (W-decoupled) equals the Cholesky solve of eq. (aligned-solve)."""
    p = _aligned_tiny(n=8, I=4, J=3, r=3)
    V = O.gram_V(p.A, p.B)
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    Bm = O.mttkrp_observed(p.y, Zhat, p.obs_t, p.n)
    Wf = O.solve_aligned_full(p.K, V, Bm, p.lam)
    dK, UK = np.linalg.eigh(p.K)
    dV, UV = np.linalg.eigh(V)
    Wd = O.solve_decoupled(UK, dK, UV, dV, Bm, p.lam)
    assert O.e_kw(p.K, Wd, Wf) < 1e-12


def test_aligned_transformed_pcg_matches_full():
    """Section 3.3: PCG on (V kron D_K + lam I) with the diagonal preconditioner."""
    p = _aligned_tiny(n=10, I=4, J=3, r=3)
    V = O.gram_V(p.A, p.B)
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    Bm = O.mttkrp_observed(p.y, Zhat, p.obs_t, p.n)
    Wf = O.solve_aligned_full(p.K, V, Bm, p.lam)
    dK, UK = np.linalg.eigh(p.K)
    res = O.solve_aligned_pcg(UK, dK, V, Bm, p.lam, 1e-13, 200)
    assert res.converged
    assert O.e_kw(p.K, res.X, Wf) < 1e-11


def test_aligned_rho_kron_equals_dense():
    """For a full observation set F^T F = V kron K^2 (O-kron == O-dense)."""
    p = _aligned_tiny(n=7, I=3, J=3, r=2)
    V = O.gram_V(p.A, p.B)
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    Bm = O.mttkrp_observed(p.y, Zhat, p.obs_t, p.n)
    Wk = O.solve_aligned_rho_kron(p.K, V, p.K @ Bm, p.lam, p.rho)
    Wd = O.solve_dense(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho)
    assert O.e_kw(p.K, Wk, Wd) < 1e-11


def test_full_tensor_mttkrp_equals_observed_mttkrp():
    """The MTTKRP of a fully observed tensor computed by unfolding (one matrix
    product) equals the per-observation segment sums of Section 4 and a
    triple loop over the entries."""
    p = _aligned_tiny(n=5, I=4, J=3, r=3)
    Y = p.y.reshape(p.n, p.I, p.J)
    full = O.mttkrp_full(Y, p.A, p.B)
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    obs = O.mttkrp_observed(p.y, Zhat, p.obs_t, p.n)
    loops = np.zeros((p.n, p.r))
    for s in range(p.n):
        for i in range(p.I):
            for j in range(p.J):
                for c in range(p.r):
                    loops[s, c] += Y[s, i, j] * p.A[i, c] * p.B[j, c]
    assert np.allclose(full, loops, rtol=1e-13, atol=1e-13)
    assert np.allclose(obs, loops, rtol=1e-13, atol=1e-13)


def test_aligned_rho_decoupled_equals_kron_and_dense():
    """For a full observation set the rho-system diagonalises in the
    eigenbases of K and V: the decoupled rho-solve equals O-kron and O-dense
    (a different algorithm for the same system), and the error estimate of
    O-kron is consistent with the distance to it."""
    p = _aligned_tiny(n=9, I=4, J=3, r=3)
    V = O.gram_V(p.A, p.B)
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    KB = p.K @ O.mttkrp_observed(p.y, Zhat, p.obs_t, p.n)
    dK, UK = np.linalg.eigh(p.K)
    dV, UV = np.linalg.eigh(V)
    Wdec = O.solve_aligned_rho_decoupled(UK, dK, UV, dV, KB, p.lam, p.rho)
    Wk, delta = O.solve_aligned_rho_kron_with_error(p.K, V, KB, p.lam, p.rho)
    Wd = O.solve_dense(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho)
    assert O.e_kw(p.K, Wdec, Wd) < 1e-11
    assert O.e_kw(p.K, Wk, Wd) < 1e-11
    assert delta < 1e-11
    # a wrong shift is caught
    Wbad = O.solve_aligned_rho_decoupled(UK, dK, UV, dV, KB, p.lam, 10 * p.rho)
    assert O.e_kw(p.K, Wbad, Wd) > 1e-8


# ------------------------------------------------------- special cases / PCG ----

def test_single_mode_case_is_kernel_ridge_regression():
    """I = J = r = 1, unit factors, every time observed once: K W equals the
    textbook kernel-ridge fit K (K + lam I)^{-1} y as rho -> 0."""
    rng = np.random.default_rng(17)
    n = 12
    t = np.sort(rng.random(n))
    K = np.exp(-((t[:, None] - t[None, :]) ** 2) / (2 * 0.3 ** 2))
    y = rng.standard_normal(n)
    lam, rho = 0.1, 1e-11
    obs_t = np.arange(n)
    Zhat = np.ones((n, 1))
    W = O.solve_dense(K, Zhat, obs_t, y, lam, rho)
    fit = (K @ W)[:, 0]
    krr = K @ sla.solve(K + lam * np.eye(n), y, assume_a="pos")
    assert np.linalg.norm(fit - krr) <= 1e-7 * np.linalg.norm(krr)


def test_pcg_iterates_match_library_cg():
    """The oracle's PCG recurrence produces the same iterates as scipy's cg with
    the same operator and preconditioner."""
    p = _tiny(n=10, I=4, J=3, r=3, q=60, lam=1e-2, rho=1e-4, seed=18)
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    V = O.gram_V(p.A, p.B)
    dK, UK = O.kernel_eig(p.K)
    dV, UV = np.linalg.eigh(V)
    n, r = p.n, p.r
    A_op = lambda X: O.matvec_twostep(p.K, Zhat, p.obs_t, p.lam, p.rho, X)
    M_op = lambda X: O.precond_apply(UK, dK, UV, dV, p.gamma, p.lam, p.rho, X)
    b = O.rhs_matrix(p.K, O.mttkrp_observed(p.y, Zhat, p.obs_t, n))
    Alin = spla.LinearOperator((n * r, n * r), dtype=float,
                               matvec=lambda v: O.vec(A_op(O.unvec(v, n, r))))
    Mlin = spla.LinearOperator((n * r, n * r), dtype=float,
                               matvec=lambda v: O.vec(M_op(O.unvec(v, n, r))))
    for k in (1, 2, 4):
        ours = O.pcg(A_op, M_op, b, tol=0.0, maxit=k)
        ref, _ = spla.cg(Alin, O.vec(b), rtol=0.0, atol=0.0, maxiter=k, M=Mlin)
        ref = O.unvec(ref, n, r)
        assert np.linalg.norm(ours.X - ref) <= 1e-9 * np.linalg.norm(ref)


def test_pcg_reaches_dense_solution_on_small_case():
    p = config_c1()
    Zhat, V = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j), O.gram_V(p.A, p.B)
    Wd = O.solve_dense(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho)
    res = O.solve_pcg(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho, p.gamma, V, 1e-12, 500)
    assert res.converged and res.iters < 100
    assert O.e_kw(p.K, res.X, Wd) < 1e-10
    # the preconditioner matters: plain CG needs many more iterations to 1e-6
    pc6 = O.solve_pcg(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho, p.gamma, V, 1e-6, 500)
    cg6 = O.solve_pcg(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho, p.gamma, V, 1e-6, 500,
                      precondition=False)
    assert cg6.iters > 4 * pc6.iters


def test_noise_free_recovery_improves_linearly_with_regularisation():
    """Noise-free rank-r data: the fitted-value misfit falls roughly in
    proportion to lambda (log-log slope near 1) and K W approaches K W*.
    rho is kept six decades below lambda so that the shift's own bias stays
    below the regularisation error being measured."""
    p = make_small(21, n=10, I=4, J=3, r=2, q=80, kernel="rbf", kernel_param=0.3,
                   noise=0.0)
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    lams = [1e-2, 1e-3, 1e-4, 1e-5, 1e-6]
    fits, ekw = [], []
    for lam in lams:
        W = O.solve_dense(p.K, Zhat, p.obs_t, p.y, lam, lam * 1e-6)
        pred = np.sum((p.K @ W)[p.obs_t] * Zhat, axis=1)
        fits.append(np.linalg.norm(pred - p.y) / np.linalg.norm(p.y))
        ekw.append(O.e_kw(p.K, W, p.Wstar))
    slopes = np.diff(np.log10(fits)) / np.diff(np.log10(lams))
    assert np.all(slopes > 0.7) and np.all(slopes < 1.3)
    assert all(b <= a for a, b in zip(ekw, ekw[1:]))
