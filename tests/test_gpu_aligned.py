"""The aligned subproblem (Section 3) on the GPU, through the C ABI, at the
aligned workload's size (n = 200 grid, I = 500, J = 100, q = 1e7, Gaussian
0.05, lambda = 1e-4, r = 10 / 20 / 40) against the oracle:

* the observed MTTKRP (cphifi_ui_mttkrp) of the fully observed tensor against
  the oracle's unfolding T Z (mttkrp_full), 1e-12 relative, row by row;
* the decoupled direct solve (eq. W-decoupled) against the oracle's decoupled
  solve (same formula in numpy) and the Cholesky solve of eq. aligned-solve
  (e_KW <= max(g, 3 delta), delta its own forward error).  g = max(5e-10, 3 s)
  with s the oracle's own spread: its decoupled solve moves by s = 2.8e-10 to
  5.4e-10 in K W when numpy's eigensolver is swapped for LAPACK's MRRR one
  (both backward stable; the GPU uses a third);
* PCG on the transformed system (eqs. pcg-matvec-ai, precond-ai) to relres
  1e-12: within g of the decoupled solve and of the oracle's transformed PCG,
  and the oracle's iteration count (+-2).
The paper reports the decoupled and PCG solves agreeing ("decoupled vs PCG,
same result"); both are also compared with the rho-system UI solve.
"""

import numpy as np
import pytest
import scipy.linalg as sla

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from synth import config_c2, make_aligned  # noqa: E402

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2603_25691_amd import cphifi as C  # noqa: E402
    from paper_2603_25691_amd.torch_api import AlignedSolver, UISolver, upload  # noqa: E402

RANKS = (10, 20, 40)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _full_aligned_with_error(K, V, Bm, lam):
    """Cholesky of V kron K + lam I and one refinement step (its own error)."""
    import scipy.linalg as sla

    n, r = Bm.shape
    H = np.kron(V, K) + lam * np.eye(n * r)
    c = sla.cho_factor(H, lower=True)
    w = sla.cho_solve(c, O.vec(Bm))
    dw = sla.cho_solve(c, O.vec(Bm) - H @ w)
    W = O.unvec(w, n, r)
    return W, float(np.linalg.norm(K @ O.unvec(dw, n, r)) / np.linalg.norm(K @ W))


@pytest.fixture(scope="module")
def cases():
    cache = {}

    def get(r):
        if r not in cache:
            p = config_c2(r=r)
            dp = upload(p)
            Bm = O.mttkrp_full(p.y.reshape(p.n, p.I, p.J), p.A, p.B)
            V = O.gram_V(p.A, p.B)
            dK, UK = O.kernel_eig(p.K)
            dV, UV = np.linalg.eigh(V)
            Wdec = O.solve_decoupled(UK, dK, UV, dV, Bm, p.lam)
            d2, U2 = sla.eigh(p.K, driver="evr")
            W2 = O.solve_decoupled(U2, np.maximum(d2, 0.0), UV, dV, Bm, p.lam)
            gate = max(5e-10, 3 * O.e_kw(p.K, W2, Wdec))
            cache[r] = dict(p=p, dp=dp, Bm=Bm, V=V, Wdec=Wdec, eig=(dK, UK), gate=gate)
        return cache[r]

    return get


@pytest.mark.parametrize("r", RANKS)
def test_mttkrp_of_full_tensor(r, cases):
    c = cases(r)
    p = c["p"]
    s = UISolver(c["dp"], p.lam, p.rho, 1e-10)
    got = host(s.mttkrp())
    want = c["Bm"]
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
    assert np.max(np.linalg.norm(got - want, axis=1)) <= 1e-12 * np.max(
        np.linalg.norm(want, axis=1))
    s.close()


@pytest.mark.parametrize("r", RANKS)
def test_decoupled_solve_matches_oracle(r, cases):
    c = cases(r)
    p = c["p"]
    # V given (formed on the host from the factors)
    Vd = torch.from_numpy((p.A.T @ p.A) * (p.B.T @ p.B)).cuda()
    a = AlignedSolver(c["dp"], p.lam, method="decoupled", V=Vd)
    Bm = torch.from_numpy(c["Bm"]).cuda()
    W, info = a.solve(Bm)
    assert info.status == C.OK, info.as_dict()
    Wg = host(W)
    assert O.e_kw(p.K, Wg, c["Wdec"]) <= c["gate"]
    Wf, delta = _full_aligned_with_error(p.K, c["V"], c["Bm"], p.lam)
    assert O.e_kw(p.K, Wg, Wf) <= max(c["gate"], 3 * delta), delta
    assert info.relres_true <= 1e-12
    # V formed from the factors on the device: the same solution
    a2 = AlignedSolver(c["dp"], p.lam, method="decoupled", with_factors=True)
    W2, info2 = a2.solve(Bm)
    assert O.e_kw(p.K, host(W2), Wg) <= c["gate"]
    a.close()
    a2.close()


@pytest.mark.parametrize("r", RANKS)
def test_transformed_pcg_matches_decoupled_and_oracle(r, cases):
    c = cases(r)
    p = c["p"]
    a = AlignedSolver(c["dp"], p.lam, method="pcg", tol=1e-12)
    W, info = a.solve(torch.from_numpy(c["Bm"]).cuda())
    assert info.status == C.OK, info.as_dict()
    assert info.relres_true <= 1e-11
    Wg = host(W)
    assert O.e_kw(p.K, Wg, c["Wdec"]) <= c["gate"]
    dK, UK = c["eig"]
    ref = O.solve_aligned_pcg(UK, dK, c["V"], c["Bm"], p.lam, 1e-12, 500)
    assert ref.converged
    assert abs(info.iters - ref.iters) <= 2
    assert O.e_kw(p.K, Wg, ref.X) <= c["gate"]
    a.close()


def test_transformed_pcg_iteration_cap_and_zero_rhs():
    p = make_aligned(3, I=6, J=5, n=40, r=4, sigma=0.1, lam=1e-3, rho=1e-6, tol=1e-10)
    dp = upload(p)
    a = AlignedSolver(dp, p.lam, method="pcg", tol=1e-14, maxit=2)
    Bm = torch.from_numpy(O.mttkrp_full(p.y.reshape(p.n, p.I, p.J), p.A, p.B)).cuda()
    W, info = a.solve(Bm)
    assert info.status == C.NOT_CONVERGED and info.iters == 2
    W0, info0 = a.solve(torch.zeros_like(Bm))
    assert info0.status == C.OK and info0.iters == 0
    assert float(torch.count_nonzero(W0)) == 0
    a.close()


def test_aligned_rejects_bad_arguments():
    p = make_aligned(3, I=6, J=5, n=40, r=4, sigma=0.1, lam=1e-3, rho=1e-6, tol=1e-10)
    dp = upload(p)
    with pytest.raises(C.CphifiError) as ei:
        AlignedSolver(dp, 0.0, method="decoupled")
    assert ei.value.status == C.INVALID_ARG
    with pytest.raises(C.CphifiError) as ei:
        AlignedSolver(dp, 1e-3, method="pcg", tol=0.0)
    assert ei.value.status == C.INVALID_ARG
