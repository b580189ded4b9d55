"""The device Jacobi eigensolver (cphifi_kernel_eig_jacobi, eq. eigK) against
numpy.  The method stops when the off-diagonal mass is at most tol ||K||_F, so
every eigenpair residual ||K u_k - d_k u_k|| and every eigenvalue's distance
from numpy's eigvalsh is bounded by tol ||K||_F plus the rounding of O(n)
operations on entries of size ||K||_2; the gate is
tol ||K||_F + 10 n u ||K||_2 (u = 2^-53; at n = 3000, tol = 1e-14 this is
~3e-12 ||K||_2, measured 1.0e-12), and the orthogonality max |U U^T - I|
<= 10 n u.  Odd and even orders, n = 1 and 2, a Gaussian and a Matern kernel
matrix; a subproblem solved with these eigenpairs meets the same gate as with
the divide-and-conquer ones."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from synth import config_c1  # noqa: E402
from synth.generator import kernel_matrix  # noqa: E402

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2603_25691_amd import cphifi as C  # noqa: E402
    from paper_2603_25691_amd.torch_api import UISolver, kernel_eig, upload  # noqa: E402


def kmat(n, kind, param, seed):
    t = np.sort(np.random.default_rng(seed).random(n))
    return kernel_matrix(t, kind, param)


@pytest.mark.parametrize("n,kind,param", [(1, "rbf", 0.1), (2, "rbf", 0.1), (7, "rbf", 0.3),
                                          (200, "rbf", 0.1), (501, "rbf", 0.05),
                                          (1200, "matern32", 0.1), (3000, "matern32", 0.1)])
def test_jacobi_eig_matches_numpy(n, kind, param):
    K = kmat(n, kind, param, n)
    UK, dK = kernel_eig(torch.from_numpy(K).cuda(), method="jacobi")
    U = UK.cpu().numpy()   # row k = eigenvector k
    d = dK.cpu().numpy()
    knorm = np.linalg.norm(K, 2)
    u = 2.0 ** -53
    gate = 1e-14 * np.linalg.norm(K) + 10 * n * u * knorm
    res = np.linalg.norm(U @ K - d[:, None] * U, axis=1)
    assert res.max() <= gate, res.max() / knorm
    assert np.abs(U @ U.T - np.eye(n)).max() <= 10 * n * u
    assert np.all(np.diff(d) >= 0)
    assert np.abs(d - np.linalg.eigvalsh(K)).max() <= gate
    assert 0 <= kernel_eig.last_sweeps <= 30


def test_subproblem_with_jacobi_eigenpairs():
    p = config_c1()
    UK, dK = kernel_eig(torch.from_numpy(p.K).cuda(), method="jacobi")
    dp = upload(p, eig=(UK.cpu().numpy(), dK.cpu().numpy()))
    s = UISolver(dp, p.lam, p.rho, 1e-12)
    W, info = s.solve_subproblem()
    assert info.status == C.OK, info.as_dict()
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    Wo, delta = O.solve_dense_with_error(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho)
    torch.cuda.synchronize()
    assert O.e_kw(p.K, W.cpu().numpy(), Wo) <= max(1e-10, 3 * delta)
    s.close()


def test_jacobi_eig_rejects_bad_arguments():
    K = torch.eye(4, dtype=torch.float64, device="cuda")
    with pytest.raises(C.CphifiError) as ei:
        kernel_eig(K, method="jacobi", tol=0.0)
    assert ei.value.status == C.INVALID_ARG
