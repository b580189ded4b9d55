"""GPU parity of the structured forms (CPHIFI_FLAG_TOEPLITZ_K,
CPHIFI_FLAG_FIBER_COLLAPSE) against the general path and the oracle.

* Toeplitz K (uniform grid, Gaussian kernel; Section 4.4.1's remark on
  structured K): the right-hand side b = K B and the operator agree with the
  dense-K plan to 1e-11 in every row (the plan admits K when every entry is
  within 1e-12 max|c| of c(|s - k|)); a K from a non-uniform grid is refused;
* fiber collapse (every observed (time, sample) pair observed at all J
  features): the operator and the low-precision eigenbasis operator agree with
  the per-observation gather-scatter to 1e-12 / 1e-6 in every row, the FP64
  and mixed solves reach the same gates as without the flag; an incomplete
  fiber is refused;
* both together on the aligned case (gamma = 1): one PCG iteration, the same
  W as the general operator's to 1e-10 in K W.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from synth import config_c1, config_c3, drop_observations, make_aligned, sample_rows  # noqa: E402

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2603_25691_amd import cphifi as C  # noqa: E402
    from paper_2603_25691_amd.torch_api import UISolver, upload  # noqa: E402


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def row_err(a, b):
    return float(np.max(np.linalg.norm(a - b, axis=1)) / np.max(np.linalg.norm(b, axis=1)))


def probe(n, r, seed):
    return torch.from_numpy(np.random.default_rng(seed).standard_normal((n, r))).cuda()


def aligned_case(r=10):
    return make_aligned(5, I=60, J=25, n=200, r=r, sigma=0.05, lam=1e-4, rho=1e-6, tol=1e-10)


@pytest.mark.parametrize("r", [10, 40])
def test_toeplitz_products_match_dense(r):
    p = aligned_case(r)
    dp = upload(p)
    s0 = UISolver(dp, p.lam, p.rho, 1e-10)
    s1 = UISolver(dp, p.lam, p.rho, 1e-10, flags=C.FLAG_TOEPLITZ_K)
    b0, b1 = host(s0.rhs()), host(s1.rhs())
    assert row_err(b1, b0) <= 1e-11
    X = probe(p.n, r, 7)
    y0, y1 = host(s0.apply(X)), host(s1.apply(X))
    assert row_err(y1, y0) <= 1e-11
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    ref = O.matvec_twostep(p.K, Zhat, p.obs_t, p.lam, p.rho, host(X))
    assert row_err(y1, ref) <= 1e-11
    s0.close()
    s1.close()


def test_toeplitz_refuses_non_uniform_grid():
    p = config_c1()
    dp = upload(p)
    with pytest.raises(C.CphifiError) as ei:
        UISolver(dp, p.lam, p.rho, 1e-10, flags=C.FLAG_TOEPLITZ_K)
    assert ei.value.status == C.INVALID_ARG


@pytest.mark.parametrize("case", ["c1", "aligned", "c3-I100"])
def test_fiber_collapse_operator_matches_gather(case):
    p = {"c1": config_c1, "aligned": aligned_case,
         "c3-I100": lambda: config_c3(I=100)}[case]()
    dp = upload(p)
    s0 = UISolver(dp, p.lam, p.rho, 1e-10)
    s1 = UISolver(dp, p.lam, p.rho, 1e-10, flags=C.FLAG_FIBER_COLLAPSE)
    X = probe(p.n, p.r, 9)
    assert row_err(host(s1.apply(X)), host(s0.apply(X))) <= 1e-12
    for prec in ("mixed_fp32", "mixed_bf16"):
        m0 = UISolver(dp, p.lam, p.rho, 1e-7, precision=prec)
        m1 = UISolver(dp, p.lam, p.rho, 1e-7, precision=prec, flags=C.FLAG_FIBER_COLLAPSE)
        m0.setup()
        m1.setup()
        assert row_err(host(m1.apply_lowp(X)), host(m0.apply_lowp(X))) <= 1e-6
        m0.close()
        m1.close()
    s0.close()
    s1.close()


@pytest.mark.parametrize("precision,tol,gate", [("fp64", 1e-12, None), ("mixed_bf16", 1e-7, 1e-6)])
def test_fiber_collapse_solves(precision, tol, gate):
    p = config_c1()
    dp = upload(p)
    s = UISolver(dp, p.lam, p.rho, tol, precision=precision, flags=C.FLAG_FIBER_COLLAPSE)
    W, info = s.solve_subproblem()
    assert info.status == C.OK, info.as_dict()
    assert info.relres_true <= 10 * tol
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    Wo, delta = O.solve_dense_with_error(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho)
    assert O.e_kw(p.K, host(W), Wo) <= (gate if gate is not None else max(1e-10, 3 * delta))
    s.close()


def test_fiber_collapse_refuses_incomplete_fiber():
    p = drop_observations(config_c1(), 0.9, 3)
    dp = upload(p)
    with pytest.raises(C.CphifiError) as ei:
        UISolver(dp, p.lam, p.rho, 1e-10, flags=C.FLAG_FIBER_COLLAPSE)
    assert ei.value.status == C.INVALID_ARG


def test_toeplitz_and_fiber_collapse_on_aligned_case():
    """With gamma = 1 the single PCG iteration returns alpha M^-1 b: only alpha
    depends on the operator, so the structured and the general operator give
    the same W up to the rounding of p^T A p (the general path is checked
    against the oracle's decoupled rho-solve in test_gpu_configs.py)."""
    p = aligned_case(20)
    dp = upload(p)
    s = UISolver(dp, p.lam, p.rho, 1e-10, flags=C.FLAG_TOEPLITZ_K | C.FLAG_FIBER_COLLAPSE)
    W, info = s.solve_subproblem()
    assert info.status == C.OK and info.iters == 1
    g = UISolver(dp, p.lam, p.rho, 1e-10)
    Wg, ig = g.solve_subproblem()
    assert ig.status == C.OK and ig.iters == 1
    assert O.e_kw(p.K, host(W), host(Wg)) <= 1e-10
    assert abs(info.relres_true - ig.relres_true) <= 1e-3 * ig.relres_true + 1e-14
    s.close()
    g.close()
