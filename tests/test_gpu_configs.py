"""GPU parity at the workloads' own sizes: the aligned case (n = 200 uniform
grid shared by I = 500 samples, J = 100 features, q = 1e7, Gaussian 0.05,
r = 10 / 20 / 40, lambda = 1e-4, rho = 1e-6) in FP64 and in the two mixed
precisions, through the C ABI, against the FP64 CPU oracle.

With every entry observed, gamma = 1 and the eq. (fx) preconditioner equals the
system matrix (Section 4.4.2), so PCG stops after one iteration and the
solution is the decoupled rho-solve O-dec: W = U_K ((U_K^T K B U_V) /
(dK^2 dV^T + lambda dK + rho)) U_V^T.  O-dec works entrywise in the
eigenbasis and is accurate to rounding in K W; O-kron (Cholesky of the
8000 x 8000 Kronecker system, condition ~1e13) lands 5e-9 to 1.1e-8 from
O-dec in K W (its one-step refinement estimate of its own error, ~1e-9,
understates that), so the gate against O-kron is that measured distance plus
the gate against O-dec.  The one PCG iteration returns alpha M^-1 b
with alpha = r^T z / p^T A p, which is 1 in exact arithmetic; its rounding
(the operator applied to z ~ A^-1 b, condition ~1e13) moves K W by |alpha - 1|.
The oracle's own PCG lands 6e-11 to 2.5e-10 from O-dec on these three cases
(tests/test_oracle_spread.py measures it at r = 10).  O-dec itself moves by
2.6e-10 to 3.5e-10 in K W when numpy's eigensolver is swapped for LAPACK's
MRRR one (both backward stable; the GPU uses a third), so the FP64 gate
against O-dec is max(5e-10, 3 s), s = that eigensolver spread, computed here.
Mixed forms refined to relres 1e-7: e_KW <= 1e-6.
"""

import numpy as np
import pytest
import scipy.linalg as sla

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from synth import config_c2  # noqa: E402

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2603_25691_amd import cphifi as C  # noqa: E402
    from paper_2603_25691_amd.torch_api import UISolver, upload  # noqa: E402

RANKS = (10, 20, 40)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def aligned():
    cache = {}

    def get(r):
        if r not in cache:
            p = config_c2(r=r)
            Bm = O.mttkrp_full(p.y.reshape(p.n, p.I, p.J), p.A, p.B)
            KB = p.K @ Bm
            V = O.gram_V(p.A, p.B)
            dK, UK = O.kernel_eig(p.K)
            dV, UV = np.linalg.eigh(V)
            Wdec = O.solve_aligned_rho_decoupled(UK, dK, UV, dV, KB, p.lam, p.rho)
            d2, U2 = sla.eigh(p.K, driver="evr")
            W2 = O.solve_aligned_rho_decoupled(U2, np.maximum(d2, 0.0), UV, dV, KB, p.lam,
                                               p.rho)
            gate = max(5e-10, 3 * O.e_kw(p.K, W2, Wdec))
            Wkron, delta = O.solve_aligned_rho_kron_with_error(p.K, V, KB, p.lam, p.rho)
            # the paper's own decoupled solve (rho = 0, right-hand side B)
            W0 = O.solve_decoupled(UK, dK, UV, dV, Bm, p.lam)
            cache[r] = dict(p=p, dp=upload(p), Bm=Bm, KB=KB, Wdec=Wdec, Wkron=Wkron,
                            delta=delta, W0=W0, gate=gate)
        return cache[r]

    return get


@pytest.mark.parametrize("r", RANKS)
def test_aligned_fp64_one_iteration_matches_decoupled_and_kron(r, aligned):
    a = aligned(r)
    p = a["p"]
    assert p.q == 10_000_000 and p.gamma == 1.0
    s = UISolver(a["dp"], p.lam, p.rho, 1e-10)
    W, info = s.solve_subproblem()
    assert info.status == C.OK, info.as_dict()
    assert info.iters == 1
    Wg = host(W)
    e_dec = O.e_kw(p.K, Wg, a["Wdec"])
    e_kron = O.e_kw(p.K, Wg, a["Wkron"])
    assert e_dec <= a["gate"], (e_dec, a["gate"])
    assert e_kron <= O.e_kw(p.K, a["Wkron"], a["Wdec"]) + a["gate"], (e_kron, a["delta"])
    # rows: the largest row error against the largest row of K W
    KW, KWo = p.K @ Wg, p.K @ a["Wdec"]
    assert np.max(np.linalg.norm(KW - KWo, axis=1)) <= a["gate"] * np.max(
        np.linalg.norm(KWo, axis=1))
    # the paper's rho = 0 decoupled solve solves a different system: reported
    # distance, bounded by the effect of the shift
    assert O.e_kw(p.K, Wg, a["W0"]) <= 1e-3
    s.close()


@pytest.mark.parametrize("r", RANKS)
def test_aligned_rhs_matches_oracle(r, aligned):
    a = aligned(r)
    p = a["p"]
    s = UISolver(a["dp"], p.lam, p.rho, 1e-10)
    b = host(s.rhs())
    want = a["KB"]
    assert np.linalg.norm(b - want) <= 1e-12 * np.linalg.norm(want)
    assert np.max(np.abs(b - want)) <= 1e-12 * np.max(np.abs(want))
    s.close()


@pytest.mark.parametrize("precision", ["mixed_bf16", "mixed_fp32"])
@pytest.mark.parametrize("r", RANKS)
def test_aligned_precision_form_reaches_1e6(r, precision, aligned):
    a = aligned(r)
    p = a["p"]
    s = UISolver(a["dp"], p.lam, p.rho, 1e-7, precision=precision)
    W, info = s.solve_subproblem()
    assert info.status == C.OK, info.as_dict()
    assert info.relres_true <= 1e-7
    assert O.e_kw(p.K, host(W), a["Wdec"]) <= 1e-6
    s.close()
