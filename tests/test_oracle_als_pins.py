"""CPU pins of the alternating-optimisation oracle (oracle/cphifi_als.py).

* the model values against a loop over entries and rank components;
* exact block updates never increase the full objective (block coordinate
  descent on a function that is quadratic in each block);
* right after its update every block is stationary: the directional
  derivative of the full objective in W_k vanishes (the objective is evaluated
  from the model values, not from the subproblem solver, so a block update
  that used the wrong Khatri-Rao rows, indices or kernel would fail here);
* the PCG form warm-started and run to a tight tolerance follows the exact
  form's error history.
"""

import numpy as np

import oracle as O
from synth import make_als_problem


def small(seed=3, r=3):
    return make_als_problem(shape=(12, 10, 9), sigmas=(2.0, 2.0, 1.5), q=400, r=r, seed=seed,
                            lam=0.1, rho=1e-6, init_scale=0.5)


def test_cp_values_by_loops():
    p = small()
    F = [K @ W for K, W in zip(p.Ks, p.Wstar)]
    got = O.cp_values(F, p.coords)
    for l in range(0, p.coords.shape[0], 37):
        i, j, k = p.coords[l]
        want = 0.0
        for c in range(p.r):
            want += F[0][i, c] * F[1][j, c] * F[2][k, c]
        assert abs(got[l] - want) <= 1e-12 * max(1.0, abs(want))


def test_block_updates_never_increase_objective():
    p = small()
    res = O.cp_hifi_als(p.Ks, p.coords, p.y, p.W0s, p.lams, p.rho, max_outer=6, als_tol=0.0,
                        solver="dense", track_objective=True)
    f0 = O.als_objective(p.Ks, p.W0s, p.coords, p.y, p.lams, p.rho)
    seq = [f0] + res.objectives
    assert len(seq) == 1 + 3 * 6
    for a, b in zip(seq, seq[1:]):
        assert b <= a * (1 + 1e-12) + 1e-14
    assert seq[-1] < 0.5 * seq[0]


def _dir_deriv(p, Ws, k, E, h=1e-3):
    Wp = [W.copy() for W in Ws]
    Wm = [W.copy() for W in Ws]
    Wp[k] = Ws[k] + h * E
    Wm[k] = Ws[k] - h * E
    fp = O.als_objective(p.Ks, Wp, p.coords, p.y, p.lams, p.rho)
    fm = O.als_objective(p.Ks, Wm, p.coords, p.y, p.lams, p.rho)
    return (fp - fm) / (2 * h)


def test_each_block_update_is_stationary_in_its_block():
    p = small()
    seen = []
    O.cp_hifi_als(p.Ks, p.coords, p.y, p.W0s, p.lams, p.rho, max_outer=2, als_tol=0.0,
                  solver="dense", on_block=lambda it, k, Ws: seen.append((k, [W.copy() for W in Ws])))
    assert [k for k, _ in seen] == [0, 1, 2, 0, 1, 2]
    rng = np.random.default_rng(11)
    for k, Ws in seen:
        E = rng.standard_normal(Ws[k].shape)
        E *= np.linalg.norm(Ws[k]) / np.linalg.norm(E)
        g0 = _dir_deriv(p, Ws, k, E)
        # the same derivative one step away from the block minimiser: the
        # curvature scale that g0 must be small against
        Ws1 = [W.copy() for W in Ws]
        Ws1[k] = Ws[k] + E
        g1 = _dir_deriv(p, Ws1, k, E)
        assert abs(g1) > 0
        assert abs(g0) <= 1e-7 * abs(g1), (k, g0, g1)


def test_pcg_form_follows_exact_form():
    p = small()
    ex = O.cp_hifi_als(p.Ks, p.coords, p.y, p.W0s, p.lams, p.rho, max_outer=4, als_tol=0.0,
                       solver="dense")
    it = O.cp_hifi_als(p.Ks, p.coords, p.y, p.W0s, p.lams, p.rho, max_outer=4, als_tol=0.0,
                       solver="pcg", tol=1e-13, maxit=2000)
    assert np.allclose(ex.errors, it.errors, rtol=1e-7, atol=0)
    for k in range(3):
        assert O.e_kw(p.Ks[k], it.Ws[k], ex.Ws[k]) <= 1e-6


def test_stop_rule_and_history_length():
    p = small()
    res = O.cp_hifi_als(p.Ks, p.coords, p.y, p.W0s, p.lams, p.rho, max_outer=50, als_tol=1e-3,
                        solver="dense")
    assert len(res.errors) == res.outer + 1
    assert abs(res.errors[-1] - res.errors[-2]) < 1e-3
    if res.outer > 1:
        assert abs(res.errors[-2] - res.errors[-3]) >= 1e-3


def mixed_modes(seed=4, r=3):
    """Samples x features x time: two finite modes and one RKHS mode."""
    return make_als_problem(shape=(11, 8, 13), sigmas=(1.0, 1.0, 1.5), q=500, r=r, seed=seed,
                            lam=0.1, rho=1e-6, init_scale=0.5, finite=(True, True, False))


def test_finite_mode_row_solve_is_ridge_least_squares():
    """Each row of a finite-mode update against an independent solve of the
    stacked least-squares problem [Z_i; sqrt(rho) I] a = [y_i; 0] (SVD)."""
    p = mixed_modes()
    F = [p.W0s[0], p.W0s[1], p.Ks[2] @ p.W0s[2]]
    W = O.finite_mode_update(p.coords, p.y, F, 0, p.W0s[0].shape[0], 10 * p.rho)
    for row in range(W.shape[0]):
        sel = p.coords[:, 0] == row
        Z = F[1][p.coords[sel, 1]] * F[2][p.coords[sel, 2]]
        M = np.vstack([Z, np.sqrt(10 * p.rho) * np.eye(p.r)])
        rhs = np.concatenate([p.y[sel], np.zeros(p.r)])
        want = np.linalg.lstsq(M, rhs, rcond=None)[0]
        assert np.allclose(W[row], want, rtol=1e-9, atol=1e-12)


def test_finite_and_rkhs_blocks_stationary_and_monotone():
    p = mixed_modes()
    seen = []
    res = O.cp_hifi_als(p.Ks, p.coords, p.y, p.W0s, p.lams, p.rho, max_outer=2, als_tol=0.0,
                        solver="dense", track_objective=True,
                        on_block=lambda it, k, Ws: seen.append((k, [W.copy() for W in Ws])))
    f0 = O.als_objective(p.Ks, p.W0s, p.coords, p.y, p.lams, p.rho)
    seq = [f0] + res.objectives
    for a, b in zip(seq, seq[1:]):
        assert b <= a * (1 + 1e-12) + 1e-14
    rng = np.random.default_rng(12)
    for k, Ws in seen:
        E = rng.standard_normal(Ws[k].shape)
        E *= np.linalg.norm(Ws[k]) / np.linalg.norm(E)
        g0 = _dir_deriv(p, Ws, k, E)
        Ws1 = [W.copy() for W in Ws]
        Ws1[k] = Ws[k] + E
        g1 = _dir_deriv(p, Ws1, k, E)
        assert abs(g0) <= 1e-7 * abs(g1), (k, g0, g1)
