"""GPU parity of the batched solver (one persistent, graph-captured launch for
many subproblems of uneven n and r), through the C ABI.

Every member is checked against the FP64 CPU oracle: the oracle's own residual
certificate ||K B - A(W)|| / ||K B|| (two-step product in numpy) must meet the
member's tolerance, and for members small enough for the dense normal-equation
solve, e_KW = ||K (W - W_o)|| / ||K W_o|| <= 1e-6 (the mixed form's bar after
refinement).  Batched and unbatched (the same member's plan solved alone by
cphifi_ui_solve_subproblem at MIXED_BF16, from the same observed values: the
batched launch also runs the per-solve setup and the MTTKRP) must agree to
e_KW <= 1e-6; both are refined to
relres 1e-8, so their distance is bounded by the conditioning of the map from
residual to K W, which for these members is far below 1e2.
"""

import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from synth import config_c1, drop_observations, make_aligned, make_batch, make_small  # noqa: E402

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2603_25691_amd import cphifi as C  # noqa: E402
    from paper_2603_25691_amd.torch_api import BatchSolver, upload  # noqa: E402

TOL = 1e-8
DENSE_MAX_NR = 6000
CAPS = dict(maxit=200, max_refine=12)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def members():
    ms = [
        ("c1", config_c1()),
        ("ragged-r3", make_small(31, n=77, I=5, J=7, r=3, q=400, kernel_param=0.2)),
        ("ragged-r17", make_small(32, n=301, I=9, J=11, r=17, q=6000, kernel_param=0.1)),
        ("r40", make_small(33, n=650, I=20, J=30, r=40, q=12000, kernel="matern32",
                           kernel_param=0.1)),
        # 1200 observations per time point: every segment spans two gather tasks
        ("aligned-multi", make_aligned(5, I=40, J=30, n=30, r=10, sigma=0.1, lam=1e-3,
                                       rho=1e-6, tol=TOL)),
        ("c1-drop", drop_observations(config_c1(), 0.5, 7)),
    ]
    for bm in make_batch(seed=1, count=2, n_lo=500, n_hi=1500):
        ms.append((bm.problem.name, bm.problem))
    return ms


MEMBERS = members()


@pytest.fixture(scope="module")
def batch():
    probs = [p for _, p in MEMBERS]
    dps = [upload(p) for p in probs]
    bs = BatchSolver(dps, [p.lam for p in probs], [p.rho for p in probs], TOL, **CAPS)
    rhs = bs.rhs()
    Ws = [torch.empty_like(b) for b in rhs]
    status, infos = bs.solve(bs.ys(), Ws)
    return {"probs": probs, "dps": dps, "bs": bs, "rhs": rhs, "W": [host(W) for W in Ws],
            "status": status, "infos": infos}


def _zhat(p):
    return O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)


@pytest.mark.parametrize("k", range(len(MEMBERS)), ids=[m[0] for m in MEMBERS])
def test_batch_member_matches_oracle(batch, k):
    p = batch["probs"][k]
    info = batch["infos"][k]
    W = batch["W"][k]
    assert info.status == C.OK, info.as_dict()
    assert info.relres_true <= TOL
    Zhat = _zhat(p)
    cert = O.relres(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho, W)
    assert cert <= 2 * TOL, cert
    assert abs(cert - info.relres_true) <= 0.05 * TOL + 1e-3 * cert
    if p.n * p.r <= DENSE_MAX_NR:
        Wo = O.solve_dense(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho)
        assert O.e_kw(p.K, W, Wo) <= 1e-6


def test_batch_status_and_rounds(batch):
    assert batch["status"] == C.OK
    rounds, grid = batch["bs"].rounds()
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    assert grid >= n_cu
    # every member needs at least SETUP, ROT_B, one inner iteration, FINAL, CERT
    assert rounds >= 5
    assert rounds >= max(i.iters for i in batch["infos"])


@pytest.mark.parametrize("k", range(len(MEMBERS)), ids=[m[0] for m in MEMBERS])
def test_batched_equals_unbatched(batch, k):
    p = batch["probs"][k]
    bs = batch["bs"]
    b = batch["rhs"][k]
    Ws = torch.zeros_like(b)
    # the same whole-subproblem method from the observed values, one member alone
    info = C.cphifi_ui_solve_subproblem(bs.plan(k), batch["dps"][k].y.data_ptr(), Ws.data_ptr())
    assert info.status == C.OK, info.as_dict()
    assert info.relres_true <= TOL
    assert O.e_kw(p.K, batch["W"][k], host(Ws)) <= 1e-6
    # same method: the refinement takes the same number of outer steps (+-1)
    assert abs(info.refine_steps - batch["infos"][k].refine_steps) <= 1


def test_batch_is_deterministic(batch):
    bs = batch["bs"]
    Ws = [torch.empty_like(b) for b in batch["rhs"]]
    status, infos = bs.solve(bs.ys(), Ws)
    assert status == C.OK
    for k, W in enumerate(Ws):
        assert np.array_equal(host(W), batch["W"][k]), MEMBERS[k][0]
        assert infos[k].iters == batch["infos"][k].iters
        assert infos[k].relres_true == batch["infos"][k].relres_true


def test_batch_rebind_scaled_observations(batch):
    bs = batch["bs"]
    ys2 = [2.0 * y for y in bs.ys()]
    Ws = [torch.empty_like(b) for b in batch["rhs"]]
    status, infos = bs.solve(ys2, Ws)
    assert status == C.OK
    for k, W in enumerate(Ws):
        p = batch["probs"][k]
        assert O.e_kw(p.K, host(W), 2.0 * batch["W"][k]) <= 1e-6


def test_batch_binding_checks_shapes(batch):
    """The C ABI takes raw pointers, so the binding checks what it hands over:
    right-hand sides (n x r) where observed values (q) belong are refused
    before any launch."""
    bs = batch["bs"]
    Ws = [torch.empty_like(b) for b in batch["rhs"]]
    with pytest.raises(ValueError):
        bs.bind(batch["rhs"], Ws)
    with pytest.raises(ValueError):
        bs.solve(batch["rhs"], Ws)
    with pytest.raises(ValueError):
        bs.bind(bs.ys(), Ws[:-1])


def test_batch_zero_observations_and_async_info(batch):
    bs = batch["bs"]
    zeros = [torch.zeros_like(y) for y in bs.ys()]
    Ws = [torch.full_like(b, 3.0) for b in batch["rhs"]]
    assert bs.solve(zeros, Ws, wait=False) is None
    status, infos = bs.info()
    assert status == C.OK
    for W, info in zip(Ws, infos):
        assert info.status == C.OK
        assert info.iters == 0 and info.refine_steps == 0
        assert float(torch.count_nonzero(W)) == 0.0


def test_batch_warm_start_from_solution(batch):
    probs, dps = batch["probs"][:3], batch["dps"][:3]
    bs = BatchSolver(dps, [p.lam for p in probs], [p.rho for p in probs], TOL,
                     flags=C.FLAG_WARM_START, **CAPS)
    try:
        rhs = bs.rhs()
        Ws = [torch.from_numpy(batch["W"][k]).cuda() for k in range(3)]
        status, infos = bs.solve(bs.ys(), Ws)
        assert status == C.OK
        for k, info in enumerate(infos):
            assert info.status == C.OK
            assert info.refine_steps == 0 and info.iters == 0
            assert info.relres_true <= TOL
            # W = U (U^T W0): the start point back, up to the rounding of two
            # orthogonal FP64 rotations
            p = probs[k]
            assert O.e_kw(p.K, host(Ws[k]), batch["W"][k]) <= 1e-12
    finally:
        bs.close()


def test_batch_barrier_timeout_is_reported_and_drains(batch):
    """A spin limit of one poll makes the bounded grid waits time out: every
    workgroup must leave the kernel and the solve must report HIP_ERROR; a
    batch built afterwards with the normal limit solves again."""
    probs, dps = batch["probs"][:2], batch["dps"][:2]
    os.environ["CPHIFI_BATCH_SPIN_LIMIT"] = "1"
    try:
        bs = BatchSolver(dps, [p.lam for p in probs], [p.rho for p in probs], TOL, **CAPS)
    finally:
        del os.environ["CPHIFI_BATCH_SPIN_LIMIT"]
    try:
        rhs = bs.rhs()
        Ws = [torch.empty_like(b) for b in rhs]
        with pytest.raises(C.CphifiError) as ei:
            bs.solve(bs.ys(), Ws)
        assert ei.value.status == C.HIP_ERROR
        assert "timed out" in str(ei.value)
    finally:
        bs.close()
    bs2 = BatchSolver(dps, [p.lam for p in probs], [p.rho for p in probs], TOL, **CAPS)
    try:
        rhs = bs2.rhs()
        Ws = [torch.empty_like(b) for b in rhs]
        status, infos = bs2.solve(bs2.ys(), Ws)
        assert status == C.OK
        for k in range(2):
            assert np.array_equal(host(Ws[k]), batch["W"][k])
    finally:
        bs2.close()


def test_batch_graph_handle(batch):
    assert batch["bs"].graph() != 0


def test_batch_with_padded_kernel_stride(batch):
    """K and U_K stored with a row stride above n (16-byte aligned rows for
    odd n): same solutions as the unpadded layout."""
    idx = [k for k, p in enumerate(batch["probs"]) if p.n % 2 == 1][:3]
    assert idx, "need members of odd n"
    probs = [batch["probs"][k] for k in idx]
    dps = [upload(p, ldk_align=64) for p in probs]
    assert all(dp.K.shape[1] % 64 == 0 and dp.K.shape[1] > dp.n for dp in dps)
    bs = BatchSolver(dps, [p.lam for p in probs], [p.rho for p in probs], TOL, **CAPS)
    try:
        rhs = bs.rhs()
        Ws = [torch.empty_like(b) for b in rhs]
        status, infos = bs.solve(bs.ys(), Ws)
        assert status == C.OK
        for j, k in enumerate(idx):
            p = batch["probs"][k]
            assert infos[j].relres_true <= TOL
            assert O.e_kw(p.K, host(Ws[j]), batch["W"][k]) <= 1e-6
    finally:
        bs.close()


def test_batch_with_tuner_table(batch, tmp_path):
    """Tiles from a table written by the batch autotuner (a k-range and BF16
    rows per wave other than the defaults): the same solutions."""
    from paper_2603_25691_amd import tune

    probs, dps = batch["probs"], batch["dps"]
    path = tmp_path / "tiles.txt"
    tune._batch_table(str(path), 1024, 2, 8192)
    bs = BatchSolver(dps, [p.lam for p in probs], [p.rho for p in probs], TOL,
                     tile_table=str(path), **CAPS)
    try:
        rhs = bs.rhs()
        Ws = [torch.empty_like(b) for b in rhs]
        status, infos = bs.solve(bs.ys(), Ws)
        assert status == C.OK
        for k, W in enumerate(Ws):
            assert infos[k].relres_true <= TOL, MEMBERS[k][0]
            assert O.e_kw(probs[k].K, host(W), batch["W"][k]) <= 1e-6, MEMBERS[k][0]
    finally:
        bs.close()


def test_batch_member_with_inexact_eigenpairs_converges():
    """A member whose eigenpairs are those of K + E (||E|| = 1e-7 ||K||): its
    certificate misses after the eigenbasis refinement converges, and the
    member must go on from the certificate's residual (and certify every later
    step) until the original system meets tol; the other member is unaffected."""
    p = config_c1()
    q = make_small(31, n=77, I=5, J=7, r=3, q=400, kernel_param=0.2)
    rng = np.random.default_rng(5)
    E = rng.standard_normal(p.K.shape)
    E = (E + E.T) / 2
    E *= 1e-7 * np.linalg.norm(p.K, 2) / np.linalg.norm(E, 2)
    dK, U = np.linalg.eigh(p.K + E)
    dps = [upload(p, eig=(np.ascontiguousarray(U.T), dK)), upload(q)]
    bs = BatchSolver(dps, [p.lam, q.lam], [p.rho, q.rho], TOL, **CAPS)
    rhs = bs.rhs()
    Ws = [torch.empty_like(b) for b in rhs]
    status, infos = bs.solve(bs.ys(), Ws)
    assert status == C.OK, [i.as_dict() for i in infos]
    assert infos[0].refine_steps > 3  # the eigenbasis alone stops at ~8e-7
    for pr, W, info in zip((p, q), Ws, infos):
        assert info.status == C.OK, info.as_dict()
        Zhat = _zhat(pr)
        cert = O.relres(pr.K, Zhat, pr.obs_t, pr.y, pr.lam, pr.rho, host(W))
        assert cert <= 2 * TOL, cert
        Wo = O.solve_dense(pr.K, Zhat, pr.obs_t, pr.y, pr.lam, pr.rho)
        assert O.e_kw(pr.K, host(W), Wo) <= 1e-6
    bs.close()
