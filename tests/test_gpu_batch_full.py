"""The batched workload at full size, against the oracle: 64 subproblems
(n_b ~ U{500..8000}, r_b in {5, 10, 20, 40}, Gaussian bandwidth ~U[0.05, 0.2),
J_b = 20, lambda = 1e-4, rho = 1e-6, seed 0) solved by one persistent,
graph-captured launch in mixed precision (BF16 inner solves, FP64 refinement),
exactly as the benchmark runs it.

A dense solve does not fit most members (n r up to 3.2e5) and the oracle's PCG
needs a host eigendecomposition of every K (minutes in all), so the references
come from tests/golden/c5_refs.npz, written by tests/golden/make_c5_refs.py
with the oracle alone (O-dense where n r <= 8000, else the oracle's PCG of
Section 4.4 to relres 1e-12).  Per member the test checks
* status OK and the library's FP64 certificate <= TOL;
* the oracle's own residual certificate of the returned W (two-step product in
  numpy) <= 2 TOL and equal to the library's to a few digits;
* K W at ~40 stored rows against the reference rows, <= 1e-6 relative;
* a 16-probe Gaussian sketch of K (W - W_o) (seeded probes; mean square =
  ||K (W - W_o)||_F^2 in expectation), as an estimate of e_KW, <= 1e-6.
"""

import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from synth import batch_members, probe_matrices  # noqa: E402

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2603_25691_amd import cphifi as C  # noqa: E402
    from paper_2603_25691_amd.torch_api import BatchSolver, upload  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
REFS = os.path.join(HERE, "golden", "c5_refs.npz")
ROOT = os.path.dirname(HERE)
TILES = os.path.join(ROOT, "paper_2603_25691_amd", "tiles_batch_mi355x.txt")
# the refinement target of the batched benchmark
TOL = 5e-8
COUNT = 64


@pytest.fixture(scope="module")
def solved():
    refs = np.load(REFS, allow_pickle=False)
    probs, dps = [], []
    for bm in batch_members(seed=0, count=COUNT):
        probs.append(bm.problem)
        dps.append(upload(bm.problem, ldk_align=16))
    assert [p.n for p in probs] == list(refs["n"]) and [p.r for p in probs] == list(refs["r"])
    bs = BatchSolver(dps, [p.lam for p in probs], [p.rho for p in probs], TOL,
                     tile_table=TILES if os.path.exists(TILES) else None)
    Ws = [torch.empty(p.n, p.r, dtype=torch.float64, device="cuda") for p in probs]
    status, infos = bs.solve(bs.ys(), Ws)
    torch.cuda.synchronize()
    out = {"probs": probs, "refs": refs, "status": status, "infos": infos,
           "W": [W.cpu().numpy() for W in Ws]}
    bs.close()
    del dps, Ws
    torch.cuda.empty_cache()
    return out


def test_full_batch_status(solved):
    assert solved["status"] == C.OK
    assert len(solved["infos"]) == COUNT


@pytest.mark.parametrize("b", range(COUNT))
def test_full_batch_member_matches_oracle(solved, b):
    p = solved["probs"][b]
    refs = solved["refs"]
    info = solved["infos"][b]
    W = solved["W"][b]
    assert info.status == C.OK, info.as_dict()
    assert info.relres_true <= TOL
    Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
    cert = O.relres(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho, W)
    assert cert <= 2 * TOL, cert
    assert abs(cert - info.relres_true) <= 0.05 * TOL + 1e-3 * cert
    KW = p.K @ W
    rows, kw_ref = refs[f"m{b}_rows"], refs[f"m{b}_kw"]
    e_rows = np.linalg.norm(KW[rows] - kw_ref) / np.linalg.norm(kw_ref)
    assert e_rows <= 1e-6, e_rows
    G = probe_matrices((13, b), p.n, p.r, refs["sketch"].shape[1])
    d = np.einsum("knr,nr->k", G, KW) - refs["sketch"][b]
    e_sketch = float(np.sqrt(np.mean(d * d)) / refs["kw_norm"][b])
    assert e_sketch <= 1e-6, e_sketch
