"""Write tests/golden/c5_refs.npz: oracle reference solutions of the 64 members
of the batched workload (synth.batch_members(seed=0, count=64): n_b ~ U{500..8000},
r_b in {5, 10, 20, 40}, Gaussian kernels of bandwidth ~U[0.05, 0.2), J_b = 20,
lambda = 1e-4, rho = 1e-6).

Each member's system is eq. (unaligned-infinite-1) of Section 4.1.  It is solved
by the oracle only: the dense normal-equation Cholesky solve (Section 4.2) where
n r <= 8000, else the oracle's PCG of Section 4.4 (two-step product, eq. fx
preconditioner from numpy's eigendecomposition of K) to relative residual 1e-12.
A full solution is too large to keep (sum n_b r_b ~ 5e6 values), so per member
the file holds what a check at this size needs:

* ``m{b}_rows`` / ``m{b}_kw``: K W_o at ~40 seeded rows (synth.sample_rows with
  seed (11, b); always the first and the last row);
* ``sketch[b]``: <G_k, K W_o> for 16 seeded N(0,1) probes G_k
  (synth.probe_matrices with seed (13, b)), so that the mean square of
  <G_k, K (W - W_o)> estimates ||K (W - W_o)||_F^2;
* ``kw_norm[b]`` = ||K W_o||_F, ``cert[b]`` = the oracle's residual certificate
  of W_o, ``method[b]`` (0 dense, 1 PCG), ``iters[b]``, ``n[b]``, ``r[b]``.

Usage: python tests/golden/make_c5_refs.py [--count 64] [--out PATH]
(about 10-20 minutes on 8 host cores; imports only oracle/ and synth/).
"""

from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from synth import batch_members, probe_matrices, sample_rows  # noqa: E402

DENSE_MAX_NR = 8000
ROWS = 40
PROBES = 16
TOL = 1e-12


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "c5_refs.npz"))
    a = ap.parse_args(argv)
    out = {}
    ns, rs, norms, certs, methods, iters, sketches = [], [], [], [], [], [], []
    t_all = time.time()
    for b, bm in enumerate(batch_members(seed=0, count=a.count)):
        p = bm.problem
        t0 = time.time()
        Zhat = O.khatri_rao_rows(p.A, p.B, p.obs_i, p.obs_j)
        if p.n * p.r <= DENSE_MAX_NR:
            W = O.solve_dense(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho)
            method, its = 0, 0
        else:
            res = O.solve_pcg(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho, p.gamma,
                              O.gram_V(p.A, p.B), TOL, 3000, eigK=O.kernel_eig(p.K))
            if not res.converged:
                raise RuntimeError(f"member {b}: oracle PCG did not reach {TOL}")
            W, method, its = res.X, 1, res.iters
        KW = p.K @ W
        rows = sample_rows((11, b), p.n, ROWS)
        G = probe_matrices((13, b), p.n, p.r, PROBES)
        out[f"m{b}_rows"] = rows
        out[f"m{b}_kw"] = KW[rows]
        sketches.append(np.einsum("knr,nr->k", G, KW))
        ns.append(p.n)
        rs.append(p.r)
        norms.append(float(np.linalg.norm(KW)))
        certs.append(O.relres(p.K, Zhat, p.obs_t, p.y, p.lam, p.rho, W))
        methods.append(method)
        iters.append(its)
        print(f"member {b}: n={p.n} r={p.r} {'dense' if method == 0 else 'pcg'} its={its} "
              f"cert={certs[-1]:.2e} ({time.time() - t0:.1f} s)", flush=True)
    out.update(n=np.array(ns), r=np.array(rs), kw_norm=np.array(norms), cert=np.array(certs),
               method=np.array(methods), iters=np.array(iters), sketch=np.array(sketches))
    np.savez_compressed(a.out, **out)
    print(f"wrote {a.out} in {time.time() - t_all:.0f} s", flush=True)


if __name__ == "__main__":
    main()
