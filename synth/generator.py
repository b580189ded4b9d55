"""Seeded generators for unaligned / aligned RKHS-subproblem inputs.

Every generator uses ``numpy.random.default_rng`` (PCG64) with a fixed draw
order, so a (recipe, seed) pair always yields the same bits.  Problem data are
laid out the way the library consumes them:

* design points ``t`` (n,) sorted ascending; the kernel matrix ``K`` (n, n)
  evaluated on them in float64;
* observations in time-major order as CSR: ``obs_ptr`` (n+1,), with the
  observation's time index ``obs_t``, sample index ``obs_i`` and feature index
  ``obs_j`` (all int32) and the value ``y`` (float64);
* the fixed factors of the other two modes, ``A`` (I, r) and ``B`` (J, r),
  row-major float64.

The ground truth used to synthesise ``y`` is a rank-r CP model whose time
factor is ``K @ Wstar`` (the RKHS form of the factor, Section 2 of the paper),
plus Gaussian noise scaled to 1% of the clean signal's norm.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

_ROW_CHUNK = 1024


def gaussian_kernel(d: np.ndarray, sigma: float) -> np.ndarray:
    """Gaussian (RBF) kernel of bandwidth sigma evaluated on distances d."""
    return np.exp(-(d * d) / (2.0 * sigma * sigma))


def matern32_kernel(d: np.ndarray, ell: float) -> np.ndarray:
    """Matern-3/2 kernel with length scale ell evaluated on distances d."""
    a = math.sqrt(3.0) * d / ell
    return (1.0 + a) * np.exp(-a)


def _kernel_fn(kind: str):
    if kind == "rbf":
        return gaussian_kernel
    if kind == "matern32":
        return matern32_kernel
    raise ValueError(f"unknown kernel kind {kind!r}")


def kernel_matrix(t: np.ndarray, kind: str, param: float) -> np.ndarray:
    """K(a, b) = kappa(|t_a - t_b|), filled in row chunks to bound temporaries."""
    fn = _kernel_fn(kind)
    n = t.shape[0]
    K = np.empty((n, n), dtype=np.float64)
    for r0 in range(0, n, _ROW_CHUNK):
        r1 = min(n, r0 + _ROW_CHUNK)
        K[r0:r1] = fn(np.abs(t[r0:r1, None] - t[None, :]), param)
    return K


@dataclass
class Problem:
    """One RKHS-mode subproblem instance (all arrays host numpy)."""

    name: str
    n: int
    r: int
    q: int
    I: int
    J: int
    t: np.ndarray
    K: np.ndarray
    obs_ptr: np.ndarray
    obs_t: np.ndarray
    obs_i: np.ndarray
    obs_j: np.ndarray
    y: np.ndarray
    A: np.ndarray
    B: np.ndarray
    Wstar: np.ndarray
    lam: float
    rho: float
    gamma: float
    tol: float
    maxit: int = 500
    kernel: str = "rbf"
    kernel_param: float = 0.1
    meta: Dict[str, object] = field(default_factory=dict)

    def summary(self) -> Dict[str, object]:
        return {
            "name": self.name,
            "n": self.n,
            "r": self.r,
            "q": self.q,
            "I": self.I,
            "J": self.J,
            "lambda": self.lam,
            "rho": self.rho,
            "gamma": self.gamma,
            "kernel": f"{self.kernel}({self.kernel_param})",
        }


def _csr_from_sorted_times(obs_t: np.ndarray, n: int) -> np.ndarray:
    counts = np.bincount(obs_t, minlength=n)
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    if ptr[-1] >= 2**31:
        raise ValueError("observation count exceeds int32 range")
    return ptr.astype(np.int32)


def _noisy(y0: np.ndarray, e: np.ndarray, noise: float) -> np.ndarray:
    ne = np.linalg.norm(e)
    if noise == 0.0 or ne == 0.0:
        return y0.copy()
    return y0 + noise * np.linalg.norm(y0) * (e / ne)


def make_unaligned(
    seed: int,
    I: int,
    J: int,
    m_lo: int,
    m_hi: int,
    r: int,
    kernel: str,
    kernel_param: float,
    lam: float,
    rho: float,
    tol: float,
    noise: float = 0.01,
    name: str = "unaligned",
) -> Problem:
    """Unaligned recipe: sample i is seen at m_i ~ U{m_lo..m_hi} own times.

    Draw order: m_i; the times of each sample in turn (U[0,1)); A; B; Wstar;
    the noise vector.  Every pooled time is its own design point (n = sum m_i),
    every feature is observed at every design point (q = n J), and observation
    l = s*J + j belongs to time s, sample owner(s), feature j.
    """
    rng = np.random.default_rng(seed)
    m = rng.integers(m_lo, m_hi + 1, size=I)
    times = []
    owners = []
    for i in range(I):
        times.append(rng.random(int(m[i])))
        owners.append(np.full(int(m[i]), i, dtype=np.int32))
    t_all = np.concatenate(times)
    own_all = np.concatenate(owners)
    n = t_all.shape[0]
    q = n * J
    A = rng.standard_normal((I, r))
    B = rng.standard_normal((J, r))
    Wstar = rng.standard_normal((n, r))
    e = rng.standard_normal(q)

    order = np.argsort(t_all, kind="stable")
    t = t_all[order]
    owner = own_all[order]
    K = kernel_matrix(t, kernel, kernel_param)

    obs_t = np.repeat(np.arange(n, dtype=np.int32), J)
    obs_i = np.repeat(owner, J).astype(np.int32)
    obs_j = np.tile(np.arange(J, dtype=np.int32), n)
    obs_ptr = _csr_from_sorted_times(obs_t, n)

    C = K @ Wstar
    # clean values in (time, feature) order: Y0[s, j] = sum_l C[s,l] A[owner(s),l] B[j,l]
    y0 = np.empty(q, dtype=np.float64)
    for r0 in range(0, n, 8192):
        r1 = min(n, r0 + 8192)
        blk = (C[r0:r1] * A[owner[r0:r1]]) @ B.T
        y0[r0 * J : r1 * J] = blk.reshape(-1)
    y = _noisy(y0, e, noise)
    return Problem(
        name=name, n=n, r=r, q=q, I=I, J=J, t=t, K=K, obs_ptr=obs_ptr, obs_t=obs_t,
        obs_i=obs_i, obs_j=obs_j, y=y, A=A, B=B, Wstar=Wstar, lam=lam, rho=rho,
        gamma=q / (n * I * J), tol=tol, kernel=kernel, kernel_param=kernel_param,
        meta={"seed": seed, "owner": owner, "m": m, "noise": noise},
    )


def make_aligned(
    seed: int,
    I: int,
    J: int,
    n: int,
    r: int,
    sigma: float,
    lam: float,
    rho: float,
    tol: float,
    noise: float = 0.01,
    name: str = "aligned",
) -> Problem:
    """Aligned recipe: every (time, sample, feature) entry is observed.

    Times are the uniform grid linspace(0, 1, n) with both ends; Gaussian
    kernel.  Draw order: A; B; Wstar; noise.  Observation
    l = (s*I + i)*J + j.
    """
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((I, r))
    B = rng.standard_normal((J, r))
    Wstar = rng.standard_normal((n, r))
    q = n * I * J
    e = rng.standard_normal(q)
    t = np.linspace(0.0, 1.0, n)
    K = kernel_matrix(t, "rbf", sigma)

    obs_t = np.repeat(np.arange(n, dtype=np.int32), I * J)
    obs_i = np.tile(np.repeat(np.arange(I, dtype=np.int32), J), n)
    obs_j = np.tile(np.arange(J, dtype=np.int32), n * I)
    obs_ptr = _csr_from_sorted_times(obs_t, n)

    C = K @ Wstar
    y0 = ((C[:, None, :] * A[None, :, :]).reshape(n * I, r) @ B.T).reshape(-1)
    y = _noisy(y0, e, noise)
    return Problem(
        name=name, n=n, r=r, q=q, I=I, J=J, t=t, K=K, obs_ptr=obs_ptr, obs_t=obs_t,
        obs_i=obs_i, obs_j=obs_j, y=y, A=A, B=B, Wstar=Wstar, lam=lam, rho=rho,
        gamma=1.0, tol=tol, kernel="rbf", kernel_param=sigma,
        meta={"seed": seed, "noise": noise},
    )


def make_small(
    seed: int,
    n: int,
    I: int,
    J: int,
    r: int,
    q: int,
    kernel: str = "rbf",
    kernel_param: float = 0.15,
    lam: float = 1e-2,
    rho: float = 1e-6,
    tol: float = 1e-10,
    noise: float = 0.01,
    name: str = "small",
) -> Problem:
    """General unaligned instance with a random observation set.

    Draw order: n design times U[0,1); q distinct entries of the n x I x J
    grid drawn without replacement; A; B; Wstar; noise.  Segments may be empty
    or of very different lengths, which exercises the ragged path.
    """
    if q > n * I * J:
        raise ValueError("q exceeds the number of tensor entries")
    rng = np.random.default_rng(seed)
    t = np.sort(rng.random(n))
    lin = np.sort(rng.choice(n * I * J, size=q, replace=False))
    A = rng.standard_normal((I, r))
    B = rng.standard_normal((J, r))
    Wstar = rng.standard_normal((n, r))
    e = rng.standard_normal(q)
    obs_t = (lin // (I * J)).astype(np.int32)
    rem = lin % (I * J)
    obs_i = (rem // J).astype(np.int32)
    obs_j = (rem % J).astype(np.int32)
    obs_ptr = _csr_from_sorted_times(obs_t, n)
    K = kernel_matrix(t, kernel, kernel_param)
    C = K @ Wstar
    y0 = np.einsum("ql,ql,ql->q", C[obs_t], A[obs_i], B[obs_j])
    y = _noisy(y0, e, noise)
    return Problem(
        name=name, n=n, r=r, q=q, I=I, J=J, t=t, K=K, obs_ptr=obs_ptr, obs_t=obs_t,
        obs_i=obs_i, obs_j=obs_j, y=y, A=A, B=B, Wstar=Wstar, lam=lam, rho=rho,
        gamma=q / (n * I * J), tol=tol, kernel=kernel, kernel_param=kernel_param,
        meta={"seed": seed, "noise": noise},
    )


def drop_observations(p: Problem, keep_frac: float, seed: int) -> Problem:
    """Keep a random subset of the observations (draw: one U[0,1) per observation)."""
    rng = np.random.default_rng(seed)
    keep = rng.random(p.q) < keep_frac
    obs_t = p.obs_t[keep]
    q = int(obs_t.shape[0])
    return Problem(
        name=p.name + f"-keep{keep_frac:g}", n=p.n, r=p.r, q=q, I=p.I, J=p.J, t=p.t,
        K=p.K, obs_ptr=_csr_from_sorted_times(obs_t, p.n), obs_t=obs_t,
        obs_i=p.obs_i[keep], obs_j=p.obs_j[keep], y=p.y[keep], A=p.A, B=p.B,
        Wstar=p.Wstar, lam=p.lam, rho=p.rho, gamma=q / (p.n * p.I * p.J), tol=p.tol,
        maxit=p.maxit, kernel=p.kernel, kernel_param=p.kernel_param,
        meta=dict(p.meta, keep_frac=keep_frac, keep_seed=seed),
    )


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def config_c1(seed: int = 0) -> Problem:
    """Small plain FP64 unaligned case: I=20, J=10, m_i~U{5..15}, RBF 0.1, r=5."""
    return make_unaligned(seed, I=20, J=10, m_lo=5, m_hi=15, r=5, kernel="rbf",
                          kernel_param=0.1, lam=1e-3, rho=1e-6, tol=1e-10, name="c1")


def config_c2(r: int = 10, seed: int = 0, I: int = 500, J: int = 100) -> Problem:
    """Aligned FP64 case: n=200 uniform grid shared by all samples, RBF 0.05."""
    return make_aligned(seed, I=I, J=J, n=200, r=r, sigma=0.05, lam=1e-4, rho=1e-6,
                        tol=1e-10, name=f"c2-r{r}")


def config_c3(seed: int = 0, I: int = 1000, J: int = 200, r: int = 40) -> Problem:
    """Large unaligned FP64 case: m_i~U{10..50}, Matern-3/2 length 0.1, r=40.

    With the default I=1000, J=200 this gives n ~ 30,000 design points and
    q ~ 6e6 observations; smaller I/J keep the same recipe at a reduced size.
    """
    return make_unaligned(seed, I=I, J=J, m_lo=10, m_hi=50, r=r, kernel="matern32",
                          kernel_param=0.1, lam=1e-4, rho=1e-6, tol=1e-8,
                          name=f"c3-I{I}-J{J}-r{r}")


@dataclass
class BatchMember:
    problem: Problem
    sigma: float


def batch_members(seed: int = 0, count: int = 64, n_lo: int = 500, n_hi: int = 8000,
                  ranks=(5, 10, 20, 40), J: int = 20, lam: float = 1e-4,
                  rho: float = 1e-6, tol: float = 1e-7):
    """Batched recipe, one member at a time (a generator, so a large batch
    never holds every kernel matrix in host memory at once).

    Member b draws from its own child seed of SeedSequence(seed).spawn(count),
    in order: n_b ~ U{n_lo..n_hi}; r_b uniform over `ranks`; RBF bandwidth
    sigma_b ~ U[0.05, 0.2); the n_b times U[0,1); the owner sample of each time
    ~ U{0..I_b-1} with I_b = ceil(n_b/30); A; B; Wstar; noise.  J_b = J.
    """
    for b, child in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.default_rng(child)
        n = int(rng.integers(n_lo, n_hi + 1))
        r = int(ranks[int(rng.integers(0, len(ranks)))])
        sigma = float(rng.uniform(0.05, 0.2))
        I = int(math.ceil(n / 30))
        t_raw = rng.random(n)
        own_raw = rng.integers(0, I, size=n).astype(np.int32)
        A = rng.standard_normal((I, r))
        B = rng.standard_normal((J, r))
        Wstar = rng.standard_normal((n, r))
        q = n * J
        e = rng.standard_normal(q)
        order = np.argsort(t_raw, kind="stable")
        t = t_raw[order]
        owner = own_raw[order]
        K = kernel_matrix(t, "rbf", sigma)
        obs_t = np.repeat(np.arange(n, dtype=np.int32), J)
        obs_i = np.repeat(owner, J).astype(np.int32)
        obs_j = np.tile(np.arange(J, dtype=np.int32), n)
        C = K @ Wstar
        y0 = ((C * A[owner]) @ B.T).reshape(-1)
        y = _noisy(y0, e, 0.01)
        p = Problem(
            name=f"batch{b}", n=n, r=r, q=q, I=I, J=J, t=t, K=K,
            obs_ptr=_csr_from_sorted_times(obs_t, n), obs_t=obs_t, obs_i=obs_i,
            obs_j=obs_j, y=y, A=A, B=B, Wstar=Wstar, lam=lam, rho=rho,
            gamma=q / (n * I * J), tol=tol, kernel="rbf", kernel_param=sigma,
            meta={"seed": seed, "member": b, "owner": owner},
        )
        yield BatchMember(problem=p, sigma=sigma)


def make_batch(seed: int = 0, count: int = 64, **kw) -> List[BatchMember]:
    """All members of the batched recipe (see batch_members)."""
    return list(batch_members(seed=seed, count=count, **kw))


def config_c5(seed: int = 0, count: int = 64, **kw) -> List[BatchMember]:
    return make_batch(seed=seed, count=count, **kw)


def make_paper_standin(shape=(199, 449, 151), sigmas=(4.0, 4.0, 3.0), q: int = 50000,
                       r: int = 10, seed: int = 0, lam: float = 0.1, rho: float = 1e-6,
                       tol: float = 1e-6, noise: float = 0.01,
                       name: Optional[str] = None) -> Problem:
    """Shape-only stand-in for the paper's unaligned 3-way experiments.

    All three modes are RKHS modes on integer grids 1..n_k with Gaussian
    kernels of the given bandwidths; the ground-truth factors are K_k Wk* with
    Wk* ~ N(0,1).  q entries are drawn uniformly without replacement from the
    full grid.  The returned subproblem is the one for the last mode, with the
    first two modes' factors as A and B.  Draw order: W1*, W2*, W3*, the
    entry set, noise.
    """
    n1, n2, n3 = shape
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((n1, r))
    W2 = rng.standard_normal((n2, r))
    W3 = rng.standard_normal((n3, r))
    lin = rng.choice(n1 * n2 * n3, size=q, replace=False)
    e = rng.standard_normal(q)
    grids = [np.arange(1, nk + 1, dtype=np.float64) for nk in shape]
    K1 = kernel_matrix(grids[0], "rbf", sigmas[0])
    K2 = kernel_matrix(grids[1], "rbf", sigmas[1])
    K3 = kernel_matrix(grids[2], "rbf", sigmas[2])
    A1, A2, A3 = K1 @ W1, K2 @ W2, K3 @ W3
    # linear index in (i1, i2, i3) with i3 fastest; reorder time-major (by i3)
    i1 = lin // (n2 * n3)
    i2 = (lin // n3) % n2
    i3 = lin % n3
    order = np.lexsort((i2, i1, i3))
    i1, i2, i3, e = i1[order], i2[order], i3[order], e[order]
    y0 = np.einsum("ql,ql,ql->q", A1[i1], A2[i2], A3[i3])
    y = _noisy(y0, e, noise)
    obs_t = i3.astype(np.int32)
    return Problem(
        name=name or f"standin-{n1}x{n2}x{n3}-r{r}", n=n3, r=r, q=q, I=n1, J=n2,
        t=grids[2], K=K3, obs_ptr=_csr_from_sorted_times(obs_t, n3), obs_t=obs_t,
        obs_i=i1.astype(np.int32), obs_j=i2.astype(np.int32), y=y, A=A1, B=A2,
        Wstar=W3, lam=lam, rho=rho, gamma=q / (n1 * n2 * n3), tol=tol, maxit=75,
        kernel="rbf", kernel_param=sigmas[2], meta={"seed": seed, "shape": shape},
    )


# --------------------------------------------------------------------------
# Seeded sampling helpers for checks at full size (random numbers only)
# --------------------------------------------------------------------------

def sample_rows(seed, n: int, count: int) -> np.ndarray:
    """Sorted distinct row indices in [0, n): the first and last row plus
    count - 2 drawn without replacement (fewer when n is small)."""
    rng = np.random.default_rng(seed)
    inner = np.arange(1, n - 1)
    k = max(0, min(count - 2, inner.shape[0]))
    pick = rng.choice(inner, size=k, replace=False) if k > 0 else np.zeros(0, dtype=np.int64)
    rows = np.concatenate([[0], pick, [n - 1]]) if n > 1 else np.array([0])
    return np.unique(rows.astype(np.int64))


def probe_matrices(seed, n: int, r: int, count: int) -> np.ndarray:
    """count independent N(0, 1) matrices of shape (n, r), stacked."""
    return np.random.default_rng(seed).standard_normal((count, n, r))


# --------------------------------------------------------------------------
# Whole-tensor stand-ins for the alternating optimisation (every mode RKHS)
# --------------------------------------------------------------------------

@dataclass
class AlsProblem:
    """A 3-way tensor observed on `coords` (q x 3, int32), every mode an RKHS
    mode with kernel matrix Ks[k] on the integer grid 1..n_k; W0s are the
    seeded starting weights, Wstar the ground truth."""
    name: str
    shape: tuple
    r: int
    Ks: List[np.ndarray]
    coords: np.ndarray
    y: np.ndarray
    W0s: List[np.ndarray]
    Wstar: List[np.ndarray]
    lams: List[float]
    rho: float
    tol: float
    maxit: int


def make_als_problem(shape=(199, 449, 151), sigmas=(4.0, 4.0, 3.0), q: int = 50000,
                     r: int = 10, seed: int = 0, lam: float = 0.1, rho: float = 1e-6,
                     tol: float = 1e-6, maxit: int = 75, noise: float = 0.01,
                     init_scale: float = 0.1, name: Optional[str] = None,
                     finite=(False, False, False)) -> AlsProblem:
    """Shape-only stand-in for the paper's unaligned vortex / Miranda runs:
    Gaussian kernels of the given bandwidths on integer grids, ground-truth
    factors K_k Wk* with Wk* ~ N(0, 1), q entries drawn uniformly without
    replacement (sorted by linear index), 1 % relative noise, and starting
    weights init_scale * N(0, 1).  Draw order: W1*, W2*, W3*, the entry set,
    noise, W1_0, W2_0, W3_0.  A mode flagged in `finite` is a plain
    finite-dimensional mode: no kernel (Ks[k] is None) and its ground-truth
    factor is Wk* itself."""
    rng = np.random.default_rng(seed)
    Wstar = [rng.standard_normal((nk, r)) for nk in shape]
    n1, n2, n3 = shape
    lin = np.sort(rng.choice(n1 * n2 * n3, size=q, replace=False))
    e = rng.standard_normal(q)
    W0s = [init_scale * rng.standard_normal((nk, r)) for nk in shape]
    Ks = [None if fin else kernel_matrix(np.arange(1, nk + 1, dtype=np.float64), "rbf", sg)
          for nk, sg, fin in zip(shape, sigmas, finite)]
    coords = np.stack([lin // (n2 * n3), (lin // n3) % n2, lin % n3], axis=1).astype(np.int32)
    A = [W if K is None else K @ W for K, W in zip(Ks, Wstar)]
    y0 = np.sum(A[0][coords[:, 0]] * A[1][coords[:, 1]] * A[2][coords[:, 2]], axis=1)
    y = _noisy(y0, e, noise)
    return AlsProblem(name=name or f"als-{n1}x{n2}x{n3}-r{r}", shape=tuple(shape), r=r, Ks=Ks,
                      coords=coords, y=y, W0s=W0s, Wstar=Wstar, lams=[lam] * 3, rho=rho,
                      tol=tol, maxit=maxit)
