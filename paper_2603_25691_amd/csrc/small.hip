// Persistent multi-workgroup FP64 PCG for small subproblems (Section 4.4).
//
// For a small UI subproblem (K of a few hundred points, a few thousand
// observations) every step of a PCG iteration is a few microseconds of work,
// and a multi-kernel iteration spends its time in the minimum duration of
// each of its ~11 dependent launches.  Here the whole iteration loop -- the
// two-step product (Section 4.4.1, eqs. vl, yhat1), the eq. (fx)
// preconditioner (Section 4.4.2) and the textbook PCG recurrence -- runs in
// ONE launch of up to 128 co-resident workgroups that meet at bounded grid
// barriers.  Each wave owns rows s = w, w + W, ... (W waves in the grid) of
// every n x r vector, and a step is done row by row:
//  * products Y(s,:) = sum_k M(s,k) X(k,:) with M one of K (symmetric), U^T
//    (the stored eigenvector rows) and U (the transposed copy), so row s of M
//    is contiguous: lanes stride over k, each lane keeps r running sums, and a
//    butterfly over the 64 lanes adds them (every lane ends with the same
//    bits);
//  * the gather-scatter of a row runs over its time point's observations, one
//    per lane: x_l = Xhat(s,:) . Zhat(l,:) (eq. vl), then x_l Zhat(l,:) summed
//    over the lanes (eq. yhat1);
//  * the r x r middle step of eq. (fx) per row, lanes over the columns.
// A vector that every row reads in the next step and that the recurrence
// updates in place (the residual and the search direction) is kept in two
// buffers and its update is formed on the fly by the reading product, so an
// iteration needs four barriers: after the gather, after p^T q, after the
// residual update and first preconditioner step, after r^T z.  Dot products
// are summed per workgroup in a fixed order, then over the workgroups in a
// fixed order by every workgroup alike, so all take the same decisions and the
// result does not depend on the schedule.  Every barrier wait is bounded: a
// workgroup that waits too long raises an error flag on which all leave.
// The setup (V, eig(V), D), the right-hand side and the FP64 certificate stay
// the library's ordinary kernels.
#include "cphifi_internal.h"
#include "small.h"

#include <cmath>

namespace cphifi {
namespace {

constexpr int kT = kSmallThreads;
constexpr int kWaves = kT / 64;
constexpr int kSmallGrid = 64;  // workgroups of a launch (at most kSmallMaxWG)
static_assert(kSmallGrid <= kSmallMaxWG, "flags and partials sized for kSmallMaxWG");
// k steps per lane whose loads are issued together (fewer for wide rows, whose
// r running sums and staged rows fill the registers)
template <int RC>
constexpr int k_steps() {
  return RC <= 8 ? 4 : RC <= 16 ? 2 : 1;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Bounded grid barrier on per-workgroup arrival flags: thread 0 releases the
// workgroup's writes and publishes the barrier count in its own line; the
// first wave waits until every workgroup's count has reached it (one load per
// lane per poll), then thread 0 acquires the other workgroups' writes.  With
// no shared counter the arrivals do not queue on one atomic (at 52
// workgroups 3.2 against 4.3 us per barrier).  False when a wait timed out here
// or in another workgroup.
__device__ __forceinline__ bool grid_sync(SmallCtl* ctl, uint32_t epoch, int64_t spin_limit,
                                          int* s_ok) {
  __syncthreads();
  if (threadIdx.x < 64) {
    if (threadIdx.x == 0) {
      // release this workgroup's writes device-wide (a release fence: the L2
      // write-back only, no invalidation)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&ctl->flag[blockIdx.x * 16], epoch, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    int ok = 1;
    for (int64_t spin = 0;; ++spin) {
      bool mine = true;
      for (int g = threadIdx.x; g < (int)gridDim.x; g += 64)
        mine = mine && __hip_atomic_load(&ctl->flag[g * 16], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) >= epoch;
      if (__all(mine)) break;
      if ((spin & 63) == 63 &&
          __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        ok = 0;
        break;
      }
      if (spin >= spin_limit) {
        if (threadIdx.x == 0)
          __hip_atomic_store(&ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (threadIdx.x == 0) {
      // acquire the other workgroups' writes (an acquire fence: invalidation only)
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      *s_ok = ok;
    }
  }
  __syncthreads();
  return *s_ok != 0;
}

// acc(c) = sum_k M[row ldm + k] X(k, c), X(k,:) = X1(k,:) + coef X2(k,:) when X2
// is given (formed with the same fma as the owner's stored copy); every lane
// returns the full sums.
template <int RC>
__device__ __forceinline__ void row_product(const double* __restrict__ M, int64_t ldm, int64_t row,
                                            int n, int r, const double* __restrict__ X1,
                                            const double* __restrict__ X2, double coef,
                                            double (&acc)[RC]) {
  constexpr int kKU = k_steps<RC>();
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < RC; ++c) acc[c] = 0.0;
  const double* mrow = M + row * ldm;
  for (int k0 = lane; k0 < n; k0 += 64 * kKU) {
    double m[kKU];
    double x[kKU][RC];
#pragma unroll
    for (int u = 0; u < kKU; ++u) {
      const int k = k0 + 64 * u;
      const bool on = k < n;
      const int kc = on ? k : 0;
      m[u] = on ? mrow[kc] : 0.0;
      const double* x1 = X1 + (int64_t)kc * r;
      const double* x2 = X2 != nullptr ? X2 + (int64_t)kc * r : nullptr;
#pragma unroll
      for (int c = 0; c < RC; ++c) {
        double v = 0.0;
        if (c < r) v = x2 != nullptr ? fma(coef, x2[c], x1[c]) : x1[c];
        x[u][c] = v;
      }
    }
#pragma unroll
    for (int u = 0; u < kKU; ++u)
#pragma unroll
      for (int c = 0; c < RC; ++c) acc[c] = fma(m[u], x[u][c], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < RC; ++c) acc[c] = c < r ? wave_sum(acc[c]) : 0.0;
}

// Yhat1(s,:) from Xhat(s,:) = xh: eqs. (vl), (yhat1) over the observations of
// time point s, one per lane.
template <int RC>
__device__ __forceinline__ void row_gather(const SmallArgs& a, int64_t s, const double (&xh)[RC],
                                           double (&acc)[RC]) {
  const int lane = threadIdx.x & 63, r = a.r;
#pragma unroll
  for (int c = 0; c < RC; ++c) acc[c] = 0.0;
  const int32_t beg = a.obs_ptr[s], end = a.obs_ptr[s + 1];
  for (int32_t l = beg + lane; l < end; l += 64) {
    double z[RC];
    if (a.Zhat != nullptr) {
      const double* zr = a.Zhat + (int64_t)l * r;
#pragma unroll
      for (int c = 0; c < RC; ++c) z[c] = c < r ? zr[c] : 0.0;
    } else {
      const double* za = a.A + (int64_t)a.obs_i[l] * r;
      const double* zb = a.B + (int64_t)a.obs_j[l] * r;
#pragma unroll
      for (int c = 0; c < RC; ++c) z[c] = c < r ? za[c] * zb[c] : 0.0;
    }
    double x = 0.0;
#pragma unroll
    for (int c = 0; c < RC; ++c) x = fma(xh[c], z[c], x);
#pragma unroll
    for (int c = 0; c < RC; ++c) acc[c] = fma(x, z[c], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < RC; ++c) acc[c] = c < r ? wave_sum(acc[c]) : 0.0;
}

// The Zhat rows of time point s's observations, one per lane (zero past the
// segment); false when the segment is longer than a wave.
template <int RC>
__device__ __forceinline__ bool row_obs(const SmallArgs& a, int64_t s, double (&z)[RC]) {
  const int lane = threadIdx.x & 63, r = a.r;
  const int32_t beg = a.obs_ptr[s], end = a.obs_ptr[s + 1];
#pragma unroll
  for (int c = 0; c < RC; ++c) z[c] = 0.0;
  if (end - beg > 64) return false;
  const int32_t l = beg + lane;
  if (l < end) {
    if (a.Zhat != nullptr) {
      const double* zr = a.Zhat + (int64_t)l * r;
#pragma unroll
      for (int c = 0; c < RC; ++c) z[c] = c < r ? zr[c] : 0.0;
    } else {
      const double* za = a.A + (int64_t)a.obs_i[l] * r;
      const double* zb = a.B + (int64_t)a.obs_j[l] * r;
#pragma unroll
      for (int c = 0; c < RC; ++c) z[c] = c < r ? za[c] * zb[c] : 0.0;
    }
  }
  return true;
}

// row_gather with the observation rows already in registers (the same
// arithmetic: lanes past the segment add zeros).
template <int RC>
__device__ __forceinline__ void row_gather_reg(int r, const double (&z)[RC],
                                               const double (&xh)[RC], double (&acc)[RC]) {
  double x = 0.0;
#pragma unroll
  for (int c = 0; c < RC; ++c) x = fma(xh[c], z[c], x);
#pragma unroll
  for (int c = 0; c < RC; ++c) acc[c] = c < r ? wave_sum(fma(x, z[c], 0.0)) : 0.0;
}

// T2(s,:) = ((T1(s,:) U_V) had D(s,:)) U_V^T, the middle step of eq. (fx);
// returns lane c's entry (c < r).
template <int RC>
__device__ __forceinline__ double row_mid(const SmallArgs& a, int64_t s, const double (&t1)[RC]) {
  const int lane = threadIdx.x & 63, r = a.r;
  double w = 0.0;
  if (lane < r) {
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < RC; ++i)
      if (i < r) v = fma(t1[i], a.UV[i * r + lane], v);
    w = v * a.D[s * r + lane];
  }
  double t = 0.0;
  for (int j = 0; j < r; ++j) {
    const double wj = __shfl(w, j, 64);
    if (lane < r) t = fma(wj, a.UV[lane * r + j], t);
  }
  return t;
}

// Sum of v over the workgroup in a fixed order, written to dst[blockIdx.x].
__device__ __forceinline__ void wg_partial(double v, double* dst, double* s_red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += s_red[w];
    dst[blockIdx.x] = t;
  }
  __syncthreads();
}

// Sum of the workgroups' partials, in the same order in every wave.
__device__ __forceinline__ double grid_total(const double* src) {
  double v = 0.0;
  for (int i = threadIdx.x & 63; i < (int)gridDim.x; i += 64) v += src[i];
  return wave_sum(v);
}

template <int RC>
__global__ __launch_bounds__(kT) void small_pcg_kernel(SmallArgs a) {
  __shared__ double s_red[kWaves];
  __shared__ int s_ok;
  SmallCtl* ctl = (SmallCtl*)a.scratch;
  double* part = (double*)((char*)a.scratch + sizeof(SmallCtl));
  double* p_pq = part;
  double* p_rr = part + kSmallMaxWG;
  double* p_rz = part + 2 * kSmallMaxWG;
  double* p_bb = part + 3 * kSmallMaxWG;
  const int n = (int)a.n, r = a.r;
  const int lane = threadIdx.x & 63;
  const int w0 = blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int nw = gridDim.x * kWaves;
  const bool lc = lane < r;  // the lane that stores column `lane` of a row
  uint32_t nbar = 0;
  bool ok = true;
  auto sync = [&]() {
    ++nbar;
    ok = ok && grid_sync(ctl, nbar, a.spin_limit, &s_ok);
    return ok;
  };
  auto at = [&](double* v, int64_t s) { return v + s * r + lane; };
  auto atc = [&](const double* v, int64_t s) { return v[s * r + lane]; };
  double acc[RC], t[RC];
  // The observation rows of the wave's first two rows stay in registers for
  // the whole solve when their segments fit a wave: the gather then reads
  // only Xhat.
  // (two rows at r <= 8, one at r <= 16: wider rows would crowd the registers)
  constexpr int kCache = RC <= 8 ? 2 : RC <= 16 ? 1 : 0;
  double zc0[RC], zc1[RC];
  bool c0 = false, c1 = false;
  if (kCache >= 1 && w0 < n) c0 = row_obs<RC>(a, w0, zc0);
  if (kCache >= 2 && w0 + nw < n) c1 = row_obs<RC>(a, w0 + nw, zc1);
  auto gather = [&](int j, int64_t s, const double (&xh)[RC], double (&out)[RC]) {
    if (kCache >= 1 && j == 0 && c0)
      row_gather_reg<RC>(r, zc0, xh, out);
    else if (kCache >= 2 && j == 1 && c1)
      row_gather_reg<RC>(r, zc1, xh, out);
    else
      row_gather<RC>(a, s, xh, out);
  };

  // x0 and r0 = b - A x0
  double bbl = 0.0, rrl = 0.0;
  if (a.warm) {
    int j = 0;
    for (int64_t s = w0; s < n; s += nw, ++j) {
      row_product<RC>(a.K, a.ldk, s, n, r, a.X, nullptr, 0.0, acc);
      gather(j, s, acc, t);
#pragma unroll
      for (int c = 0; c < RC; ++c)
        if (c < r && lane == c) {
          a.Xh[s * r + c] = acc[c];
          a.Y1[s * r + c] = t[c];
        }
    }
    if (!sync()) goto out;
    for (int64_t s = w0; s < n; s += nw) {
      row_product<RC>(a.K, a.ldk, s, n, r, a.Y1, nullptr, 0.0, acc);
#pragma unroll
      for (int c = 0; c < RC; ++c)
        if (c < r && lane == c) {
          const int64_t e = s * r + c;
          const double q = acc[c] + a.lam * a.Xh[e] + a.rho * a.X[e];
          const double v = a.b[e] - q;
          a.R0[e] = v;
          rrl += v * v;
          bbl += a.b[e] * a.b[e];
        }
    }
  } else {
    for (int64_t s = w0; s < n; s += nw)
      if (lc) {
        const double v = atc(a.b, s);
        *at(a.X, s) = 0.0;
        *at(a.R0, s) = v;
        bbl += v * v;
      }
    rrl = bbl;
  }
  for (int64_t s = w0; s < n; s += nw)
    if (lc) *at(a.P1, s) = 0.0;  // the "previous" direction of the first iteration
  wg_partial(bbl, p_bb, s_red);
  wg_partial(rrl, p_rr, s_red);
  {
    if (!sync()) goto out;
    const double bb = grid_total(p_bb);
    double rr = grid_total(p_rr);
    const double tol2 = a.tol * a.tol * bb;
    if (a.hist != nullptr && blockIdx.x == 0 && threadIdx.x == 0)
      a.hist[0] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    int status = CPHIFI_NOT_CONVERGED, it = 0;
    double rz = 0.0, beta = 0.0;
    if (!isfinite(bb) || !isfinite(rr)) {
      status = CPHIFI_NUMERIC;
    } else if (bb == 0.0 || rr <= tol2) {
      status = CPHIFI_OK;
    } else {
      // z0 = M^{-1} r0 (eq. fx), rz = r0 . z0
      double rzl = 0.0;
      if (a.precond) {
        for (int64_t s = w0; s < n; s += nw) {
          row_product<RC>(a.UK, a.ldk, s, n, r, a.R0, nullptr, 0.0, acc);
          const double v = row_mid<RC>(a, s, acc);
          if (lc) *at(a.T2, s) = v;
        }
        if (!sync()) goto out;
        for (int64_t s = w0; s < n; s += nw) {
          row_product<RC>(a.UKT, a.ldk, s, n, r, a.T2, nullptr, 0.0, acc);
#pragma unroll
          for (int c = 0; c < RC; ++c)
            if (c < r && lane == c) {
              a.Z[s * r + c] = acc[c];
              rzl += a.R0[s * r + c] * acc[c];
            }
        }
      } else {
        for (int64_t s = w0; s < n; s += nw)
          if (lc) {
            const double v = atc(a.R0, s);
            *at(a.Z, s) = v;
            rzl += v * v;
          }
      }
      wg_partial(rzl, p_rz, s_red);
      if (!sync()) goto out;
      rz = grid_total(p_rz);
      if (!(rz > 0.0) || !isfinite(rz)) status = isfinite(rz) ? CPHIFI_BREAKDOWN : CPHIFI_NUMERIC;
    }
    while (status == CPHIFI_NOT_CONVERGED && it < a.maxit) {
      double* Pc = (it & 1) ? a.P1 : a.P0;   // this iteration's direction
      double* Pp = (it & 1) ? a.P0 : a.P1;   // the previous one
      double* Ro = (it & 1) ? a.R1 : a.R0;   // residual before the update
      double* Rn = (it & 1) ? a.R0 : a.R1;   // and after it
      // Xhat = K p with p = z + beta p_prev formed on the fly; Yhat1 = G(Xhat)
      int j = 0;
      for (int64_t s = w0; s < n; s += nw, ++j) {
        row_product<RC>(a.K, a.ldk, s, n, r, a.Z, Pp, beta, acc);
        gather(j, s, acc, t);
#pragma unroll
        for (int c = 0; c < RC; ++c)
          if (c < r && lane == c) {
            const int64_t e = s * r + c;
            Pc[e] = fma(beta, Pp[e], a.Z[e]);
            a.Xh[e] = acc[c];
            a.Y1[e] = t[c];
          }
      }
      if (!sync()) goto out;
      // q = K Yhat1 + lambda Xhat + rho p, p . q
      double pql = 0.0;
      for (int64_t s = w0; s < n; s += nw) {
        row_product<RC>(a.K, a.ldk, s, n, r, a.Y1, nullptr, 0.0, acc);
#pragma unroll
        for (int c = 0; c < RC; ++c)
          if (c < r && lane == c) {
            const int64_t e = s * r + c;
            const double q = acc[c] + a.lam * a.Xh[e] + a.rho * Pc[e];
            a.Q[e] = q;
            pql += Pc[e] * q;
          }
      }
      wg_partial(pql, p_pq, s_red);
      if (!sync()) goto out;
      const double pq = grid_total(p_pq);
      if (!(pq > 0.0) || !isfinite(pq)) {
        status = isfinite(pq) ? CPHIFI_BREAKDOWN : CPHIFI_NUMERIC;
        break;
      }
      const double alpha = rz / pq;
      // x += alpha p, r_new = r - alpha q, ||r_new||^2; first step of eq. fx
      // on r_new (formed on the fly from r and q)
      double rrn = 0.0, rzn = 0.0;
      for (int64_t s = w0; s < n; s += nw) {
        if (a.precond) row_product<RC>(a.UK, a.ldk, s, n, r, Ro, a.Q, -alpha, acc);
        const double mid = a.precond ? row_mid<RC>(a, s, acc) : 0.0;
        if (lc) {
          const int64_t e = s * r + lane;
          a.X[e] += alpha * Pc[e];
          const double v = fma(-alpha, a.Q[e], Ro[e]);
          Rn[e] = v;
          rrn += v * v;
          if (a.precond) {
            a.T2[e] = mid;
          } else {
            a.Z[e] = v;
            rzn += v * v;
          }
        }
      }
      wg_partial(rrn, p_rr, s_red);
      if (!a.precond) wg_partial(rzn, p_rz, s_red);
      if (!sync()) goto out;
      rr = grid_total(p_rr);
      ++it;
      if (a.hist != nullptr && blockIdx.x == 0 && threadIdx.x == 0 && it < a.hist_len)
        a.hist[it] = sqrt(rr / bb);
      if (!isfinite(rr)) {
        status = CPHIFI_NUMERIC;
        break;
      }
      if (rr <= tol2) {
        status = CPHIFI_OK;
        break;
      }
      if (it >= a.maxit) break;
      if (a.precond) {
        // z = U T2 (eq. fx), r . z
        for (int64_t s = w0; s < n; s += nw) {
          row_product<RC>(a.UKT, a.ldk, s, n, r, a.T2, nullptr, 0.0, acc);
#pragma unroll
          for (int c = 0; c < RC; ++c)
            if (c < r && lane == c) {
              a.Z[s * r + c] = acc[c];
              rzn += Rn[s * r + c] * acc[c];
            }
        }
        wg_partial(rzn, p_rz, s_red);
        if (!sync()) goto out;
      }
      const double rz_new = grid_total(p_rz);
      if (!(rz_new > 0.0) || !isfinite(rz_new)) {
        status = isfinite(rz_new) ? CPHIFI_BREAKDOWN : CPHIFI_NUMERIC;
        break;
      }
      beta = rz_new / rz;
      rz = rz_new;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.out->iters = it;
      a.out->status = status;
      a.out->rr = rr;
      a.out->bb = bb;
    }
    return;
  }
out:
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.out->iters = 0;
    a.out->status = kSmallTimeout;
    a.out->rr = 0.0;
    a.out->bb = 0.0;
  }
}

__global__ __launch_bounds__(256) void small_reset_kernel(SmallCtl* ctl) {
  for (int i = threadIdx.x; i < kSmallMaxWG * 16; i += blockDim.x) ctl->flag[i] = 0u;
  if (threadIdx.x == 0) ctl->err = 0;
}

}  // namespace

bool small_path_fits(int64_t n, int r) {
  return n >= 1 && n <= kSmallMaxN && r >= 1 && r <= kSmallMaxRank;
}

int launch_small_pcg(const SmallArgs& a, hipStream_t st) {
  if (!small_path_fits(a.n, a.r) || a.UKT == nullptr || a.UK == nullptr ||
      a.scratch == nullptr || a.out == nullptr || a.spin_limit < 1) {
    set_error("internal: persistent PCG launched outside its bounds");
    return CPHIFI_INVALID_ARG;
  }
  // one row per wave up to 256 rows, then 64 workgroups (a barrier over more
  // workgroups costs more than the rows it spreads: 3.2 us at 52, 7.2 at 128)
  const int grid = (int)std::min<int64_t>(kSmallGrid, (a.n + kWaves - 1) / kWaves);
  hipLaunchKernelGGL(small_reset_kernel, dim3(1), dim3(256), 0, st, (SmallCtl*)a.scratch);
  CPHIFI_CHECK_LAUNCH();
  if (a.r <= 8)
    hipLaunchKernelGGL(small_pcg_kernel<8>, dim3(grid), dim3(kT), 0, st, a);
  else if (a.r <= 16)
    hipLaunchKernelGGL(small_pcg_kernel<16>, dim3(grid), dim3(kT), 0, st, a);
  else
    hipLaunchKernelGGL(small_pcg_kernel<32>, dim3(grid), dim3(kT), 0, st, a);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

}  // namespace cphifi
