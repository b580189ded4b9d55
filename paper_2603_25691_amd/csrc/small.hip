// Persistent single-workgroup FP64 PCG for small subproblems (Section 4.4).
//
// For a small UI subproblem (K of a few hundred points, a few thousand
// observations) every step of a PCG iteration is a few microseconds of work,
// and a multi-kernel iteration spends its time in launches and in the host's
// convergence polls.  Here the whole iteration loop -- the two-step product
// (Section 4.4.1, eqs. vl, yhat1), the eq. (fx) preconditioner (Section
// 4.4.2) and the textbook PCG recurrence -- runs in ONE workgroup of 1024
// threads.  Every reduction is a fixed-order workgroup sum, so the result does
// not depend on scheduling, and the scalars stay in registers.
//
// The steps are laid out for latency, not bandwidth (the operands sit in L2):
//  * the n x n products are all of the form Y(s, c) = sum_k M[k ldm + s] X(k, c)
//    (K is symmetric; U and U^T come from the two stored layouts), so a wave's
//    64 lanes read 64 consecutive entries of a row of M per k; X is staged in
//    LDS; the k range is split over the waves that share a (64-row block,
//    4-column group) item, with 8 loads per lane in flight, and the slices
//    are added in a fixed order through LDS;
//  * the gather-scatter runs one thread per observation (its time index from
//    a per-observation copy), writing x_l Zhat(l, :) to a scratch row, then one
//    thread per (row, column) adds its segment's rows in order.
// The setup (V, eig(V), D), the right-hand side and the FP64 certificate stay
// the library's ordinary kernels.
#include "cphifi_internal.h"
#include "small.h"

#include <cmath>

namespace cphifi {
namespace {

constexpr int kT = kSmallThreads;
constexpr int kW = kT / 64;
constexpr int kSC = kSmallCols;
constexpr int kUnroll = 8;

struct Lds {
  double xs[kSmallMaxNR];         // X of the current product
  double red[kW * 64 * kSC];      // k-slice partial sums (also the workgroup sums)
};

__device__ double wg_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kW; ++w) t += red[w];
  return t;
}

// Y (n x r) = op(M) X with op(M)(s, k) = M[k ldm + s].
__device__ void sprod(const double* __restrict__ M, int64_t ldm, const double* __restrict__ X,
                      double* __restrict__ Y, int n, int r, Lds& L) {
  __syncthreads();  // X complete, xs / red free
  for (int e = threadIdx.x; e < n * r; e += kT) L.xs[e] = X[e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nb = (n + 63) / 64, ng = (r + kSC - 1) / kSC;
  const int items = nb * ng;
  const int nsl = max(1, kW / items);      // waves per item (k slices)
  const int ngroups = kW / nsl;            // items in flight
  const int grp = wave / nsl, sl = wave % nsl;
  const int kchunk = (n + nsl - 1) / nsl;
  const int kb = min(n, sl * kchunk), ke = min(n, kb + kchunk);
  const int trips = (items + ngroups - 1) / ngroups;
  for (int t = 0; t < trips; ++t) {
    const int it = grp + t * ngroups;
    const bool active = grp < ngroups && it < items;
    int s = 0, c0 = 0, nc = 0;
    if (active) {
      const int b = it / ng, g = it % ng;
      c0 = g * kSC;
      nc = min(kSC, r - c0);
      s = b * 64 + lane;
      double acc[kSC];
#pragma unroll
      for (int j = 0; j < kSC; ++j) acc[j] = 0.0;
      const double* mp = M + min(s, n - 1);  // lanes past n compute a row they do not store
      int k = kb;
      for (; k + kUnroll <= ke; k += kUnroll) {
        double m[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) m[u] = mp[(int64_t)(k + u) * ldm];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const double* xr = L.xs + (k + u) * r + c0;
#pragma unroll
          for (int j = 0; j < kSC; ++j)
            if (j < nc) acc[j] = fma(m[u], xr[j], acc[j]);
        }
      }
      for (; k < ke; ++k) {
        const double mv = mp[(int64_t)k * ldm];
        const double* xr = L.xs + k * r + c0;
#pragma unroll
        for (int j = 0; j < kSC; ++j)
          if (j < nc) acc[j] = fma(mv, xr[j], acc[j]);
      }
#pragma unroll
      for (int j = 0; j < kSC; ++j) L.red[(wave * 64 + lane) * kSC + j] = acc[j];
    }
    __syncthreads();
    if (active && sl == 0 && s < n) {
      for (int j = 0; j < nc; ++j) {
        double v = 0.0;
        for (int q = 0; q < nsl; ++q) v += L.red[((wave + q) * 64 + lane) * kSC + j];
        Y[(int64_t)s * r + c0 + j] = v;
      }
    }
    __syncthreads();
  }
}

// Y1 = G(Xh): x_l = <Xh(t_l,:), Zhat(l,:)> (eq. vl), Y1(s,:) = sum over the
// segment of x_l Zhat(l,:) (eq. yhat1).
__device__ void sgather(const SmallArgs& a, const int32_t* __restrict__ obs_t, int64_t q,
                        const double* __restrict__ Xh, double* __restrict__ Y1) {
  const int r = a.r;
  __syncthreads();  // Xh complete
  for (int64_t l = threadIdx.x; l < q; l += kT) {
    const int32_t t = obs_t[l];
    const double* xh = Xh + (int64_t)t * r;
    double* w = a.Wq + l * r;
    if (a.Zhat != nullptr) {
      const double* z = a.Zhat + l * r;
      double x = 0.0;
      for (int c = 0; c < r; ++c) x = fma(xh[c], z[c], x);
      for (int c = 0; c < r; ++c) w[c] = x * z[c];
    } else {
      const double* za = a.A + (int64_t)a.obs_i[l] * r;
      const double* zb = a.B + (int64_t)a.obs_j[l] * r;
      double x = 0.0;
      for (int c = 0; c < r; ++c) x = fma(xh[c], za[c] * zb[c], x);
      for (int c = 0; c < r; ++c) w[c] = x * (za[c] * zb[c]);
    }
  }
  __syncthreads();
  const int64_t len = a.n * r;
  for (int64_t e = threadIdx.x; e < len; e += kT) {
    const int64_t s = e / r;
    const int c = (int)(e % r);
    const int32_t b0 = a.obs_ptr[s], e0 = a.obs_ptr[s + 1];
    double acc = 0.0;
    int32_t l = b0;
    for (; l + 4 <= e0; l += 4) {
      const double w0 = a.Wq[(int64_t)l * r + c], w1 = a.Wq[(int64_t)(l + 1) * r + c];
      const double w2 = a.Wq[(int64_t)(l + 2) * r + c], w3 = a.Wq[(int64_t)(l + 3) * r + c];
      acc += w0;
      acc += w1;
      acc += w2;
      acc += w3;
    }
    for (; l < e0; ++l) acc += a.Wq[(int64_t)l * r + c];
    Y1[e] = acc;
  }
}

// Z = M^{-1} R by eq. fx: T1 = U^T R, T2(s,:) = ((T1(s,:) U_V) had D(s,:)) U_V^T,
// Z = U T2.
__device__ void sprecond(const SmallArgs& a, const double* R, double* Z, Lds& L) {
  const int n = (int)a.n, r = a.r;
  sprod(a.UKT, a.ldk, R, a.T1, n, r, L);
  __syncthreads();
  const int64_t len = a.n * r;
  for (int64_t e = threadIdx.x; e < len; e += kT) {
    const int64_t s = e / r;
    const int c = (int)(e % r);
    const double* t1 = a.T1 + s * r;
    double acc = 0.0;
    for (int j = 0; j < r; ++j) {
      double v = 0.0;
      for (int i = 0; i < r; ++i) v = fma(t1[i], a.UV[i * r + j], v);
      acc = fma(v * a.D[s * r + j], a.UV[c * r + j], acc);
    }
    a.T2[e] = acc;
  }
  sprod(a.UK, a.ldk, a.T2, Z, n, r, L);
}

// Q = A P (paper form): Xh = K P, Y1 = G(Xh), Q = K Y1 + lambda Xh + rho P.
__device__ void sapply(const SmallArgs& a, const int32_t* obs_t, int64_t q, const double* P,
                       double* Q, Lds& L) {
  const int n = (int)a.n, r = a.r;
  sprod(a.K, a.ldk, P, a.Xh, n, r, L);
  sgather(a, obs_t, q, a.Xh, a.Y1);
  sprod(a.K, a.ldk, a.Y1, a.T2, n, r, L);
  __syncthreads();
  const int64_t len = a.n * r;
  for (int64_t e = threadIdx.x; e < len; e += kT) Q[e] = a.T2[e] + a.lam * a.Xh[e] + a.rho * P[e];
}

__global__ __launch_bounds__(kT) void small_pcg_kernel(SmallArgs a, const int32_t* obs_t,
                                                       int64_t q) {
  __shared__ Lds L;
  double* red = L.red;
  const int64_t len = a.n * a.r;
  double* X = a.X;
  double* R = a.R;
  double* Z = a.Z;
  double* P = a.P;
  double* Q = a.Q;
  // r = b (x0 = 0) or b - A x0
  if (a.warm) {
    sapply(a, obs_t, q, X, Q, L);
    __syncthreads();
    for (int64_t e = threadIdx.x; e < len; e += kT) R[e] = a.b[e] - Q[e];
  } else {
    for (int64_t e = threadIdx.x; e < len; e += kT) {
      X[e] = 0.0;
      R[e] = a.b[e];
    }
  }
  double bb = 0.0, rr = 0.0;
  for (int64_t e = threadIdx.x; e < len; e += kT) bb += a.b[e] * a.b[e];
  bb = wg_sum(bb, red);
  for (int64_t e = threadIdx.x; e < len; e += kT) rr += R[e] * R[e];
  rr = wg_sum(rr, red);
  const double tol2 = a.tol * a.tol * bb;
  if (a.hist != nullptr && threadIdx.x == 0) a.hist[0] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
  int status = CPHIFI_NOT_CONVERGED, it = 0;
  if (!isfinite(bb) || !isfinite(rr)) {
    status = CPHIFI_NUMERIC;
  } else if (bb == 0.0 || rr <= tol2) {
    status = CPHIFI_OK;
  } else {
    if (a.precond)
      sprecond(a, R, Z, L);
    else
      for (int64_t e = threadIdx.x; e < len; e += kT) Z[e] = R[e];
    __syncthreads();
    double rz = 0.0;
    for (int64_t e = threadIdx.x; e < len; e += kT) {
      P[e] = Z[e];
      rz += R[e] * Z[e];
    }
    rz = wg_sum(rz, red);
    if (!(rz > 0.0) || !isfinite(rz)) status = isfinite(rz) ? CPHIFI_BREAKDOWN : CPHIFI_NUMERIC;
    while (status == CPHIFI_NOT_CONVERGED && it < a.maxit) {
      sapply(a, obs_t, q, P, Q, L);
      __syncthreads();
      double pq = 0.0;
      for (int64_t e = threadIdx.x; e < len; e += kT) pq += P[e] * Q[e];
      pq = wg_sum(pq, red);
      if (!(pq > 0.0) || !isfinite(pq)) {
        status = isfinite(pq) ? CPHIFI_BREAKDOWN : CPHIFI_NUMERIC;
        break;
      }
      const double alpha = rz / pq;
      double rrl = 0.0;
      for (int64_t e = threadIdx.x; e < len; e += kT) {
        X[e] += alpha * P[e];
        const double v = R[e] - alpha * Q[e];
        R[e] = v;
        rrl += v * v;
      }
      rr = wg_sum(rrl, red);
      ++it;
      if (a.hist != nullptr && threadIdx.x == 0 && it < a.hist_len)
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
      if (a.precond)
        sprecond(a, R, Z, L);
      else
        for (int64_t e = threadIdx.x; e < len; e += kT) Z[e] = R[e];
      __syncthreads();
      double rzl = 0.0;
      for (int64_t e = threadIdx.x; e < len; e += kT) rzl += R[e] * Z[e];
      const double rz_new = wg_sum(rzl, red);
      if (!(rz_new > 0.0) || !isfinite(rz_new)) {
        status = isfinite(rz_new) ? CPHIFI_BREAKDOWN : CPHIFI_NUMERIC;
        break;
      }
      const double beta = rz_new / rz;
      rz = rz_new;
      for (int64_t e = threadIdx.x; e < len; e += kT) P[e] = Z[e] + beta * P[e];
    }
  }
  if (threadIdx.x == 0) {
    a.out->iters = it;
    a.out->status = status;
    a.out->rr = rr;
    a.out->bb = bb;
  }
}

}  // namespace

bool small_path_fits(int64_t n, int r, int64_t q, int64_t wq_cap) {
  return n <= kSmallMaxN && r <= kSmallMaxRank && n * r <= kSmallMaxNR &&
         (double)n * (double)n * r <= kSmallMaxProductWork &&
         (double)q * r <= kSmallMaxObsWork && q * r <= wq_cap;
}

int launch_small_pcg(const SmallArgs& a, const int32_t* obs_t, int64_t q, hipStream_t st) {
  if (!small_path_fits(a.n, a.r, q, q * a.r) || a.UKT == nullptr || a.Wq == nullptr ||
      (q > 0 && obs_t == nullptr)) {
    set_error("internal: persistent PCG launched outside its bounds");
    return CPHIFI_INVALID_ARG;
  }
  hipLaunchKernelGGL(small_pcg_kernel, dim3(1), dim3(kT), 0, st, a, obs_t, q);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

}  // namespace cphifi
