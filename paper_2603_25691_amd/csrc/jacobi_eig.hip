// Symmetric eigendecomposition K = U D U^T (eq. eigK) by the cyclic Jacobi
// method with the parallel (round-robin) ordering, written for the device.
//
// Each sweep runs m - 1 steps (m = n rounded up to even); a step pairs every
// index with one other (the round-robin tournament: one player fixed -- a
// dummy when n is odd -- the others rotating), so its m / 2 plane rotations
// touch disjoint rows and columns and apply together.  A step is two launches:
//  * rows: for each pair (p, q) the rotation that annihilates A(p, q)
//    (c, s from the classical symmetric 2 x 2 Schur decomposition: with
//    theta = (a_qq - a_pp) / (2 a_pq), t = sign(theta) / (|theta| +
//    sqrt(theta^2 + 1)), c = 1 / sqrt(t^2 + 1), s = t c) is formed by the
//    workgroup that owns the pair and applied to rows p and q of A: A <- J^T A;
//  * columns: the same rotations applied to columns p and q of A and of the
//    accumulated eigenvector matrix V: A <- A J, V <- V J.
// After every sweep the off-diagonal mass ||A - diag(A)||_F is compared with
// tol ||K||_F on the host; the diagonal then holds the eigenvalues, V the
// eigenvectors (columns), which are sorted ascending and written in the
// library's layout (row k of UK = eigenvector k).
//
// Work and traffic: 4 n^2 doubles of A and 2 n^2 of V read and written per
// step, n steps per sweep: O(n^3) per sweep, ~6-10 sweeps.  Meant for the
// small and medium kernel matrices (n up to a few thousand); larger ones go
// to the divide-and-conquer solver of cphifi_kernel_eig.
#include "cphifi_internal.h"

#include <cmath>
#include <numeric>

namespace cphifi {
namespace {

constexpr int kJT = 256;

// Pair i of step k in the round-robin schedule on m (even) players: player 0
// stays; the others take positions rotated by k.  Player x is index x - shift:
// for odd n (shift 1) the fixed player is the dummy, so each step one real
// index idles.  (With the dummy as the last player instead, a CPU model of this
// solver stalled near 1e-9 relative off-diagonal mass on Gaussian kernel
// matrices of odd order, the fixed index's couplings to the near-null
// eigenvectors decaying only linearly; with the dummy fixed it converged
// quadratically to rounding in 10 sweeps, like even orders.)  Returns false
// for a pair that involves the dummy.
__host__ __device__ inline bool rr_pair(int64_t n, int64_t m, int64_t k, int64_t i, int64_t* p,
                                        int64_t* q) {
  auto player = [&](int64_t pos) -> int64_t {
    return pos == 0 ? 0 : ((pos - 1 + k) % (m - 1)) + 1;
  };
  const int64_t a = player(i), b = player(m - 1 - i);
  const int64_t shift = m - n;
  *p = (a < b ? a : b) - shift;
  *q = (a < b ? b : a) - shift;
  return *p >= 0;
}

// Rows phase: block bx owns pairs [bx * pp, ...) and all columns j in chunks.
__global__ __launch_bounds__(kJT) void jac_rows_kernel(double* __restrict__ A, int64_t n,
                                                       int64_t m, int64_t k, int pairs_per_block,
                                                       double* __restrict__ cs) {
  __shared__ double c_s[2 * kJT];
  const int64_t npairs = m / 2;
  const int64_t i0 = (int64_t)blockIdx.x * pairs_per_block;
  for (int t = threadIdx.x; t < pairs_per_block; t += kJT) {
    const int64_t i = i0 + t;
    double c = 1.0, s = 0.0;
    if (i < npairs) {
      int64_t p, q;
      if (rr_pair(n, m, k, i, &p, &q)) {
        const double apq = A[p * n + q];
        if (apq != 0.0) {
          const double app = A[p * n + p], aqq = A[q * n + q];
          const double theta = (aqq - app) / (2.0 * apq);
          const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
          c = 1.0 / sqrt(tt * tt + 1.0);
          s = tt * c;
        }
      }
      cs[2 * i] = c;
      cs[2 * i + 1] = s;
    }
    c_s[2 * t] = c;
    c_s[2 * t + 1] = s;
  }
  __syncthreads();
  const int64_t work = (int64_t)pairs_per_block * n;
  for (int64_t e = threadIdx.x; e < work; e += kJT) {
    const int t = (int)(e / n);
    const int64_t j = e % n;
    const int64_t i = i0 + t;
    if (i >= npairs) break;
    int64_t p, q;
    if (!rr_pair(n, m, k, i, &p, &q)) continue;
    const double c = c_s[2 * t], s = c_s[2 * t + 1];
    const double ap = A[p * n + j], aq = A[q * n + j];
    A[p * n + j] = c * ap - s * aq;
    A[q * n + j] = s * ap + c * aq;
  }
}

// Columns phase: thread per (row i, pair): columns p, q of A and of V.
__global__ __launch_bounds__(kJT) void jac_cols_kernel(double* __restrict__ A,
                                                       double* __restrict__ V, int64_t n,
                                                       int64_t m, int64_t k,
                                                       const double* __restrict__ cs) {
  const int64_t npairs = m / 2;
  const int64_t work = npairs * n;
  for (int64_t e = (int64_t)blockIdx.x * kJT + threadIdx.x; e < work;
       e += (int64_t)gridDim.x * kJT) {
    const int64_t i = e / n;  // pair
    const int64_t row = e % n;
    int64_t p, q;
    if (!rr_pair(n, m, k, i, &p, &q)) continue;
    const double c = cs[2 * i], s = cs[2 * i + 1];
    const double ap = A[row * n + p], aq = A[row * n + q];
    A[row * n + p] = c * ap - s * aq;
    A[row * n + q] = s * ap + c * aq;
    const double vp = V[row * n + p], vq = V[row * n + q];
    V[row * n + p] = c * vp - s * vq;
    V[row * n + q] = s * vp + c * vq;
  }
}

// Partials of the off-diagonal and total squared mass.
__global__ __launch_bounds__(kJT) void jac_off_kernel(const double* __restrict__ A, int64_t n,
                                                      double* __restrict__ part) {
  double off = 0.0, tot = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kJT + threadIdx.x; e < n * n;
       e += (int64_t)gridDim.x * kJT) {
    const double v = A[e];
    tot += v * v;
    if (e / n != e % n) off += v * v;
  }
  __shared__ double so[kJT / kWave], st[kJT / kWave];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    off += __shfl_xor(off, d, 64);
    tot += __shfl_xor(tot, d, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    so[threadIdx.x >> 6] = off;
    st[threadIdx.x >> 6] = tot;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < kJT / kWave; ++w) {
      a += so[w];
      b += st[w];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

__global__ void jac_copy_in_kernel(const double* __restrict__ K, int64_t ldk, int64_t n,
                                   double* __restrict__ A, double* __restrict__ V) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e % n;
    // symmetrise: the method assumes an exactly symmetric A
    A[e] = 0.5 * (K[i * ldk + j] + K[j * ldk + i]);
    V[e] = i == j ? 1.0 : 0.0;
  }
}

// inv[j] = 1 / ||V(:, j)||: the accumulated rotations let the column norms
// drift from 1 by O(rotations x u) (6e-13 at n = 1200); the off-diagonal
// inner products stay ~1e-14, so normalising restores orthonormality.
__global__ __launch_bounds__(kJT) void jac_colnorm_kernel(const double* __restrict__ V,
                                                          int64_t n, double* __restrict__ inv) {
  __shared__ double red[kJT / kWave];
  for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
    double acc = 0.0;
    for (int64_t s = threadIdx.x; s < n; s += kJT) acc += V[s * n + j] * V[s * n + j];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kJT / kWave; ++w) t += red[w];
      inv[j] = 1.0 / sqrt(t);
    }
  }
}

// UK[kk * ldk + s] = V[s][perm[kk]] / ||V(:, perm[kk])|| (row kk = eigenvector
// kk), dK[kk] = A[perm[kk]][perm[kk]].
__global__ void jac_copy_out_kernel(const double* __restrict__ V, const double* __restrict__ A,
                                    const int32_t* __restrict__ perm,
                                    const double* __restrict__ inv, int64_t n, int64_t ldk,
                                    double* __restrict__ UK, double* __restrict__ dK) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t kk = e / n, s = e % n;
    const int32_t src = perm[kk];
    UK[kk * ldk + s] = V[s * n + src] * inv[src];
    if (s == 0) dK[kk] = A[(int64_t)src * n + src];
  }
}

int grid_of(int64_t work) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(4096, (work + kJT - 1) / kJT));
}

}  // namespace
}  // namespace cphifi

using namespace cphifi;

extern "C" int cphifi_kernel_eig_jacobi(int64_t n, const double* K, int64_t ldk, double* UK,
                                        double* dK, double tol, int max_sweeps, int* sweeps_out,
                                        void* stream) {
  clear_error();
  if (n < 1 || n > kJacobiMaxN || K == nullptr || UK == nullptr || dK == nullptr || ldk < n ||
      !(tol > 0.0) || max_sweeps < 1) {
    set_error("kernel_eig_jacobi: need 1 <= n <= %lld, ldk >= n, tol > 0, max_sweeps >= 1 and "
              "non-null K, UK, dK", (long long)kJacobiMaxN);
    return CPHIFI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  const int64_t m = n + (n & 1);
  const int64_t npairs = m / 2;
  const int offb = grid_of(n * n);
  double *A = nullptr, *V = nullptr, *cs = nullptr, *part = nullptr;
  int32_t* perm_d = nullptr;
  auto release = [&]() {
    if (A) (void)hipFree(A);
    if (V) (void)hipFree(V);
    if (cs) (void)hipFree(cs);
    if (part) (void)hipFree(part);
    if (perm_d) (void)hipFree(perm_d);
  };
  if (hipMalloc(&A, sizeof(double) * n * n) != hipSuccess ||
      hipMalloc(&V, sizeof(double) * n * n) != hipSuccess ||
      hipMalloc(&cs, sizeof(double) * 2 * npairs) != hipSuccess ||
      hipMalloc(&part, sizeof(double) * 2 * offb) != hipSuccess ||
      hipMalloc(&perm_d, sizeof(int32_t) * n) != hipSuccess) {
    release();
    set_error("kernel_eig_jacobi: device allocation failed");
    return CPHIFI_HIP_ERROR;
  }
  int rc = CPHIFI_OK;
  auto sweep_mass = [&](double* off, double* tot) -> int {
    hipLaunchKernelGGL(jac_off_kernel, dim3(offb), dim3(kJT), 0, st, A, n, part);
    CPHIFI_CHECK_LAUNCH();
    std::vector<double> h(2 * offb);
    CPHIFI_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost,
                              st));
    CPHIFI_HIP(hipStreamSynchronize(st));
    double a = 0.0, b = 0.0;
    for (int i = 0; i < offb; ++i) {
      a += h[2 * i];
      b += h[2 * i + 1];
    }
    *off = std::sqrt(a);
    *tot = std::sqrt(b);
    return CPHIFI_OK;
  };
  hipLaunchKernelGGL(jac_copy_in_kernel, dim3(grid_of(n * n)), dim3(kJT), 0, st, K, ldk, n, A, V);
  if (hipGetLastError() != hipSuccess) {
    release();
    set_error("kernel_eig_jacobi: launch failed");
    return CPHIFI_HIP_ERROR;
  }
  double off = 0.0, tot = 0.0;
  if ((rc = sweep_mass(&off, &tot)) != CPHIFI_OK) {
    release();
    return rc;
  }
  const double target = tol * tot;
  // pairs per rows-phase block: enough blocks to fill the chip at small n
  const int ppb = (int)std::max<int64_t>(1, std::min<int64_t>(16, npairs / 512 + 1));
  const int rows_blocks = (int)((npairs + ppb - 1) / ppb);
  const int cols_blocks = grid_of(npairs * n);
  int sweeps = 0;
  while (off > target && sweeps < max_sweeps) {
    for (int64_t k = 0; k < m - 1; ++k) {
      hipLaunchKernelGGL(jac_rows_kernel, dim3(rows_blocks), dim3(kJT), 0, st, A, n, m, k, ppb,
                         cs);
      hipLaunchKernelGGL(jac_cols_kernel, dim3(cols_blocks), dim3(kJT), 0, st, A, V, n, m, k,
                         cs);
    }
    if (hipGetLastError() != hipSuccess) {
      release();
      set_error("kernel_eig_jacobi: launch failed");
      return CPHIFI_HIP_ERROR;
    }
    ++sweeps;
    if ((rc = sweep_mass(&off, &tot)) != CPHIFI_OK) {
      release();
      return rc;
    }
    if (!std::isfinite(off)) break;
  }
  if (sweeps_out != nullptr) *sweeps_out = sweeps;
  if (!(off <= target)) {
    release();
    set_error("kernel_eig_jacobi: off-diagonal mass %.3e above %.3e after %d sweeps", off,
              target, sweeps);
    return CPHIFI_NUMERIC;
  }
  // eigenvalues (the diagonal) to the host, ascending order, then the output layout
  std::vector<double> diag(n);
  if (hipMemcpy2DAsync(diag.data(), sizeof(double), A, sizeof(double) * (n + 1), sizeof(double),
                       n, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    release();
    set_error("kernel_eig_jacobi: copy of the diagonal failed");
    return CPHIFI_HIP_ERROR;
  }
  std::vector<int32_t> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(),
                   [&](int32_t a, int32_t b) { return diag[a] < diag[b]; });
  if (hipMemcpyAsync(perm_d, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st) !=
      hipSuccess) {
    release();
    set_error("kernel_eig_jacobi: upload of the order failed");
    return CPHIFI_HIP_ERROR;
  }
  // the rotation coefficients' buffer (2 npairs >= n doubles) holds the inverse norms
  hipLaunchKernelGGL(jac_colnorm_kernel, dim3((unsigned)std::min<int64_t>(n, 4096)), dim3(kJT), 0,
                     st, V, n, cs);
  hipLaunchKernelGGL(jac_copy_out_kernel, dim3(grid_of(n * n)), dim3(kJT), 0, st, V, A, perm_d, cs,
                     n, ldk, UK, dK);
  const hipError_t e1 = hipGetLastError();
  const hipError_t e2 = hipStreamSynchronize(st);
  release();
  if (e1 != hipSuccess || e2 != hipSuccess) {
    set_error("kernel_eig_jacobi: output failed");
    return CPHIFI_HIP_ERROR;
  }
  return CPHIFI_OK;
}
