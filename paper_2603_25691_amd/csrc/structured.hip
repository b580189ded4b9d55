// Structured forms of the two-step product of Section 4.4.1, each behind a
// plan flag:
//
//  * Toeplitz K (CPHIFI_FLAG_TOEPLITZ_K).  A translation-invariant kernel on a
//    uniform grid makes K symmetric Toeplitz, K(s, k) = c(|s - k|) with c the
//    first row of K (the paper notes this structure as a way to cut the cost
//    of the K products).  The products K X then read the n values of c
//    instead of the n^2 entries of K: each workgroup stages, per chunk of 64
//    k, the rows of X and the 127 values of c its 64 x 64 block of K needs in
//    LDS, and multiplies in FP64 with 4 x 4 register tiles.  Work is
//    2 n^2 r flops as before, HBM traffic O(n r).
//
//  * Fiber collapse (CPHIFI_FLAG_FIBER_COLLAPSE).  When every (time, sample)
//    pair that is observed at all is observed at all J features, the
//    gather-scatter of eqs. vl and yhat1 over the J observations of such a
//    fiber (i, s) collapses: with G = B^T B,
//        sum_j <Xhat(s,:), A(i,:) had B(j,:)> (A(i,:) had B(j,:))
//          = A(i,:) had ((Xhat(s,:) had A(i,:)) G),
//    r^2 work per fiber instead of 2 J r per fiber, and no per-observation
//    indices are read.  A wave per time point when time points have few
//    fibers, a workgroup per time point when they have many.
#include "cphifi_internal.h"

#include <cmath>

namespace cphifi {
namespace {

constexpr int kTRows = 64;  // rows of K per Toeplitz workgroup
constexpr int kTK = 64;     // k per staged chunk
// Time points with at most this many fibers get one wave each; more, one workgroup.
constexpr int kFibersPerWave = 8;

__device__ __forceinline__ bool structured_done(const int32_t* done) {
  return done != nullptr && *(volatile const int32_t*)done != 0;
}

// flag <- 1 where |K(s, k) - c(|s - k|)| > tol.
__global__ void toeplitz_check_kernel(const double* __restrict__ K, int64_t ldk, int64_t n,
                                      const double* __restrict__ c, double tol,
                                      int32_t* __restrict__ flag) {
  const int64_t len = n * n;
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / n, k = e % n;
    const int64_t d = s >= k ? s - k : k - s;
    bad |= !(fabs(K[s * ldk + k] - c[d]) <= tol);
  }
  if (bad) *flag = 1;
}

// part[slab blockIdx.y] rows [r0, r0 + 64) = sum over k in the slab's range of
// c(|s - k|) X(k, :).  Thread t: rows r0 + 4 (t / 16) + i, columns 4 (t % 16) + j.
__global__ __launch_bounds__(256) void toeplitz_product_kernel(
    const double* __restrict__ c, int64_t n, const double* __restrict__ X, int64_t ldx, int r,
    double* __restrict__ part, int ldp, int64_t kper, const int32_t* done) {
  if (structured_done(done)) return;
  __shared__ double xs[kTK * kMaxRank];
  __shared__ double cw[2 * kTK];
  const int tid = threadIdx.x;
  const int rg = tid >> 4, cg = tid & 15;
  const int64_t r0 = (int64_t)blockIdx.x * kTRows;
  const int64_t kbeg = (int64_t)blockIdx.y * kper;
  const int64_t kend = min(n, kbeg + kper);
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += kTK) {
    const int kc = (int)min<int64_t>(kTK, kend - k0);
    for (int e = tid; e < kTK * r; e += 256) {
      const int kk = e / r, col = e % r;
      xs[kk * r + col] = kk < kc ? X[(k0 + kk) * ldx + col] : 0.0;
    }
    // cw[m] = c(|d|) for d = (r0 - k0) + m - (kTK - 1), m in [0, 2 kTK - 1)
    for (int m = tid; m < 2 * kTK - 1; m += 256) {
      int64_t d = (r0 - k0) + m - (kTK - 1);
      d = d < 0 ? -d : d;
      cw[m] = d < n ? c[d] : 0.0;
    }
    __syncthreads();
    if (4 * cg < r) {
      for (int kk = 0; kk < kc; ++kk) {
        double xv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) xv[j] = (4 * cg + j < r) ? xs[kk * r + 4 * cg + j] : 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double cv = cw[4 * rg + i - kk + (kTK - 1)];
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = fma(cv, xv[j], acc[i][j]);
        }
      }
    }
    __syncthreads();
  }
  double* out = part + (int64_t)blockIdx.y * n * ldp;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = r0 + 4 * rg + i;
    if (row >= n) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (4 * cg + j < r) out[row * ldp + 4 * cg + j] = acc[i][j];
  }
}

// G = B^T B (r x r), one thread per entry.
__global__ void fiber_gram_kernel(const double* __restrict__ B, int64_t J, int r,
                                  double* __restrict__ G) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r * r) return;
  const int a = e / r, b = e % r;
  double s = 0.0;
  for (int64_t j = 0; j < J; ++j) s += B[j * r + a] * B[j * r + b];
  G[e] = s;
}

// Y1(s,:) = sum over the fibers f of time s of A(i_f,:) had ((Xhat(s,:) had A(i_f,:)) G),
// Xhat(s,:) from the split-K partials of K P (PT) or from xin; written to
// xhat_out when given.  Lane c holds column c; G in LDS; u G by lane
// broadcasts.  Two forms: WAVE = one wave per time point (few fibers per time
// point, e.g. one: the unaligned recipes), else one workgroup per time point
// whose four waves take the fibers in turn, their sums added in a fixed order
// (many fibers per time point: the aligned case's I = 500 per grid point, where
// a wave per time point left the chip nearly idle).
template <typename PT, bool WAVE>
__global__ __launch_bounds__(256) void fiber_gather_kernel(
    const PT* __restrict__ part, int ksplit, int ldp, const double* __restrict__ xin, int64_t n,
    int r, const int32_t* __restrict__ fib_ptr, const int32_t* __restrict__ fib_i,
    const double* __restrict__ A, const double* __restrict__ G, double* __restrict__ xhat_out,
    double* __restrict__ y1, const int32_t* done) {
  if (structured_done(done)) return;
  __shared__ double Gs[kMaxRank * kMaxRank];
  __shared__ double red[4][kMaxRank];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < r * r; e += 256) Gs[e] = G[e];
  __syncthreads();
  const bool on = lane < r;
  const int64_t first = WAVE ? (int64_t)blockIdx.x * 4 + wave : blockIdx.x;
  const int64_t step = WAVE ? (int64_t)gridDim.x * 4 : gridDim.x;
  for (int64_t s = first; s < n; s += step) {
    double x = 0.0;
    if (on) {
      if (part != nullptr) {
        for (int k = 0; k < ksplit; ++k) x += (double)part[((int64_t)k * n + s) * ldp + lane];
      } else {
        x = xin[s * r + lane];
      }
      if (xhat_out != nullptr && (WAVE || wave == 0)) xhat_out[s * r + lane] = x;
    }
    double acc = 0.0;
    for (int32_t f = fib_ptr[s] + (WAVE ? 0 : wave); f < fib_ptr[s + 1]; f += (WAVE ? 1 : 4)) {
      const double a = on ? A[(int64_t)fib_i[f] * r + lane] : 0.0;
      const double u = x * a;
      double v = 0.0;
      for (int cc = 0; cc < r; ++cc) v = fma(__shfl(u, cc, 64), on ? Gs[cc * r + lane] : 0.0, v);
      acc = fma(a, v, acc);
    }
    if (WAVE) {
      if (on) y1[s * r + lane] = acc;
    } else {
      if (on) red[wave][lane] = acc;
      __syncthreads();
      if (tid < r) y1[s * r + tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
      __syncthreads();
    }
  }
}

}  // namespace

int launch_toeplitz_check(const double* K, int64_t ldk, int64_t n, const double* c, double tol,
                          int32_t* flag, hipStream_t st) {
  const int64_t len = n * n;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(2048, (len + 255) / 256));
  hipLaunchKernelGGL(toeplitz_check_kernel, dim3(blocks), dim3(256), 0, st, K, ldk, n, c, tol,
                     flag);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_toeplitz_product(const double* c, int64_t n, const double* X, int64_t ldx, int r,
                            double* part, int ldp, int num_cu, int* ksplit_out,
                            const int32_t* done, hipStream_t st) {
  if (r < 1 || r > kMaxRank || ldp < r) {
    set_error("toeplitz product: r = %d outside [1, %d] or ldp < r", r, kMaxRank);
    return CPHIFI_INVALID_ARG;
  }
  const int64_t nbx = (n + kTRows - 1) / kTRows;
  const int64_t nchunks = (n + kTK - 1) / kTK;
  // split k so that the grid covers every CU about twice
  int64_t ks = std::max<int64_t>(1, (2 * (int64_t)num_cu + nbx - 1) / nbx);
  ks = std::min<int64_t>({ks, (int64_t)kMaxSplit, nchunks});
  const int64_t kper = (nchunks + ks - 1) / ks * kTK;
  ks = (n + kper - 1) / kper;
  hipLaunchKernelGGL(toeplitz_product_kernel, dim3((unsigned)nbx, (unsigned)ks), dim3(256), 0,
                     st, c, n, X, ldx, r, part, ldp, kper, done);
  CPHIFI_CHECK_LAUNCH();
  *ksplit_out = (int)ks;
  return CPHIFI_OK;
}

int launch_fiber_gram(const double* B, int64_t J, int r, double* G, hipStream_t st) {
  hipLaunchKernelGGL(fiber_gram_kernel, dim3((r * r + 255) / 256), dim3(256), 0, st, B, J, r,
                     G);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_fiber_gather(const void* part, bool is_float, int ksplit, int ldp, const double* xin,
                        int64_t n, int r, const int32_t* fib_ptr, const int32_t* fib_i,
                        const double* A, const double* G, double* xhat_out, double* y1,
                        int max_fibers, const int32_t* done, hipStream_t st) {
  if (r < 1 || r > kMaxRank) {
    set_error("fiber gather: r = %d outside [1, %d]", r, kMaxRank);
    return CPHIFI_INVALID_ARG;
  }
  const bool wave = max_fibers <= kFibersPerWave;
  const int64_t units = wave ? (n + 3) / 4 : n;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(units, 2048));
#define CPHIFI_FIBER_LAUNCH(PT, W)                                                            \
  hipLaunchKernelGGL((fiber_gather_kernel<PT, W>), dim3(blocks), dim3(256), 0, st,            \
                     (const PT*)part, ksplit, ldp, xin, n, r, fib_ptr, fib_i, A, G, xhat_out, \
                     y1, done)
  if (part != nullptr && is_float) {
    if (wave)
      CPHIFI_FIBER_LAUNCH(float, true);
    else
      CPHIFI_FIBER_LAUNCH(float, false);
  } else {
    if (wave)
      CPHIFI_FIBER_LAUNCH(double, true);
    else
      CPHIFI_FIBER_LAUNCH(double, false);
  }
#undef CPHIFI_FIBER_LAUNCH
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

}  // namespace cphifi
