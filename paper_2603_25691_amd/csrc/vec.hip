// FP64 vector kernels of the PCG iteration (Section 4.4; the recurrence is the
// textbook preconditioned CG), the r x r steps of the preconditioner (eq. fx),
// the per-solve setup of Section 4.4.2 (Gram V, eigendecomposition of V, the
// inverse diagonal D) and the low-precision copies of U_K.
//
// Every reduction is two-stage and deterministic: a kernel writes one partial
// per block, and each consumer adds all partials in one fixed order.  Kernels
// that need a finished scalar (alpha, beta, the convergence test) recompute it
// from the partials themselves, so no host round trip sits inside an iteration.
#include "cphifi_internal.h"
#include "jacobi.h"

#include <cmath>

namespace cphifi {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic sum over a 256-thread block; result valid in every thread.
__device__ double block_sum(double v) {
  __shared__ double ws[4];
  __shared__ double total;
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) ws[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) total = ((ws[0] + ws[1]) + ws[2]) + ws[3];
  __syncthreads();
  return total;
}

// Sum of red[0..nblk) in a fixed order (identical in every block that calls it).
__device__ double sum_partials(const double* red, int nblk) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) v += red[i];
  return block_sum(v);
}

__device__ __forceinline__ bool is_done(const int32_t* done) { return done != nullptr && *done; }

template <typename PT>
__device__ __forceinline__ double part_sum(const PT* part, int ksplit, int64_t n, int ldp,
                                           int64_t s, int c) {
  double v = 0.0;
  for (int sp = 0; sp < ksplit; ++sp) v += (double)part[((int64_t)sp * n + s) * ldp + c];
  return v;
}

template <typename PT>
__global__ __launch_bounds__(256) void reduce_partials_kernel(const PT* part, int ksplit, int ldp,
                                                              int64_t n, int r, double* out,
                                                              const double* dotwith, double* red,
                                                              const double* rowscale,
                                                              const int32_t* done) {
  if (is_done(done)) return;
  const int64_t len = n * r;
  double loc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / r;
    const int c = (int)(e % r);
    double v = part_sum(part, ksplit, n, ldp, s, c);
    if (rowscale != nullptr) v *= rowscale[s];
    out[e] = v;
    if (dotwith != nullptr) loc += dotwith[e] * v;
  }
  if (red != nullptr) {
    const double b = block_sum(loc);
    if (threadIdx.x == 0) red[blockIdx.x] = b;
  }
}

template <typename PT>
__global__ __launch_bounds__(256) void apply_finish_kernel(const PT* part, int ksplit, int ldp,
                                                           int64_t n, int r, const double* xhat,
                                                           const double* p, const double* dscale,
                                                           double lam, double rho, double* q,
                                                           double* red, const int32_t* done) {
  if (is_done(done)) return;
  const int64_t len = n * r;
  double loc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / r;
    const int c = (int)(e % r);
    const double y = part_sum(part, ksplit, n, ldp, s, c);
    const double pe = p[e];
    double v;
    if (dscale != nullptr)
      v = dscale[s] * (y + lam * pe) + rho * pe;
    else
      v = y + lam * xhat[e] + rho * pe;
    q[e] = v;
    loc += pe * v;
  }
  if (red != nullptr) {
    const double b = block_sum(loc);
    if (threadIdx.x == 0) red[blockIdx.x] = b;
  }
}

__global__ __launch_bounds__(256) void dot_kernel(const double* a, const double* b, int64_t len,
                                                  double* red, const int32_t* done) {
  if (is_done(done)) return;
  double loc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    loc += a[e] * b[e];
  const double s = block_sum(loc);
  if (threadIdx.x == 0) red[blockIdx.x] = s;
}

// alpha = rz / p^T q; x += alpha p; r -= alpha q; partial ||r||^2.
__global__ __launch_bounds__(256) void update_xr_kernel(double* x, double* r, const double* p,
                                                        const double* q, int64_t len,
                                                        const double* red_pq, int nblk_pq,
                                                        double* red_rr, DevScalars* sc, int it) {
  if (sc->done) return;
  if (it < 0) it = sc->it;  // captured loop: the device counter
  const double pq = sum_partials(red_pq, nblk_pq);
  const double rz = sc->rz[it & 1];
  if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rz)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->pq = pq;
      sc->status = (isfinite(pq) && isfinite(rz)) ? CPHIFI_BREAKDOWN : CPHIFI_NUMERIC;
      sc->iters = it;
      sc->done = 1;
    }
    return;
  }
  const double alpha = rz / pq;
  double loc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x) {
    x[e] += alpha * p[e];
    const double rv = r[e] - alpha * q[e];
    r[e] = rv;
    loc += rv * rv;
  }
  const double b = block_sum(loc);
  if (threadIdx.x == 0) red_rr[blockIdx.x] = b;
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->pq = pq;
}

// flag (host memory, may be null) receives sc->done as of this iteration.
__global__ __launch_bounds__(256) void check_conv_kernel(const double* red_rr, int nblk,
                                                         DevScalars* sc, int it, double* hist,
                                                         int hist_len, int32_t* flag) {
  if (sc->done) {
    if (flag != nullptr && threadIdx.x == 0) *(volatile int32_t*)flag = 1;
    return;
  }
  const bool counted = it < 0;  // captured loop: read and advance the device counter
  if (counted) it = sc->it;
  const double rr = sum_partials(red_rr, nblk);
  if (threadIdx.x == 0) {
    sc->rr = rr;
    if (hist != nullptr && it + 1 < hist_len) hist[it + 1] = sqrt(rr / sc->bb);
    int32_t done = 0;
    if (!isfinite(rr)) {
      sc->status = CPHIFI_NUMERIC;
      sc->iters = it + 1;
      sc->done = done = 1;
    } else if (rr <= sc->tol2) {
      sc->status = CPHIFI_OK;
      sc->iters = it + 1;
      sc->done = done = 1;
    }
    if (flag != nullptr) *(volatile int32_t*)flag = done;
    if (counted) sc->it = it + 1;
  }
}

// beta = r+^T z+ / r^T z; p = z + beta p.
__global__ __launch_bounds__(256) void update_p_kernel(double* p, const double* z, int64_t len,
                                                       const double* red_rz, int nblk,
                                                       DevScalars* sc, int it) {
  if (sc->done) return;
  if (it < 0) it = sc->it - 1;  // captured loop: the check of this iteration advanced it
  const double rz_new = sum_partials(red_rz, nblk);
  const double rz_old = sc->rz[it & 1];
  if (!(rz_new > 0.0) || !isfinite(rz_new)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->status = isfinite(rz_new) ? CPHIFI_BREAKDOWN : CPHIFI_NUMERIC;
      sc->iters = it + 1;
      sc->done = 1;
    }
    return;
  }
  const double beta = rz_new / rz_old;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = z[e] + beta * p[e];
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->rz[(it + 1) & 1] = rz_new;
}

__global__ __launch_bounds__(256) void pcg_init_kernel(DevScalars* sc, const double* red_bb,
                                                       int nblk_bb, const double* red_rr,
                                                       int nblk_rr, const double* red_rz,
                                                       int nblk_rz, double tol, double* hist,
                                                       int hist_len) {
  const double bb = sum_partials(red_bb, nblk_bb);
  const double rr = sum_partials(red_rr, nblk_rr);
  const double rz = red_rz != nullptr ? sum_partials(red_rz, nblk_rz) : 1.0;
  if (threadIdx.x == 0) {
    sc->bb = bb;
    sc->rr = rr;
    sc->rz[0] = rz;
    sc->rz[1] = rz;
    sc->pq = 0.0;
    sc->tol2 = tol * tol * bb;
    sc->iters = 0;
    sc->status = CPHIFI_OK;
    sc->done = 0;
    sc->zero = 0;
    sc->it = 0;
    if (hist != nullptr && hist_len > 0) hist[0] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    if (!isfinite(bb) || !isfinite(rr) || !isfinite(rz)) {
      sc->status = CPHIFI_NUMERIC;
      sc->done = 1;
    } else if (bb == 0.0 || rr <= sc->tol2) {
      sc->done = 1;  // already converged (x is the answer; b == 0 gives x = 0)
    } else if (!(rz > 0.0)) {
      sc->status = CPHIFI_BREAKDOWN;
      sc->done = 1;
    }
  }
}

__global__ void store_sum_kernel(const double* red, int nblk, DevScalars* sc, int slot) {
  const double v = sum_partials(red, nblk);
  if (threadIdx.x == 0) sc->scratch[slot] = v;
}

// dst (host-mapped memory) <- *src, word by word.
__global__ void mirror_kernel(const DevScalars* src, DevScalars* dst) {
  constexpr int kWords = sizeof(DevScalars) / sizeof(int32_t);
  static_assert(sizeof(DevScalars) % sizeof(int32_t) == 0, "DevScalars is whole words");
  const int32_t* s = (const int32_t*)src;
  volatile int32_t* d = (volatile int32_t*)dst;
  for (int i = threadIdx.x; i < kWords; i += blockDim.x) d[i] = s[i];
}

// out[s,:] = ((t U_V) * D[s,:]) U_V^T (the middle step of eq. fx), t = in[s,:]
// or the sum of split-K partials; red <- partials of dotwith . out.  The two
// r x r products run on the FP64 4x4x4 MFMA
// (v_mfma_f64_4x4x4_4b: four independent 4x4x4 products; block b =
// (lane / 4) % 4, A_b[i][k] in lane 16 k + 4 b + i, B_b[k][j] in lane
// 16 k + 4 b + j, D_b[i][j] in lane 16 i + 4 b + j).  A wave takes 16 rows at
// a time: the four blocks are four groups of 4 rows sharing one group of 4
// columns, so lane (li = lane % 16, kk = lane / 16) supplies A = T[row li][k]
// and the result of column group c lands at row 4 ((lane / 4) % 4) + lane / 16,
// column 4 c + lane % 4.  r is padded to rp = 4 NC4 with zeros.  The rows of T
// (and of T U_V * D, for the second product) pass through a per-wave LDS tile,
// U_V through a block-shared one.
// With UPD (a PCG iteration in the eigenbasis), the rows are first updated as
// they are staged -- alpha = r^T z / p^T q from the partials of p^T q, x +=
// alpha p, r -= alpha q, partials of r^T r into u.red_rr -- and the map is
// applied to the new r (`in` is r then, and `dotwith` too): the update and the
// preconditioner share one pass over the rows.
struct UpdArgs {
  double* x;
  double* r;
  const double* p;
  const double* q;
  const double* red_pq;
  int nblk_pq;
  double* red_rr;
  DevScalars* sc;
  int it;
};

template <typename PT, int NC4, bool UPD>
__global__ __launch_bounds__(256) void prec_mid_mfma_kernel(const PT* part, int ksplit, int ldp,
                                                            const double* in, int64_t n, int r,
                                                            const double* UV, const double* D,
                                                            double* out, const double* dotwith,
                                                            double* red, const int32_t* done,
                                                            UpdArgs u) {
  if (UPD ? u.sc->done != 0 : is_done(done)) return;
  double alpha = 0.0;
  if (UPD) {  // as update_xr_kernel
    if (u.it < 0) u.it = u.sc->it;  // captured loop: the device counter
    const double pq = sum_partials(u.red_pq, u.nblk_pq);
    const double rz = u.sc->rz[u.it & 1];
    if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rz)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        u.sc->pq = pq;
        u.sc->status = (isfinite(pq) && isfinite(rz)) ? CPHIFI_BREAKDOWN : CPHIFI_NUMERIC;
        u.sc->iters = u.it;
        u.sc->done = 1;
      }
      return;
    }
    alpha = rz / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) u.sc->pq = pq;
  }
  constexpr int RP = 4 * NC4;
  constexpr int LT = RP + 1;  // row stride of the per-wave tile (bank spread)
  extern __shared__ double lds[];
  double* uv = lds;                                   // RP x RP
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* wt = lds + RP * RP + wave * (16 * LT);     // 16 x LT
  for (int e = threadIdx.x; e < RP * RP; e += blockDim.x) {
    const int j = e / RP, c = e % RP;
    uv[e] = (j < r && c < r) ? UV[j * r + c] : 0.0;
  }
  __syncthreads();
  const int li = lane & 15, kk = lane >> 4, jj = lane & 3;
  const int orow = 4 * ((lane >> 2) & 3) + kk;
  double loc = 0.0, loc_rr = 0.0;
  for (int64_t rb = (int64_t)blockIdx.x * 4 + wave; rb * 16 < n; rb += (int64_t)gridDim.x * 4) {
    const int64_t row0 = rb * 16;
    if (UPD) {
      // Every load of the block's x, p, r, q first, then the updates: the
      // stores to x and r would otherwise hold each later load back (the
      // pointers may alias), one memory round trip per element.
      constexpr int EPL = 16 * RP / 64;  // elements per lane (= NC4)
      double xv[EPL], pv[EPL], rv[EPL], qv[EPL];
#pragma unroll
      for (int k = 0; k < EPL; ++k) {
        const int e = lane + 64 * k;
        const int i = e / RP, c = e % RP;
        const int64_t s = row0 + i;
        const bool on = s < n && c < r;
        const int64_t o = on ? s * r + c : 0;
        xv[k] = on ? u.x[o] : 0.0;
        pv[k] = on ? u.p[o] : 0.0;
        rv[k] = on ? u.r[o] : 0.0;
        qv[k] = on ? u.q[o] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < EPL; ++k) {
        const int e = lane + 64 * k;
        const int i = e / RP, c = e % RP;
        const int64_t s = row0 + i;
        double v = 0.0;
        if (s < n && c < r) {
          const int64_t o = s * r + c;
          u.x[o] = xv[k] + alpha * pv[k];
          v = rv[k] - alpha * qv[k];
          u.r[o] = v;
          loc_rr += v * v;
        }
        wt[i * LT + c] = v;
      }
    } else {
      for (int e = lane; e < 16 * RP; e += 64) {
        const int i = e / RP, c = e % RP;
        const int64_t s = row0 + i;
        double v = 0.0;
        if (s < n && c < r) {
          const int64_t o = s * r + c;
          v = part != nullptr ? part_sum(part, ksplit, n, ldp, s, c) : in[o];
        }
        wt[i * LT + c] = v;
      }
    }
    __builtin_amdgcn_wave_barrier();
    double acc[NC4];
#pragma unroll
    for (int c = 0; c < NC4; ++c) acc[c] = 0.0;
#pragma unroll
    for (int ks = 0; ks < NC4; ++ks) {  // (T U_V): k in groups of 4
      const double a = wt[li * LT + 4 * ks + kk];
#pragma unroll
      for (int c = 0; c < NC4; ++c)
        acc[c] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, uv[(4 * ks + kk) * RP + 4 * c + jj],
                                                    acc[c], 0, 0, 0);
    }
    const int64_t s = row0 + orow;
    double tv[UPD ? NC4 : 1];  // UPD: the updated r at this lane's outputs, for r^T z
#pragma unroll
    for (int c = 0; c < NC4; ++c) {
      const int col = 4 * c + jj;
      if (UPD) tv[c] = wt[orow * LT + col];
      acc[c] *= (s < n && col < r) ? D[s * r + col] : 0.0;
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = 0; c < NC4; ++c) wt[orow * LT + 4 * c + jj] = acc[c];
    __builtin_amdgcn_wave_barrier();
    double z[NC4];
#pragma unroll
    for (int c = 0; c < NC4; ++c) z[c] = 0.0;
#pragma unroll
    for (int ks = 0; ks < NC4; ++ks) {  // (. U_V^T)
      const double a = wt[li * LT + 4 * ks + kk];
#pragma unroll
      for (int c = 0; c < NC4; ++c)
        z[c] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, uv[(4 * c + jj) * RP + 4 * ks + kk], z[c],
                                                  0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < NC4; ++c) {
      const int col = 4 * c + jj;
      if (s < n && col < r) {
        out[s * r + col] = z[c];
        if (UPD)
          loc += tv[c] * z[c];
        else if (dotwith != nullptr)
          loc += dotwith[s * r + col] * z[c];
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (UPD) {
    const double b = block_sum(loc_rr);
    if (threadIdx.x == 0) u.red_rr[blockIdx.x] = b;
  }
  if (red != nullptr) {
    const double b = block_sum(loc);
    if (threadIdx.x == 0) red[blockIdx.x] = b;
  }
}

template <typename PT, bool UPD = false>
int launch_prec_mfma(int nc4, int blocks, const PT* part, int ksplit, int ldp, const double* in,
                     int64_t n, int r, const double* UV, const double* D, double* out,
                     const double* dotwith, double* red, const int32_t* done, hipStream_t st,
                     const UpdArgs& u = UpdArgs{}) {
  const size_t lds = sizeof(double) * ((size_t)16 * nc4 * nc4 + 4 * 16 * (4 * nc4 + 1));
  // (r > 60 needs more than the default 64 KB of dynamic LDS)
#define CPHIFI_PREC_CASE(K)                                                                   \
  case K:                                                                                     \
    if (lds > 65536)                                                                          \
      CPHIFI_HIP(hipFuncSetAttribute((const void*)prec_mid_mfma_kernel<PT, K, UPD>,           \
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));  \
    hipLaunchKernelGGL((prec_mid_mfma_kernel<PT, K, UPD>), dim3(blocks), dim3(256), lds, st,  \
                       part, ksplit, ldp, in, n, r, UV, D, out, dotwith, red, done, u);       \
    break;
  switch (nc4) {
    CPHIFI_PREC_CASE(1) CPHIFI_PREC_CASE(2) CPHIFI_PREC_CASE(3) CPHIFI_PREC_CASE(4)
    CPHIFI_PREC_CASE(5) CPHIFI_PREC_CASE(6) CPHIFI_PREC_CASE(7) CPHIFI_PREC_CASE(8)
    CPHIFI_PREC_CASE(9) CPHIFI_PREC_CASE(10) CPHIFI_PREC_CASE(11) CPHIFI_PREC_CASE(12)
    CPHIFI_PREC_CASE(13) CPHIFI_PREC_CASE(14) CPHIFI_PREC_CASE(15) CPHIFI_PREC_CASE(16)
    default:
      set_error("preconditioner: rank %d beyond %d", r, kMaxRank);
      return CPHIFI_INVALID_ARG;
  }
#undef CPHIFI_PREC_CASE
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

__global__ void axpby_kernel(double* y, double a, const double* x, double b, int64_t len,
                             const int32_t* done) {
  if (is_done(done)) return;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    y[e] = a * x[e] + b * y[e];
}

__global__ void copy_kernel(double* dst, const double* src, int64_t len) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

__global__ void fill_kernel(double* dst, double v, int64_t len) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = v;
}

__global__ void fill_i32_kernel(int32_t* dst, int32_t v, int64_t len) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = v;
}

// V = (A^T A) had (B^T B): the Gram of the Khatri-Rao product of the other
// modes' factors (Section 3, reused in Section 4.4.2).  One thread per entry
// of the upper triangle, each summed in a fixed order (gram_entry, shared with
// the batched solver's setup phase).
// V = (A^T A) had (B^T B): one workgroup per entry (a <= b); thread t adds
// rows t, t + 256, ... and the partial sums meet in a fixed order.  (One thread
// per entry, summing all I + J rows in sequence, took 0.35 ms at I = 1000,
// J = 200, r = 40: a chain of dependent loads per thread.)
__global__ __launch_bounds__(256) void gram_kernel(const double* A, int64_t I, const double* B,
                                                   int64_t J, int r, double* V) {
  __shared__ double red[2][4];
  // blockIdx.x enumerates the upper triangle row by row
  int a = 0, rem = blockIdx.x;
  while (rem >= r - a) {
    rem -= r - a;
    ++a;
  }
  const int b = a + rem;
  double ga = 0.0, gb = 0.0;
  for (int64_t i = threadIdx.x; i < I; i += 256) ga += A[i * r + a] * A[i * r + b];
  for (int64_t j = threadIdx.x; j < J; j += 256) gb += B[j * r + a] * B[j * r + b];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    ga += __shfl_xor(ga, off, 64);
    gb += __shfl_xor(gb, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = ga;
    red[1][threadIdx.x >> 6] = gb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double v = (((red[0][0] + red[0][1]) + red[0][2]) + red[0][3]) *
                     (((red[1][0] + red[1][1]) + red[1][2]) + red[1][3]);
    V[a * r + b] = v;
    V[b * r + a] = v;
  }
}

// Eigendecomposition of the r x r Gram V (eq. eigV) by one workgroup
// (jacobi_sym, shared with the batched solver's setup phase).
__global__ __launch_bounds__(256) void jacobi_kernel(const double* Vin, int r, double* UV,
                                                     double* dV) {
  __shared__ JacobiLds<kMaxRank> w;
  jacobi_sym<kMaxRank>(Vin, r, UV, dV, w, threadIdx.x);
}

__global__ void precond_diag_kernel(const double* dK, const double* dV, int64_t n, int r,
                                    double gamma, double lam, double rho, double* D) {
  const int64_t len = n * r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / r;
    const int c = (int)(e % r);
    D[e] = precond_entry(dK[s], dV[c], gamma, lam, rho);
  }
}

__global__ void clamp_kernel(const double* src, double* dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = fmax(src[e], 0.0);
}

// Destination offset of element (i, k): row-major, or the BF16 product's
// 16 x 64 tiles.
__device__ __forceinline__ int64_t dst_off(int64_t i, int64_t k, int64_t ld, bool tiled) {
  return tiled ? ((i >> 4) * (ld >> 6) + (k >> 6)) * 1024 + (i & 15) * 64 + (k & 63) : i * ld + k;
}

__global__ void scale_rows_kernel(double* __restrict__ out, const double* __restrict__ x,
                                  const double* __restrict__ s, int64_t n, int r,
                                  const int32_t* done) {
  if (done != nullptr && *done) return;
  const int64_t len = n * r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = s[e / r] * x[e];
}

__global__ void to_f32_kernel(float* __restrict__ dst, const double* __restrict__ src,
                              int64_t len) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

template <typename T>
__global__ void convert_kernel(const double* src, int64_t ld_src, int64_t n, T* dst,
                               int64_t ld_dst, bool tiled) {
  const int64_t len = n * ld_dst;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / ld_dst, k = e % ld_dst;
    dst[dst_off(i, k, ld_dst, tiled)] = (T)(k < n ? src[i * ld_src + k] : 0.0);
  }
}

// Tiled transpose-convert: dst[i][k] = src[k][i] (i, k < n), zero for k >= n.
template <typename T>
__global__ __launch_bounds__(256) void convert_t_kernel(const double* src, int64_t ld_src,
                                                        int64_t n, T* dst, int64_t ld_dst,
                                                        bool tiled) {
  __shared__ double tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.y * 32;  // dst row block
  const int64_t k0 = (int64_t)blockIdx.x * 32;  // dst column block
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t k = k0 + yy, i = i0 + tx;
    tile[yy][tx] = (k < n && i < n) ? src[k * ld_src + i] : 0.0;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t i = i0 + yy, k = k0 + tx;
    if (i < n && k < ld_dst) dst[dst_off(i, k, ld_dst, tiled)] = (T)tile[tx][yy];
  }
}

}  // namespace

int vec_blocks(int64_t len) {
  int64_t b = (len + 1023) / 1024;
  if (b < 1) b = 1;
  if (b > kMaxVecBlocks) b = kMaxVecBlocks;
  return (int)b;
}

static int grid_for(int64_t len) {
  int64_t b = (len + 255) / 256;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return (int)b;
}

int launch_reduce_partials(const void* part, bool is_float, int ksplit, int ldp, int64_t n,
                           int r, double* out, const double* dotwith, double* red,
                           int* nblk_out, const int32_t* done, hipStream_t st,
                           const double* rowscale) {
  const int nb = vec_blocks(n * r);
  if (is_float)
    hipLaunchKernelGGL(reduce_partials_kernel<float>, dim3(nb), dim3(256), 0, st,
                       (const float*)part, ksplit, ldp, n, r, out, dotwith, red, rowscale, done);
  else
    hipLaunchKernelGGL(reduce_partials_kernel<double>, dim3(nb), dim3(256), 0, st,
                       (const double*)part, ksplit, ldp, n, r, out, dotwith, red, rowscale,
                       done);
  CPHIFI_CHECK_LAUNCH();
  if (nblk_out) *nblk_out = nb;
  return CPHIFI_OK;
}

int launch_apply_finish(const void* part, bool is_float, int ksplit, int ldp, int64_t n, int r,
                        const double* xhat, const double* p, const double* dscale, double lam,
                        double rho, double* q, double* red, int* nblk_out, const int32_t* done,
                        hipStream_t st) {
  const int nb = vec_blocks(n * r);
  if (is_float)
    hipLaunchKernelGGL(apply_finish_kernel<float>, dim3(nb), dim3(256), 0, st, (const float*)part,
                       ksplit, ldp, n, r, xhat, p, dscale, lam, rho, q, red, done);
  else
    hipLaunchKernelGGL(apply_finish_kernel<double>, dim3(nb), dim3(256), 0, st,
                       (const double*)part, ksplit, ldp, n, r, xhat, p, dscale, lam, rho, q, red,
                       done);
  CPHIFI_CHECK_LAUNCH();
  if (nblk_out) *nblk_out = nb;
  return CPHIFI_OK;
}

int launch_dot(const double* a, const double* b, int64_t len, double* red, int* nblk_out,
               const int32_t* done, hipStream_t st) {
  const int nb = vec_blocks(len);
  hipLaunchKernelGGL(dot_kernel, dim3(nb), dim3(256), 0, st, a, b, len, red, done);
  CPHIFI_CHECK_LAUNCH();
  if (nblk_out) *nblk_out = nb;
  return CPHIFI_OK;
}

int launch_update_prec(double* x, double* r, const double* p, const double* q, int64_t n,
                       int rank, const double* UV, const double* D, double* z,
                       const double* red_pq, int nblk_pq, double* red_rr, double* red_rz,
                       int* nblk_out, DevScalars* sc, int it, hipStream_t st) {
  const int nb = (int)std::min<int64_t>(kMaxVecBlocks, (n + 63) / 64);
  UpdArgs u{x, r, p, q, red_pq, nblk_pq, red_rr, sc, it};
  const int rc = launch_prec_mfma<double, true>((rank + 3) / 4, nb, nullptr, 1, 0, r, n, rank,
                                                UV, D, z, nullptr, red_rz, nullptr, st, u);
  if (rc != CPHIFI_OK) return rc;
  if (nblk_out) *nblk_out = nb;
  return CPHIFI_OK;
}

int launch_update_xr(double* x, double* r, const double* p, const double* q, int64_t len,
                     const double* red_pq, int nblk_pq, double* red_rr, int* nblk_out,
                     DevScalars* sc, int it, hipStream_t st) {
  const int nb = vec_blocks(len);
  hipLaunchKernelGGL(update_xr_kernel, dim3(nb), dim3(256), 0, st, x, r, p, q, len, red_pq,
                     nblk_pq, red_rr, sc, it);
  CPHIFI_CHECK_LAUNCH();
  if (nblk_out) *nblk_out = nb;
  return CPHIFI_OK;
}

int launch_check_conv(const double* red_rr, int nblk, DevScalars* sc, int it, double* hist,
                      int hist_len, int32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(check_conv_kernel, dim3(1), dim3(256), 0, st, red_rr, nblk, sc, it, hist,
                     hist_len, flag);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_prec_mid(const void* part, bool is_float, int ksplit, int ldp, const double* in,
                    int64_t n, int r, const double* UV, const double* D, double* out,
                    const double* dotwith, double* red, int* nblk_out, const int32_t* done,
                    hipStream_t st) {
  // 16 rows per wave and step, 4 waves per block
  const int nb = (int)std::min<int64_t>(kMaxVecBlocks, (n + 63) / 64);
  const int nc4 = (r + 3) / 4;
  const int rc = is_float ? launch_prec_mfma<float>(nc4, nb, (const float*)part, ksplit, ldp, in,
                                                    n, r, UV, D, out, dotwith, red, done, st)
                          : launch_prec_mfma<double>(nc4, nb, (const double*)part, ksplit, ldp,
                                                     in, n, r, UV, D, out, dotwith, red, done,
                                                     st);
  if (rc != CPHIFI_OK) return rc;
  if (nblk_out) *nblk_out = nb;
  return CPHIFI_OK;
}

int launch_update_p(double* p, const double* z, int64_t len, const double* red_rz, int nblk,
                    DevScalars* sc, int it, hipStream_t st) {
  hipLaunchKernelGGL(update_p_kernel, dim3(vec_blocks(len)), dim3(256), 0, st, p, z, len, red_rz,
                     nblk, sc, it);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_pcg_init(DevScalars* sc, const double* red_bb, int nblk_bb, const double* red_rr,
                    int nblk_rr, const double* red_rz, int nblk_rz, double tol, double* hist,
                    int hist_len, hipStream_t st) {
  hipLaunchKernelGGL(pcg_init_kernel, dim3(1), dim3(256), 0, st, sc, red_bb, nblk_bb, red_rr,
                     nblk_rr, red_rz, nblk_rz, tol, hist, hist_len);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_store_sum(const double* red, int nblk, DevScalars* sc, int slot, hipStream_t st) {
  hipLaunchKernelGGL(store_sum_kernel, dim3(1), dim3(256), 0, st, red, nblk, sc, slot);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_mirror(const DevScalars* src, DevScalars* dst, hipStream_t st) {
  hipLaunchKernelGGL(mirror_kernel, dim3(1), dim3(64), 0, st, src, dst);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_axpby(double* y, double a, const double* x, double b, int64_t len,
                 const int32_t* done, hipStream_t st) {
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(len)), dim3(256), 0, st, y, a, x, b, len, done);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_copy(double* dst, const double* src, int64_t len, hipStream_t st) {
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(len)), dim3(256), 0, st, dst, src, len);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_fill(double* dst, double v, int64_t len, hipStream_t st) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(len)), dim3(256), 0, st, dst, v, len);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_fill_i32(int32_t* dst, int32_t v, int64_t len, hipStream_t st) {
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(len)), dim3(256), 0, st, dst, v, len);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_gram(const double* A, int64_t I, const double* B, int64_t J, int r, double* V,
                hipStream_t st) {
  hipLaunchKernelGGL(gram_kernel, dim3(r * (r + 1) / 2), dim3(256), 0, st, A, I, B, J, r, V);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_jacobi_eig(const double* V, int r, double* UV, double* dV, hipStream_t st) {
  if (r < 1 || r > kMaxRank) {
    set_error("jacobi: bad rank %d", r);
    return CPHIFI_INVALID_ARG;
  }
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(256), 0, st, V, r, UV, dV);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_precond_diag(const double* dK, const double* dV, int64_t n, int r, double gamma,
                        double lam, double rho, double* D, hipStream_t st) {
  hipLaunchKernelGGL(precond_diag_kernel, dim3(grid_for(n * r)), dim3(256), 0, st, dK, dV, n, r,
                     gamma, lam, rho, D);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_clamp_nonneg(const double* src, double* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(clamp_kernel, dim3(grid_for(n)), dim3(256), 0, st, src, dst, n);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_scale_rows(double* out, const double* x, const double* s, int64_t n, int r,
                      const int32_t* done, hipStream_t st) {
  hipLaunchKernelGGL(scale_rows_kernel, dim3(vec_blocks(n * r)), dim3(kVecThreads), 0, st, out,
                     x, s, n, r, done);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_to_f32(float* dst, const double* src, int64_t len, hipStream_t st) {
  if (len <= 0) return CPHIFI_OK;
  hipLaunchKernelGGL(to_f32_kernel, dim3(grid_for(len)), dim3(256), 0, st, dst, src, len);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

int launch_convert_lowp(Elt elt, bool transpose, const double* src, int64_t ld_src, int64_t n,
                        void* dst, int64_t ld_dst, hipStream_t st, bool tiled) {
  if (ld_dst < n || (tiled && (elt != Elt::BF16 || ld_dst % 64 != 0))) {
    set_error("convert: ld_dst < n, or a tiled copy that is not BF16 with ld_dst %% 64 == 0");
    return CPHIFI_INVALID_ARG;
  }
  if (!transpose) {
    const int g = grid_for(n * ld_dst);
    if (elt == Elt::F32)
      hipLaunchKernelGGL(convert_kernel<float>, dim3(g), dim3(256), 0, st, src, ld_src, n,
                         (float*)dst, ld_dst, tiled);
    else if (elt == Elt::BF16)
      hipLaunchKernelGGL(convert_kernel<__bf16>, dim3(g), dim3(256), 0, st, src, ld_src, n,
                         (__bf16*)dst, ld_dst, tiled);
    else
      hipLaunchKernelGGL(convert_kernel<double>, dim3(g), dim3(256), 0, st, src, ld_src, n,
                         (double*)dst, ld_dst, tiled);
  } else {
    dim3 grid((unsigned)((ld_dst + 31) / 32), (unsigned)((n + 31) / 32));
    if (elt == Elt::F32)
      hipLaunchKernelGGL(convert_t_kernel<float>, grid, dim3(256), 0, st, src, ld_src, n,
                         (float*)dst, ld_dst, tiled);
    else if (elt == Elt::BF16)
      hipLaunchKernelGGL(convert_t_kernel<__bf16>, grid, dim3(256), 0, st, src, ld_src, n,
                         (__bf16*)dst, ld_dst, tiled);
    else
      hipLaunchKernelGGL(convert_t_kernel<double>, grid, dim3(256), 0, st, src, ld_src, n,
                         (double*)dst, ld_dst, tiled);
  }
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

}  // namespace cphifi
