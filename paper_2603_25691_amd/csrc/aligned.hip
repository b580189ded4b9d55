// Solvers of the aligned subproblem (Section 3): every entry of the data
// tensor is observed, and the RKHS factor solves
//
//     (V kron K + lambda I) vec(W) = vec(B),   V = Z^T Z,  B = T Z
//
// (eq. aligned-solve).  Two methods, both on the eigendecomposition of K:
//
//  * the decoupled direct solve of Section 3.2 (eq. W-decoupled):
//      W = U_K ((U_K^T B U_V) had D) U_V^T,  D(s, c) = 1 / (dV_c dK_s + lambda),
//    one FP64 product with U_K^T, the r x r middle step on MFMA, one product
//    with U_K;
//  * PCG on the transformed system of Section 3.3: with Wbar = U_K^T W and
//    Bbar = U_K^T B, (V kron D_K + lambda I) vec(Wbar) = vec(Bbar), whose
//    product is D_K X V + lambda X (eq. pcg-matvec-ai) and whose diagonal
//    preconditioner is diag(V)_c dK_s + lambda (eq. precond-ai).  Every
//    iteration is n r^2 work, so the whole iteration loop runs in ONE
//    persistent single-workgroup kernel (no launch or host round trip per
//    iteration); W = U_K Wbar at the end.
//
// Both report the FP64 residual of the rotated system, ||Bbar - D_K Wbar V -
// lambda Wbar|| / ||Bbar||, which equals that of eq. aligned-solve for an
// orthogonal U_K.
#include "cphifi_internal.h"

#include <cmath>
#include <cstring>

using namespace cphifi;

namespace {

constexpr size_t kAlignA = 256;
constexpr int kPcgThreads = 1024;

size_t align_a(size_t v) { return (v + kAlignA - 1) / kAlignA * kAlignA; }
int64_t round_a(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct AlignedLayout {
  size_t part, bbar, wbar, r, p, q, D, UV, dV, V, dKc, stats, total;
};

AlignedLayout aligned_layout(int64_t n, int64_t r) {
  AlignedLayout L{};
  const int64_t ldp = round_a(r, 16);
  const size_t nr = sizeof(double) * (size_t)n * r;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align_a(off);
    const size_t o = off;
    off += std::max<size_t>(bytes, 1);
    return o;
  };
  L.part = take(sizeof(double) * (size_t)kMaxSplit * n * ldp);
  L.bbar = take(nr);
  L.wbar = take(nr);
  L.r = take(nr);
  L.p = take(nr);
  L.q = take(nr);
  L.D = take(nr);
  L.UV = take(sizeof(double) * r * r);
  L.dV = take(sizeof(double) * r);
  L.V = take(sizeof(double) * r * r);
  L.dKc = take(sizeof(double) * n);
  L.stats = take(64);
  L.total = align_a(off);
  return L;
}

// Per-solve statistics written by the kernels (read by the host at the end).
struct AlignedStats {
  double rr, bb;       // ||residual||^2, ||Bbar||^2 of the final iterate
  int32_t iters, status;
};

__device__ double wg_sum(double v, double* ws) {
  // deterministic sum over the workgroup (kPcgThreads / 64 waves)
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) ws[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += ws[w];
  return t;
}

// D(s, c) = 1 / (max(dK_s, 0) v_c + lambda): v = dV (eq. W-decoupled).
__global__ void aligned_diag_kernel(const double* dK, const double* v, int64_t n, int r,
                                    double lam, double* D, double* dKc) {
  const int64_t len = n * r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / r;
    const int c = (int)(e % r);
    const double d = fmax(dK[s], 0.0);
    D[e] = 1.0 / (d * v[c] + lam);
    if (c == 0) dKc[s] = d;
  }
}

// out[s, c] = dKc[s] (X[s, :] V[:, c]) + lambda X[s, c]: eq. pcg-matvec-ai
// for one element (V in LDS, row-major r x r).
__device__ __forceinline__ double tmatvec(const double* __restrict__ X, const double* Vs,
                                          const double* __restrict__ dKc, double lam, int r,
                                          int64_t s, int c) {
  const double* xr = X + s * r;
  double acc = 0.0;
  for (int j = 0; j < r; ++j) acc += xr[j] * Vs[j * r + c];
  return dKc[s] * acc + lam * xr[c];
}

// The residual of the rotated system for Wbar: st->rr = ||Bbar - (D_K Wbar V +
// lambda Wbar)||^2, st->bb = ||Bbar||^2.  One workgroup.
__global__ __launch_bounds__(kPcgThreads) void aligned_resid_kernel(
    const double* __restrict__ Bbar, const double* __restrict__ Wbar,
    const double* __restrict__ V, const double* __restrict__ dKc, int64_t n, int r, double lam,
    AlignedStats* st) {
  __shared__ double Vs[kMaxRank * kMaxRank];
  __shared__ double ws[kPcgThreads / 64];
  for (int e = threadIdx.x; e < r * r; e += blockDim.x) Vs[e] = V[e];
  __syncthreads();
  const int64_t len = n * r;
  double rr = 0.0, bb = 0.0;
  for (int64_t e = threadIdx.x; e < len; e += blockDim.x) {
    const int64_t s = e / r;
    const int c = (int)(e % r);
    const double b = Bbar[e];
    const double res = b - tmatvec(Wbar, Vs, dKc, lam, r, s, c);
    rr += res * res;
    bb += b * b;
  }
  rr = wg_sum(rr, ws);
  bb = wg_sum(bb, ws);
  if (threadIdx.x == 0) {
    st->rr = rr;
    st->bb = bb;
  }
}

// Textbook PCG on (V kron D_K + lambda I) vec(X) = vec(Bbar) from X = 0 with
// the diagonal preconditioner diag(V)_c dK_s + lambda (eq. precond-ai), the
// whole loop in one workgroup.  Stops when ||r|| <= tol ||Bbar|| or after
// maxit iterations; breakdown (p^T A p <= 0 or r^T z <= 0) and NaN end it
// with that status.  Every sum is a fixed-order workgroup reduction.
__global__ __launch_bounds__(kPcgThreads) void aligned_pcg_kernel(
    const double* __restrict__ Bbar, const double* __restrict__ V,
    const double* __restrict__ dKc, int64_t n, int r, double lam, double tol, int maxit,
    double* __restrict__ X, double* __restrict__ R, double* __restrict__ P,
    double* __restrict__ Q, AlignedStats* st) {
  __shared__ double Vs[kMaxRank * kMaxRank];
  __shared__ double ws[kPcgThreads / 64];
  for (int e = threadIdx.x; e < r * r; e += blockDim.x) Vs[e] = V[e];
  __syncthreads();
  const int64_t len = n * r;
  auto minv = [&](int64_t e) {
    const int c = (int)(e % r);
    return 1.0 / (Vs[c * r + c] * dKc[e / r] + lam);
  };
  double bb = 0.0, rz = 0.0;
  for (int64_t e = threadIdx.x; e < len; e += blockDim.x) {
    const double b = Bbar[e];
    const double z = minv(e) * b;
    X[e] = 0.0;
    R[e] = b;
    P[e] = z;
    bb += b * b;
    rz += b * z;
  }
  bb = wg_sum(bb, ws);
  rz = wg_sum(rz, ws);
  int status = CPHIFI_NOT_CONVERGED, it = 0;
  double rr = bb;
  const double tol2 = tol * tol * bb;
  if (!isfinite(bb) || !isfinite(rz)) {
    status = CPHIFI_NUMERIC;
  } else if (bb == 0.0) {
    status = CPHIFI_OK;
  } else if (!(rz > 0.0)) {
    status = CPHIFI_BREAKDOWN;
  } else {
    for (it = 0; it < maxit;) {
      __syncthreads();  // P complete
      double pq = 0.0;
      for (int64_t e = threadIdx.x; e < len; e += blockDim.x) {
        const double qe = tmatvec(P, Vs, dKc, lam, r, e / r, (int)(e % r));
        Q[e] = qe;
        pq += P[e] * qe;
      }
      pq = wg_sum(pq, ws);
      if (!(pq > 0.0) || !isfinite(pq)) {
        status = isfinite(pq) ? CPHIFI_BREAKDOWN : CPHIFI_NUMERIC;
        break;
      }
      const double alpha = rz / pq;
      double rrl = 0.0;
      for (int64_t e = threadIdx.x; e < len; e += blockDim.x) {
        X[e] += alpha * P[e];
        const double re = R[e] - alpha * Q[e];
        R[e] = re;
        rrl += re * re;
      }
      rr = wg_sum(rrl, ws);
      ++it;
      if (!isfinite(rr)) {
        status = CPHIFI_NUMERIC;
        break;
      }
      if (rr <= tol2) {
        status = CPHIFI_OK;
        break;
      }
      double rzl = 0.0;
      for (int64_t e = threadIdx.x; e < len; e += blockDim.x) rzl += R[e] * minv(e) * R[e];
      const double rz_new = wg_sum(rzl, ws);
      if (!(rz_new > 0.0) || !isfinite(rz_new)) {
        status = isfinite(rz_new) ? CPHIFI_BREAKDOWN : CPHIFI_NUMERIC;
        break;
      }
      const double beta = rz_new / rz;
      rz = rz_new;
      for (int64_t e = threadIdx.x; e < len; e += blockDim.x)
        P[e] = minv(e) * R[e] + beta * P[e];
    }
  }
  if (threadIdx.x == 0) {
    st->iters = it;
    st->status = status;
  }
}

int check_aligned(const cphifi_aligned_desc* d, size_t* bytes_needed) {
  if (d == nullptr) {
    set_error("aligned: desc is NULL");
    return CPHIFI_INVALID_ARG;
  }
  if (d->n < 1 || d->n > INT32_MAX || d->r < 1 || d->r > kMaxRank || (d->ldk != 0 && d->ldk < d->n)) {
    set_error("aligned: bad sizes n=%lld r=%lld ldk=%lld", (long long)d->n, (long long)d->r,
              (long long)d->ldk);
    return CPHIFI_INVALID_ARG;
  }
  if (!(d->lambda > 0.0) || !std::isfinite(d->lambda)) {
    set_error("aligned: need lambda > 0 (got %g)", d->lambda);
    return CPHIFI_INVALID_ARG;
  }
  if (d->method != CPHIFI_ALIGNED_DECOUPLED && d->method != CPHIFI_ALIGNED_PCG) {
    set_error("aligned: unknown method %d", d->method);
    return CPHIFI_INVALID_ARG;
  }
  if (d->method == CPHIFI_ALIGNED_PCG && !(d->tol > 0.0)) {
    set_error("aligned: PCG needs tol > 0");
    return CPHIFI_INVALID_ARG;
  }
  if (bytes_needed) *bytes_needed = aligned_layout(d->n, d->r).total;
  return CPHIFI_OK;
}

#define TRYA(x)                      \
  do {                               \
    const int s_ = (x);              \
    if (s_ != CPHIFI_OK) return s_;  \
  } while (0)

}  // namespace

extern "C" {

int cphifi_aligned_workspace_bytes(const cphifi_aligned_desc* d, size_t* bytes) {
  clear_error();
  if (bytes == nullptr) {
    set_error("aligned_workspace_bytes: bytes is NULL");
    return CPHIFI_INVALID_ARG;
  }
  return check_aligned(d, bytes);
}

int cphifi_aligned_solve(const cphifi_aligned_desc* d, const cphifi_aligned_inputs* in,
                         double* W, void* workspace, size_t workspace_bytes, void* stream,
                         cphifi_solve_info* info) {
  clear_error();
  size_t need = 0;
  TRYA(check_aligned(d, &need));
  if (in == nullptr || in->UK == nullptr || in->dK == nullptr || in->Bm == nullptr ||
      W == nullptr || info == nullptr) {
    set_error("aligned: UK, dK, Bm, W and info are required");
    return CPHIFI_INVALID_ARG;
  }
  const bool have_v = in->V != nullptr;
  if (!have_v && (in->A == nullptr || in->B == nullptr || in->I < 1 || in->J < 1)) {
    set_error("aligned: give V, or the factors A (I x r) and B (J x r)");
    return CPHIFI_INVALID_ARG;
  }
  if (workspace == nullptr || workspace_bytes < need ||
      reinterpret_cast<uintptr_t>(workspace) % kAlignA != 0) {
    set_error("aligned: workspace must be >= %zu bytes and 256-byte aligned", need);
    return CPHIFI_INVALID_ARG;
  }
  double* hist = info->history;
  std::memset(info, 0, sizeof(*info));
  info->history = hist;
  const int64_t n = d->n;
  const int r = (int)d->r;
  const int64_t ldk = d->ldk > 0 ? d->ldk : n;
  const int ldp = (int)round_a(r, 16);
  hipStream_t st = (hipStream_t)stream;
  const AlignedLayout L = aligned_layout(n, r);
  char* ws = (char*)workspace;
  void* part = ws + L.part;
  double* bbar = (double*)(ws + L.bbar);
  double* wbar = (double*)(ws + L.wbar);
  double* D = (double*)(ws + L.D);
  double* UV = (double*)(ws + L.UV);
  double* dV = (double*)(ws + L.dV);
  double* dKc = (double*)(ws + L.dKc);
  AlignedStats* stats = (AlignedStats*)(ws + L.stats);
  const double* V = in->V;
  if (!have_v) {
    double* Vw = (double*)(ws + L.V);
    TRYA(launch_gram(in->A, in->I, in->B, in->J, r, Vw, st));
    V = Vw;
  }
  int num_cu = 256, dev = 0;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (num_cu <= 0) num_cu = 256;
  // UK holds eigenvector k in row k: U_K^T X is the row-major product on UK,
  // U_K X the transposed one.
  const GemmPlan gn = choose_gemm(Elt::F64, false, n, r, num_cu);
  const GemmPlan gt = choose_gemm(Elt::F64, true, n, r, num_cu);
  TRYA(launch_gemm(Elt::F64, false, gn, in->UK, ldk, n, in->Bm, r, r, nullptr, part, nullptr, st));
  TRYA(launch_reduce_partials(part, false, gn.ksplit, ldp, n, r, bbar, nullptr, nullptr, nullptr,
                              nullptr, st));
  if (d->method == CPHIFI_ALIGNED_DECOUPLED) {
    // eq. eigV, then D and the r x r middle step of eq. W-decoupled
    TRYA(launch_jacobi_eig(V, r, UV, dV, st));
    hipLaunchKernelGGL(aligned_diag_kernel, dim3((unsigned)std::min<int64_t>(1024, (n * r + 255) / 256)),
                       dim3(256), 0, st, in->dK, dV, n, r, d->lambda, D, dKc);
    CPHIFI_CHECK_LAUNCH();
    TRYA(launch_prec_mid(nullptr, false, 1, ldp, bbar, n, r, UV, D, wbar, nullptr, nullptr,
                         nullptr, nullptr, st));
    info->iters = 0;
  } else {
    TRYA(launch_clamp_nonneg(in->dK, dKc, n, st));
    const int maxit = d->maxit > 0 ? d->maxit : 500;
    hipLaunchKernelGGL(aligned_pcg_kernel, dim3(1), dim3(kPcgThreads), 0, st, bbar, V, dKc, n, r,
                       d->lambda, d->tol, maxit, wbar, (double*)(ws + L.r), (double*)(ws + L.p),
                       (double*)(ws + L.q), stats);
    CPHIFI_CHECK_LAUNCH();
  }
  // W = U_K Wbar
  TRYA(launch_gemm(Elt::F64, true, gt, in->UK, ldk, n, wbar, r, r, nullptr, part, nullptr, st));
  TRYA(launch_reduce_partials(part, false, gt.ksplit, ldp, n, r, W, nullptr, nullptr, nullptr,
                              nullptr, st));
  hipLaunchKernelGGL(aligned_resid_kernel, dim3(1), dim3(kPcgThreads), 0, st, bbar, wbar, V, dKc,
                     n, r, d->lambda, stats);
  CPHIFI_CHECK_LAUNCH();
  AlignedStats h{};
  CPHIFI_HIP(hipMemcpyAsync(&h, stats, sizeof(h), hipMemcpyDeviceToHost, st));
  CPHIFI_HIP(hipStreamSynchronize(st));
  const double rel = h.bb > 0.0 ? std::sqrt(h.rr / h.bb) : (h.rr > 0.0 ? INFINITY : 0.0);
  info->relres_true = rel;
  info->relres_recursive = rel;
  int status = CPHIFI_OK;
  if (d->method == CPHIFI_ALIGNED_PCG) {
    info->iters = h.iters;
    status = h.status;
    if (status == CPHIFI_OK && !(rel <= 10.0 * d->tol)) status = CPHIFI_NOT_CONVERGED;
  }
  if (!std::isfinite(rel)) status = CPHIFI_NUMERIC;
  info->status = status;
  return status;
}

}  // extern "C"
