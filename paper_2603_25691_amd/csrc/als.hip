// CP-HIFI alternating optimisation (Section 2, eq. cp-hifi-subproblem) for a
// 3-way tensor whose three modes are all infinite-dimensional, as in the
// paper's unaligned vortex and Miranda runs (Section 5.2).
//
// Mode k's factor is A_k = K_k W_k.  With the other two factors fixed, W_k
// solves the unaligned subproblem of eq. unaligned-infinite-1: the
// observations grouped by their mode-k index (CSR), the Khatri-Rao row of an
// observation the Hadamard product of the other two factors' rows at its
// indices.  Each mode keeps one subproblem plan for the whole run (its
// observation lists are fixed; V, eig(V), D and the FP32 factor copies are
// redone by the per-solve setup because the other factors move), so an outer
// iteration is three warm-started subproblem solves, three products
// A_k = K_k W_k and one pass over the observations for the relative error
// ||y - model|| / ||y|| that the stopping rule watches.
#include "cphifi_internal.h"
#include "plan.h"

#include <cmath>
#include <cstring>

using namespace cphifi;

namespace {

constexpr size_t kAlignL = 256;
constexpr int kErrThreads = 256;
constexpr int kErrBlocks = 512;

size_t align_l(size_t v) { return (v + kAlignL - 1) / kAlignL * kAlignL; }

// Workspace: per mode the CSR lists, the permuted values and the plan's own
// workspace; the three factors; the error partials.
struct AlsLayout {
  size_t ptr[3], oi[3], oj[3], y[3], plan[3];
  size_t F[3];
  size_t err;
  size_t total;
};

cphifi_ui_desc mode_desc(const cphifi_als_desc& d, int k) {
  const int a = k == 0 ? 1 : 0, b = k == 2 ? 1 : 2;
  cphifi_ui_desc u{};
  u.n = d.n[k];
  u.r = d.r;
  u.q = d.q;
  u.I = d.n[a];
  u.J = d.n[b];
  u.ldk = d.n[k];
  u.lambda = d.lambda[k];
  u.rho = d.rho;
  u.gamma = 0.0;
  u.tol = d.tol;
  u.inner_tol = 0.0;
  u.precision = d.precision;
  u.flags = d.flags | CPHIFI_FLAG_WARM_START;
  u.maxit = d.maxit;
  return u;
}

int als_layout(const cphifi_als_desc& d, AlsLayout* L) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align_l(off);
    const size_t o = off;
    off += std::max<size_t>(bytes, 1);
    return o;
  };
  for (int k = 0; k < 3; ++k) {
    const cphifi_ui_desc u = mode_desc(d, k);
    size_t pb = 0;
    if (!d.finite[k]) {
      const int rc = cphifi_ui_workspace_bytes(&u, &pb);
      if (rc != CPHIFI_OK) return rc;
    }
    L->ptr[k] = take(sizeof(int32_t) * (size_t)(d.n[k] + 1));
    L->oi[k] = take(sizeof(int32_t) * (size_t)d.q);
    L->oj[k] = take(sizeof(int32_t) * (size_t)d.q);
    L->y[k] = take(sizeof(double) * (size_t)d.q);
    L->plan[k] = take(pb);
  }
  for (int k = 0; k < 3; ++k) L->F[k] = take(sizeof(double) * (size_t)d.n[k] * d.r);
  L->err = take(sizeof(double) * 2 * (kErrBlocks + 1));
  L->total = align_l(off);
  return CPHIFI_OK;
}

int check_desc(const cphifi_als_desc* d) {
  if (d == nullptr) {
    set_error("als: desc is NULL");
    return CPHIFI_INVALID_ARG;
  }
  for (int k = 0; k < 3; ++k)
    if (d->n[k] < 1 || d->n[k] > INT32_MAX || (!d->finite[k] && !(d->lambda[k] > 0.0))) {
      set_error("als: mode %d needs n >= 1 and (an RKHS mode) lambda > 0", k);
      return CPHIFI_INVALID_ARG;
    }
  if (d->q < 1 || d->q > INT32_MAX || d->r < 1 || d->r > kMaxRank || !(d->rho > 0.0) ||
      !(d->tol > 0.0) || d->max_outer < 1 || !(d->als_tol >= 0.0)) {
    set_error("als: need 1 <= q < 2^31, 1 <= r <= %d, rho > 0, tol > 0, max_outer >= 1, "
              "als_tol >= 0", kMaxRank);
    return CPHIFI_INVALID_ARG;
  }
  return CPHIFI_OK;
}

// Partials of sum (y_l - m_l)^2 and sum y_l^2, m_l = sum_c F0(i0,c) F1(i1,c) F2(i2,c);
// block b writes part[2 b], part[2 b + 1].  Fixed grid and order: deterministic.
__global__ __launch_bounds__(kErrThreads) void als_error_kernel(
    const int32_t* __restrict__ coords, const double* __restrict__ y, int64_t q, int r,
    const double* __restrict__ F0, const double* __restrict__ F1,
    const double* __restrict__ F2, double* __restrict__ part) {
  double ee = 0.0, yy = 0.0;
  for (int64_t l = (int64_t)blockIdx.x * kErrThreads + threadIdx.x; l < q;
       l += (int64_t)gridDim.x * kErrThreads) {
    const double* a = F0 + (int64_t)coords[3 * l] * r;
    const double* b = F1 + (int64_t)coords[3 * l + 1] * r;
    const double* c = F2 + (int64_t)coords[3 * l + 2] * r;
    double m = 0.0;
    for (int j = 0; j < r; ++j) m += a[j] * b[j] * c[j];
    const double v = y[l];
    ee += (v - m) * (v - m);
    yy += v * v;
  }
  __shared__ double s_e[kErrThreads / kWave], s_y[kErrThreads / kWave];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    ee += __shfl_xor(ee, off, 64);
    yy += __shfl_xor(yy, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_e[threadIdx.x >> 6] = ee;
    s_y[threadIdx.x >> 6] = yy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double te = 0.0, ty = 0.0;
    for (int w = 0; w < kErrThreads / kWave; ++w) {
      te += s_e[w];
      ty += s_y[w];
    }
    part[2 * blockIdx.x] = te;
    part[2 * blockIdx.x + 1] = ty;
  }
}

// Finite-dimensional mode (Section 2: no regulariser, a CP-ALS block with
// missing data): row i of A_k solves (sum_l z_l z_l^T + rho I) a_i = sum_l y_l z_l
// over the observations l of row i, z_l = Fa(oi_l,:) had Fb(oj_l,:).  One
// workgroup per row: the observations pass through LDS in chunks, each
// thread accumulates its entries of the Gram matrix in a fixed order, then a
// Cholesky factorisation and the two triangular solves in LDS.
constexpr int kFinChunk = 32;
constexpr int kFinPer = kMaxRank * kMaxRank / kErrThreads;  // Gram entries per thread

__global__ __launch_bounds__(kErrThreads) void als_finite_kernel(
    const int32_t* __restrict__ ptr, const int32_t* __restrict__ oi,
    const int32_t* __restrict__ oj, const double* __restrict__ y,
    const double* __restrict__ Fa, const double* __restrict__ Fb, int64_t n, int r, double rho,
    double* __restrict__ Aout) {
  __shared__ double G[kMaxRank * kMaxRank];
  __shared__ double zs[kFinChunk * kMaxRank];
  __shared__ double ys[kFinChunk];
  __shared__ double rhs[kMaxRank];
  const int tid = threadIdx.x;
  for (int64_t row = blockIdx.x; row < n; row += gridDim.x) {
    double acc[kFinPer];
#pragma unroll
    for (int m = 0; m < kFinPer; ++m) acc[m] = 0.0;
    double racc = 0.0;
    const int32_t l_end = ptr[row + 1];
    for (int32_t l0 = ptr[row]; l0 < l_end; l0 += kFinChunk) {
      const int cnt = min(kFinChunk, l_end - l0);
      __syncthreads();  // zs / ys of the previous chunk consumed
      for (int e = tid; e < cnt * r; e += kErrThreads) {
        const int l = e / r, c = e % r;
        zs[l * r + c] = Fa[(int64_t)oi[l0 + l] * r + c] * Fb[(int64_t)oj[l0 + l] * r + c];
      }
      for (int e = tid; e < cnt; e += kErrThreads) ys[e] = y[l0 + e];
      __syncthreads();
#pragma unroll
      for (int m = 0; m < kFinPer; ++m) {
        const int e = tid + m * kErrThreads;
        if (e < r * r) {
          const int a = e / r, b = e % r;
          for (int l = 0; l < cnt; ++l) acc[m] = fma(zs[l * r + a], zs[l * r + b], acc[m]);
        }
      }
      if (tid < r)
        for (int l = 0; l < cnt; ++l) racc = fma(ys[l], zs[l * r + tid], racc);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kFinPer; ++m) {
      const int e = tid + m * kErrThreads;
      if (e < r * r) G[e] = acc[m] + ((e / r == e % r) ? rho : 0.0);
    }
    if (tid < r) rhs[tid] = racc;
    __syncthreads();
    // Cholesky G = L L^T (lower triangle in place), column by column
    for (int k = 0; k < r; ++k) {
      if (tid == 0) G[k * r + k] = sqrt(G[k * r + k]);
      __syncthreads();
      for (int i = k + 1 + tid; i < r; i += kErrThreads) G[i * r + k] /= G[k * r + k];
      __syncthreads();
      for (int e = tid; e < r * r; e += kErrThreads) {
        const int i = e / r, j = e % r;
        if (j > k && i >= j) G[i * r + j] -= G[i * r + k] * G[j * r + k];
      }
      __syncthreads();
    }
    // L z = rhs, then L^T a = z (rhs overwritten)
    for (int k = 0; k < r; ++k) {
      if (tid == 0) rhs[k] /= G[k * r + k];
      __syncthreads();
      for (int i = k + 1 + tid; i < r; i += kErrThreads) rhs[i] -= G[i * r + k] * rhs[k];
      __syncthreads();
    }
    for (int k = r - 1; k >= 0; --k) {
      if (tid == 0) rhs[k] /= G[k * r + k];
      __syncthreads();
      for (int i = tid; i < k; i += kErrThreads) rhs[i] -= G[k * r + i] * rhs[k];
      __syncthreads();
    }
    if (tid < r) Aout[row * r + tid] = rhs[tid];
  }
}

// out[0], out[1] = sums of the partials in block order.
__global__ void als_error_sum_kernel(const double* __restrict__ part, int nblk,
                                     double* __restrict__ out) {
  if (threadIdx.x == 0) {
    double te = 0.0, ty = 0.0;
    for (int b = 0; b < nblk; ++b) {
      te += part[2 * b];
      ty += part[2 * b + 1];
    }
    out[0] = te;
    out[1] = ty;
  }
}

}  // namespace

struct cphifi_als {
  cphifi_als_desc d{};
  cphifi_als_inputs in{};
  hipStream_t st = nullptr;
  AlsLayout L{};
  char* ws = nullptr;
  cphifi_plan* plan[3]{};
  double* F[3]{};
  double* y[3]{};
  double* err = nullptr;
  int err_blocks = 1;
};

namespace {

void destroy_plans(cphifi_als* a) {
  for (int k = 0; k < 3; ++k) {
    if (a->plan[k] != nullptr) (void)cphifi_ui_plan_destroy(a->plan[k]);
    a->plan[k] = nullptr;
  }
}

// ||y - model|| / ||y|| on the current factors.
int rel_error(cphifi_als* a, double* out) {
  const int64_t q = a->d.q;
  hipLaunchKernelGGL(als_error_kernel, dim3(a->err_blocks), dim3(kErrThreads), 0, a->st,
                     a->in.coords, a->in.y, q, (int)a->d.r, a->F[0], a->F[1], a->F[2], a->err);
  CPHIFI_CHECK_LAUNCH();
  double* sums = a->err + 2 * kErrBlocks;
  hipLaunchKernelGGL(als_error_sum_kernel, dim3(1), dim3(64), 0, a->st, a->err, a->err_blocks,
                     sums);
  CPHIFI_CHECK_LAUNCH();
  double h[2] = {0.0, 0.0};
  CPHIFI_HIP(hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, a->st));
  CPHIFI_HIP(hipStreamSynchronize(a->st));
  if (!std::isfinite(h[0]) || !std::isfinite(h[1])) {
    set_error("als: non-finite model error");
    return CPHIFI_NUMERIC;
  }
  *out = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : 0.0;
  return CPHIFI_OK;
}

}  // namespace

extern "C" {

int cphifi_als_workspace_bytes(const cphifi_als_desc* d, size_t* bytes) {
  clear_error();
  if (bytes == nullptr) {
    set_error("als: bytes is NULL");
    return CPHIFI_INVALID_ARG;
  }
  int rc = check_desc(d);
  if (rc != CPHIFI_OK) return rc;
  AlsLayout L{};
  rc = als_layout(*d, &L);
  if (rc != CPHIFI_OK) return rc;
  *bytes = L.total;
  return CPHIFI_OK;
}

int cphifi_als_create(cphifi_als** out, const cphifi_als_desc* d, const cphifi_als_inputs* in,
                      void* workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  if (out == nullptr || in == nullptr || in->coords == nullptr || in->y == nullptr) {
    set_error("als: out, inputs, coords and y are required");
    return CPHIFI_INVALID_ARG;
  }
  *out = nullptr;
  int rc = check_desc(d);
  if (rc != CPHIFI_OK) return rc;
  for (int k = 0; k < 3; ++k)
    if (!d->finite[k] && (in->K[k] == nullptr || in->UK[k] == nullptr || in->dK[k] == nullptr)) {
      set_error("als: K, UK and dK of RKHS mode %d are required", k);
      return CPHIFI_INVALID_ARG;
    }
  AlsLayout L{};
  rc = als_layout(*d, &L);
  if (rc != CPHIFI_OK) return rc;
  if (workspace == nullptr || workspace_bytes < L.total ||
      reinterpret_cast<uintptr_t>(workspace) % kAlignL != 0) {
    set_error("als: workspace must be >= %zu bytes and 256-byte aligned", L.total);
    return CPHIFI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  const int64_t q = d->q;
  // Observations to the host once: range checks and the per-mode CSR lists.
  std::vector<int32_t> co((size_t)q * 3);
  std::vector<double> yh((size_t)q);
  CPHIFI_HIP(hipMemcpyAsync(co.data(), in->coords, sizeof(int32_t) * co.size(),
                            hipMemcpyDeviceToHost, st));
  CPHIFI_HIP(hipMemcpyAsync(yh.data(), in->y, sizeof(double) * yh.size(), hipMemcpyDeviceToHost,
                            st));
  CPHIFI_HIP(hipStreamSynchronize(st));
  for (int64_t l = 0; l < q; ++l)
    for (int k = 0; k < 3; ++k)
      if (co[3 * l + k] < 0 || co[3 * l + k] >= d->n[k]) {
        set_error("als: coordinate %d of entry %lld is %d, outside [0, %lld)", k, (long long)l,
                  co[3 * l + k], (long long)d->n[k]);
        return CPHIFI_INVALID_ARG;
      }
  cphifi_als* a = new cphifi_als();
  a->d = *d;
  a->in = *in;
  a->st = st;
  a->L = L;
  a->ws = (char*)workspace;
  for (int k = 0; k < 3; ++k) {
    a->F[k] = (double*)(a->ws + L.F[k]);
    a->y[k] = (double*)(a->ws + L.y[k]);
  }
  a->err = (double*)(a->ws + L.err);
  a->err_blocks = (int)std::min<int64_t>(kErrBlocks, (q + kErrThreads - 1) / kErrThreads);
  // Per mode: counting sort of the entries by their mode-k index (stable, so
  // within a segment the entries keep the caller's order).
  std::vector<int32_t> ptr, oi, oj;
  std::vector<double> ys;
  for (int k = 0; k < 3; ++k) {
    const int m0 = k == 0 ? 1 : 0, m1 = k == 2 ? 1 : 2;
    const int64_t n = d->n[k];
    ptr.assign((size_t)n + 1, 0);
    for (int64_t l = 0; l < q; ++l) ++ptr[(size_t)co[3 * l + k] + 1];
    for (int64_t s = 0; s < n; ++s) ptr[s + 1] += ptr[s];
    std::vector<int32_t> pos(ptr.begin(), ptr.end() - 1);
    oi.assign((size_t)q, 0);
    oj.assign((size_t)q, 0);
    ys.assign((size_t)q, 0.0);
    for (int64_t l = 0; l < q; ++l) {
      const int32_t dst = pos[co[3 * l + k]]++;
      oi[dst] = co[3 * l + m0];
      oj[dst] = co[3 * l + m1];
      ys[dst] = yh[l];
    }
    int32_t* dptr = (int32_t*)(a->ws + L.ptr[k]);
    int32_t* doi = (int32_t*)(a->ws + L.oi[k]);
    int32_t* doj = (int32_t*)(a->ws + L.oj[k]);
    hipError_t e = hipSuccess;
    if ((e = hipMemcpyAsync(dptr, ptr.data(), sizeof(int32_t) * ptr.size(),
                            hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(doi, oi.data(), sizeof(int32_t) * q, hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(doj, oj.data(), sizeof(int32_t) * q, hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(a->y[k], ys.data(), sizeof(double) * q, hipMemcpyHostToDevice,
                            st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
      set_error("als: upload of mode %d lists failed: %s", k,
                hipGetErrorString(e));
      destroy_plans(a);
      delete a;
      return CPHIFI_HIP_ERROR;
    }
    if (d->finite[k]) continue;  // a finite mode has no subproblem plan
    const cphifi_ui_desc u = mode_desc(*d, k);
    cphifi_ui_inputs ui{};
    ui.K = in->K[k];
    ui.UK = in->UK[k];
    ui.dK = in->dK[k];
    ui.obs_ptr = dptr;
    ui.obs_i = doi;
    ui.obs_j = doj;
    ui.A = a->F[m0];
    ui.B = a->F[m1];
    size_t pb = 0;
    (void)cphifi_ui_workspace_bytes(&u, &pb);
    rc = cphifi_ui_plan_create(&a->plan[k], &u, &ui, a->ws + L.plan[k], pb, stream);
    if (rc != CPHIFI_OK) {
      destroy_plans(a);
      delete a;
      return rc;
    }
  }
  *out = a;
  return CPHIFI_OK;
}

int cphifi_als_run(cphifi_als* a, double* const* W, double* const* F, cphifi_als_info* info) {
  clear_error();
  if (a == nullptr || W == nullptr || info == nullptr || W[0] == nullptr || W[1] == nullptr ||
      W[2] == nullptr) {
    set_error("als_run: plan, W[3] and info are required");
    return CPHIFI_INVALID_ARG;
  }
  double* errors = info->errors;
  std::memset(info, 0, sizeof(*info));
  info->errors = errors;
  int rc = CPHIFI_OK;
  const int64_t r = a->d.r;
  for (int k = 0; k < 3; ++k) {
    if (a->d.finite[k]) {  // the factor is the unknown itself
      CPHIFI_HIP(hipMemcpyAsync(a->F[k], W[k], sizeof(double) * a->d.n[k] * r,
                                hipMemcpyDeviceToDevice, a->st));
    } else if ((rc = plan_times_K(a->plan[k], W[k], a->F[k])) != CPHIFI_OK) {
      return rc;
    }
  }
  double err = 0.0;
  if ((rc = rel_error(a, &err)) != CPHIFI_OK) return rc;
  if (errors != nullptr) errors[0] = err;
  for (int it = 0; it < a->d.max_outer; ++it) {
    for (int k = 0; k < 3; ++k) {
      if (a->d.finite[k]) {
        const int m0 = k == 0 ? 1 : 0, m1 = k == 2 ? 1 : 2;
        const int blocks = (int)std::min<int64_t>(a->d.n[k], 4096);
        hipLaunchKernelGGL(als_finite_kernel, dim3(blocks), dim3(kErrThreads), 0, a->st,
                           (const int32_t*)(a->ws + a->L.ptr[k]),
                           (const int32_t*)(a->ws + a->L.oi[k]),
                           (const int32_t*)(a->ws + a->L.oj[k]), a->y[k], a->F[m0], a->F[m1],
                           a->d.n[k], (int)r, a->d.rho, a->F[k]);
        CPHIFI_CHECK_LAUNCH();
        continue;
      }
      cphifi_solve_info si{};
      rc = cphifi_ui_solve_subproblem(a->plan[k], a->y[k], W[k], &si);
      if (rc == CPHIFI_NOT_CONVERGED) {
        ++info->capped;  // the iteration cap of the paper's runs: keep going
      } else if (rc != CPHIFI_OK) {
        const std::string why = cphifi_last_error();
        set_error("als: outer iteration %d, mode %d: %s", it, k, why.c_str());
        return rc;
      }
      info->inner_iters += si.iters;
      if ((rc = plan_times_K(a->plan[k], W[k], a->F[k])) != CPHIFI_OK) return rc;
    }
    const double prev = err;
    if ((rc = rel_error(a, &err)) != CPHIFI_OK) return rc;
    info->outer = it + 1;
    if (errors != nullptr) errors[it + 1] = err;
    if (std::fabs(prev - err) < a->d.als_tol) {
      info->converged = 1;
      break;
    }
  }
  info->rel_error = err;
  for (int k = 0; k < 3; ++k)
    if (a->d.finite[k])
      CPHIFI_HIP(hipMemcpyAsync(W[k], a->F[k], sizeof(double) * a->d.n[k] * r,
                                hipMemcpyDeviceToDevice, a->st));
  if (F != nullptr)
    for (int k = 0; k < 3; ++k)
      if (F[k] != nullptr)
        CPHIFI_HIP(hipMemcpyAsync(F[k], a->F[k], sizeof(double) * a->d.n[k] * a->d.r,
                                  hipMemcpyDeviceToDevice, a->st));
  CPHIFI_HIP(hipStreamSynchronize(a->st));
  return CPHIFI_OK;
}

int cphifi_als_destroy(cphifi_als* a) {
  clear_error();
  if (a == nullptr) return CPHIFI_OK;
  destroy_plans(a);
  delete a;
  return CPHIFI_OK;
}

}  // extern "C"
