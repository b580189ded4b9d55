// Skinny products Y = op(U) * diag(xscale) * X with U n x n and X n x r (r <= 64)
// on gfx950 MFMA.  These are the K X, K Yhat1, U_K^T R and U_K T products of the
// two-step matrix-free product (Section 4.4.1) and of the preconditioner
// apply (eq. fx); each streams the n x n operand from HBM exactly once.
//
// Design (per workgroup of 4 waves):
//  * a wave owns MW blocks of 16 output rows and all 16*NB output columns;
//  * the n x n operand goes straight from HBM to registers (it is used once,
//    so it never touches LDS).  The reduction index k is permuted per lane:
//    at MFMA step s lane (row li, k-group kk) consumes k = k0 + kk*S + s, so
//    each lane reads S consecutive elements of its row (NN form), or 16 lanes
//    read 16 consecutive elements of a row of U (transposed form);
//  * the n x r operand is staged through LDS in chunks of BK rows, double
//    buffered, shared by the 4 waves, and read with the same k permutation;
//  * split-K over blockIdx.y writes deterministic partial sums that the
//    consumer kernel adds in a fixed order (no atomics).
#include "cphifi_internal.h"

#include <type_traits>

namespace cphifi {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

struct GArgs {
  const void* U;
  int64_t ldu;
  int64_t n;
  const double* X;
  int64_t ldx;
  int r;
  const double* xscale;
  void* part;
  int64_t kper;
  int ldp;
  const int32_t* done;
  // BF16 only: the n x r operand pre-split into hi/lo bf16, transposed (c-major)
  const __bf16* xt_hi;
  const __bf16* xt_lo;
  int64_t ldxt;
};

// Output row held in accumulator element v of lane (kk = lane/16) inside a 16x16
// block: the FP64 16x16x4 MFMA interleaves its rows (row = kk + 4v), the FP32
// 16x16x4 and BF16 16x16x32 forms stack them (row = 4kk + v); column = lane%16.
template <typename TA>
__device__ __forceinline__ int out_row(int kk, int v) {
  return std::is_same<TA, double>::value ? kk + 4 * v : 4 * kk + v;
}

__device__ __forceinline__ d4 mfma4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ------------------------------------------------- FP64 / FP32 (16x16x4) kernel
template <typename TA, int NB, int MW, int S, bool TRANS>
__global__ __launch_bounds__(256) void gemm_k4_kernel(GArgs g) {
  using AccT = typename std::conditional<std::is_same<TA, double>::value, d4, f4>::type;
  if (g.done != nullptr && *g.done) return;
  constexpr int BK = 4 * S;
  constexpr int NC = NB * 16;
  constexpr int LDX = NC + 16 / S;  // pad spreads the 4 k-groups over distinct banks
  constexpr int XE = BK * NC;       // staged elements per chunk
  constexpr int XPT = (XE + 255) / 256;
  __shared__ TA xs[2][BK * LDX];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, kk = lane >> 4;
  const int64_t n = g.n;
  const int64_t mbase = (int64_t)blockIdx.x * (4 * MW * 16) + (int64_t)wave * (MW * 16);
  const int64_t kbeg = (int64_t)blockIdx.y * g.kper;
  const int64_t kend = min(n, kbeg + g.kper);
  const TA* __restrict__ U = (const TA*)g.U;
  const double* __restrict__ X = g.X;
  const int64_t ldu = g.ldu;

  int64_t rowc[MW];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb) rowc[mb] = min(mbase + mb * 16 + li, n - 1);

  AccT acc[MW][NB];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = AccT{0, 0, 0, 0};

  const int64_t span = kend - kbeg;
  const int64_t nchunk = span > 0 ? (span + BK - 1) / BK : 0;
  const bool tail = (span % BK) != 0;

  auto loadA = [&](TA (&dst)[MW][S], int64_t k0, bool check) {
#pragma unroll
    for (int mb = 0; mb < MW; ++mb)
#pragma unroll
      for (int s = 0; s < S; ++s) {
        int64_t k = k0 + kk * S + s;
        if (check) {
          const int64_t kc = min(k, n - 1);
          const TA v = TRANS ? U[kc * ldu + rowc[mb]] : U[rowc[mb] * ldu + kc];
          dst[mb][s] = (k < kend) ? v : TA(0);
        } else {
          dst[mb][s] = TRANS ? U[k * ldu + rowc[mb]] : U[rowc[mb] * ldu + k];
        }
      }
  };
  auto stageX = [&](TA (&xr)[XPT], int64_t k0) {
#pragma unroll
    for (int j = 0; j < XPT; ++j) {
      const int e = tid + j * 256;
      const int kidx = e / NC, c = e % NC;
      const int64_t k = k0 + kidx;
      double v = 0.0;
      if (e < XE && k < kend && c < g.r) {
        v = X[k * g.ldx + c];
        if (g.xscale != nullptr) v *= g.xscale[k];
      }
      xr[j] = (TA)v;
    }
  };
  auto storeX = [&](int buf, const TA (&xr)[XPT]) {
#pragma unroll
    for (int j = 0; j < XPT; ++j) {
      const int e = tid + j * 256;
      if (e < XE) xs[buf][(e / NC) * LDX + (e % NC)] = xr[j];
    }
  };
  auto compute = [&](const TA (&a)[MW][S], int buf) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      TA b[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) b[nb] = xs[buf][(kk * S + s) * LDX + nb * 16 + li];
#pragma unroll
      for (int mb = 0; mb < MW; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mfma4(a[mb][s], b[nb], acc[mb][nb]);
    }
  };

  if (nchunk > 0) {
    TA a0[MW][S], a1[MW][S];
    TA xr[XPT];
    loadA(a0, kbeg, tail && nchunk == 1);
    stageX(xr, kbeg);
    storeX(0, xr);
    __syncthreads();
    for (int64_t c = 0; c < nchunk; c += 2) {
      const bool has1 = c + 1 < nchunk;
      if (has1) {
        const int64_t k1 = kbeg + (c + 1) * BK;
        loadA(a1, k1, tail && (c + 1 == nchunk - 1));
        stageX(xr, k1);
      }
      compute(a0, 0);
      if (has1) storeX(1, xr);
      __syncthreads();
      if (!has1) break;
      const bool has2 = c + 2 < nchunk;
      if (has2) {
        const int64_t k2 = kbeg + (c + 2) * BK;
        loadA(a0, k2, tail && (c + 2 == nchunk - 1));
        stageX(xr, k2);
      }
      compute(a1, 1);
      if (has2) storeX(0, xr);
      __syncthreads();
    }
  }

  TA* part = (TA*)g.part + (int64_t)blockIdx.y * n * g.ldp;
#pragma unroll
  for (int mb = 0; mb < MW; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = mbase + mb * 16 + out_row<TA>(kk, v);
        if (row < n) part[row * g.ldp + nb * 16 + li] = acc[mb][nb][v];
      }
}

// ----------------------------------------------------- BF16 (16x16x32) kernel
// U is a zero-padded bf16 copy (row stride ldu >= round_up(n, BK)); the n x r
// operand arrives pre-split as hi + lo bf16 parts, transposed to c-major rows
// of stride ldxt, so the product carries ~16 significant bits of X while U
// stays at bf16.  Accumulation is FP32.
template <int NB, int MW, int S>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GArgs g) {
  if (g.done != nullptr && *g.done) return;
  constexpr int BK = 32 * S;
  constexpr int NC = NB * 16;
  constexpr int LDK = BK + 8;           // bf16 elements per LDS row (bank spread)
  constexpr int V8 = BK / 8;            // 16-byte vectors per staged row
  constexpr int XV = NC * V8;           // 16-byte vectors per chunk and part
  constexpr int XPT = (XV + 255) / 256;
  __shared__ __attribute__((aligned(16))) __bf16 xs[2][2][NC * LDK];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, kk = lane >> 4;
  const int64_t n = g.n;
  const int64_t mbase = (int64_t)blockIdx.x * (4 * MW * 16) + (int64_t)wave * (MW * 16);
  const int64_t kbeg = (int64_t)blockIdx.y * g.kper;
  const int64_t kend = min(n, kbeg + g.kper);
  const __bf16* __restrict__ U = (const __bf16*)g.U;

  int64_t rowc[MW];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb) rowc[mb] = min(mbase + mb * 16 + li, n - 1);

  f4 acc[MW][NB];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f4{0, 0, 0, 0};

  const int64_t span = kend - kbeg;
  const int64_t nchunk = span > 0 ? (span + BK - 1) / BK : 0;

  auto loadA = [&](u32x4 (&dst)[MW][S], int64_t k0) {
#pragma unroll
    for (int mb = 0; mb < MW; ++mb)
#pragma unroll
      for (int s = 0; s < S; ++s)
        dst[mb][s] = *(const u32x4*)(U + rowc[mb] * g.ldu + k0 + kk * (8 * S) + 8 * s);
  };
  // Staged vectors of the chunk: (part p, column c, vector v) -> 8 consecutive k.
  auto stageX = [&](u32x4 (&xr)[2][XPT], int64_t k0) {
#pragma unroll
    for (int j = 0; j < XPT; ++j) {
      const int e = tid + j * 256;
      if (e < XV) {
        const int c = e / V8, v = e % V8;
        const int64_t off = (int64_t)c * g.ldxt + k0 + 8 * v;
        xr[0][j] = *(const u32x4*)(g.xt_hi + off);
        xr[1][j] = *(const u32x4*)(g.xt_lo + off);
      }
    }
  };
  auto storeX = [&](int buf, const u32x4 (&xr)[2][XPT]) {
#pragma unroll
    for (int j = 0; j < XPT; ++j) {
      const int e = tid + j * 256;
      if (e < XV) {
        const int c = e / V8, v = e % V8;
        *(u32x4*)(&xs[buf][0][c * LDK + 8 * v]) = xr[0][j];
        *(u32x4*)(&xs[buf][1][c * LDK + 8 * v]) = xr[1][j];
      }
    }
  };
  auto compute = [&](const u32x4 (&a)[MW][S], int buf) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int off = (nb * 16 + li) * LDK + kk * (8 * S) + 8 * s;
        const bf16x8 bh = __builtin_bit_cast(bf16x8, *(const u32x4*)(&xs[buf][0][off]));
        const bf16x8 bl = __builtin_bit_cast(bf16x8, *(const u32x4*)(&xs[buf][1][off]));
#pragma unroll
        for (int mb = 0; mb < MW; ++mb) {
          const bf16x8 av = __builtin_bit_cast(bf16x8, a[mb][s]);
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bh, acc[mb][nb], 0, 0, 0);
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bl, acc[mb][nb], 0, 0, 0);
        }
      }
    }
  };

  if (nchunk > 0) {
    u32x4 a0[MW][S], a1[MW][S];
    u32x4 xr[2][XPT];
    loadA(a0, kbeg);
    stageX(xr, kbeg);
    storeX(0, xr);
    __syncthreads();
    for (int64_t c = 0; c < nchunk; c += 2) {
      const bool has1 = c + 1 < nchunk;
      if (has1) {
        loadA(a1, kbeg + (c + 1) * BK);
        stageX(xr, kbeg + (c + 1) * BK);
      }
      compute(a0, 0);
      if (has1) storeX(1, xr);
      __syncthreads();
      if (!has1) break;
      const bool has2 = c + 2 < nchunk;
      if (has2) {
        loadA(a0, kbeg + (c + 2) * BK);
        stageX(xr, kbeg + (c + 2) * BK);
      }
      compute(a1, 1);
      if (has2) storeX(0, xr);
      __syncthreads();
    }
  }

  float* part = (float*)g.part + (int64_t)blockIdx.y * n * g.ldp;
#pragma unroll
  for (int mb = 0; mb < MW; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = mbase + mb * 16 + out_row<float>(kk, v);
        if (row < n) part[row * g.ldp + nb * 16 + li] = acc[mb][nb][v];
      }
}

// X (n x r, row-major, optionally row-scaled) -> hi/lo bf16, c-major rows of
// stride ldxt covering k in [0, ldxt); zero outside k < n, c < r.
__global__ void split_bf16_kernel(const double* __restrict__ X, int64_t ldx, int r,
                                  const double* __restrict__ xscale, int64_t n, int nc,
                                  __bf16* __restrict__ hi, __bf16* __restrict__ lo,
                                  int64_t ldxt, const int32_t* done) {
  if (done != nullptr && *done) return;
  const int64_t total = (int64_t)nc * ldxt;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / ldxt, k = e % ldxt;
    float h = 0.f, l = 0.f;
    if (k < n && c < r) {
      double v = X[k * ldx + c];
      if (xscale != nullptr) v *= xscale[k];
      const __bf16 hb = (__bf16)(float)v;
      h = (float)hb;
      l = (float)(v - (double)h);
    }
    hi[e] = (__bf16)h;
    lo[e] = (__bf16)l;
  }
}

template <typename TA, int NB, int MW, int S, bool TRANS>
int launch_k4(const GArgs& g, int ksplit, hipStream_t st) {
  const int64_t rows = 4 * MW * 16;
  dim3 grid((unsigned)((g.n + rows - 1) / rows), (unsigned)ksplit);
  hipLaunchKernelGGL((gemm_k4_kernel<TA, NB, MW, S, TRANS>), grid, dim3(256), 0, st, g);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

template <typename TA, int MW, int S, bool TRANS>
int dispatch_nb_k4(int nb, const GArgs& g, int ksplit, hipStream_t st) {
  switch (nb) {
    case 1: return launch_k4<TA, 1, MW, S, TRANS>(g, ksplit, st);
    case 2: return launch_k4<TA, 2, MW, S, TRANS>(g, ksplit, st);
    case 3: return launch_k4<TA, 3, MW, S, TRANS>(g, ksplit, st);
    case 4: return launch_k4<TA, 4, MW, S, TRANS>(g, ksplit, st);
  }
  set_error("unsupported column block count %d", nb);
  return CPHIFI_INVALID_ARG;
}

template <typename TA, bool TRANS>
int dispatch_cfg_k4(int mw, int s, int nb, const GArgs& g, int ksplit, hipStream_t st) {
  if (mw == 1 && s == 4) return dispatch_nb_k4<TA, 1, 4, TRANS>(nb, g, ksplit, st);
  if (mw == 1 && s == 8) return dispatch_nb_k4<TA, 1, 8, TRANS>(nb, g, ksplit, st);
  if (mw == 2 && s == 4) return dispatch_nb_k4<TA, 2, 4, TRANS>(nb, g, ksplit, st);
  if (mw == 2 && s == 8) return dispatch_nb_k4<TA, 2, 8, TRANS>(nb, g, ksplit, st);
  if (mw == 4 && s == 4) return dispatch_nb_k4<TA, 4, 4, TRANS>(nb, g, ksplit, st);
  set_error("unsupported product tile (mw=%d, s=%d)", mw, s);
  return CPHIFI_INVALID_ARG;
}

template <int NB, int MW, int S>
int launch_bf16(const GArgs& g, int ksplit, hipStream_t st) {
  const int64_t rows = 4 * MW * 16;
  dim3 grid((unsigned)((g.n + rows - 1) / rows), (unsigned)ksplit);
  hipLaunchKernelGGL((gemm_bf16_kernel<NB, MW, S>), grid, dim3(256), 0, st, g);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

template <int MW, int S>
int dispatch_nb_bf16(int nb, const GArgs& g, int ksplit, hipStream_t st) {
  switch (nb) {
    case 1: return launch_bf16<1, MW, S>(g, ksplit, st);
    case 2: return launch_bf16<2, MW, S>(g, ksplit, st);
    case 3: return launch_bf16<3, MW, S>(g, ksplit, st);
    case 4: return launch_bf16<4, MW, S>(g, ksplit, st);
  }
  set_error("unsupported column block count %d", nb);
  return CPHIFI_INVALID_ARG;
}

int dispatch_cfg_bf16(int mw, int s, int nb, const GArgs& g, int ksplit, hipStream_t st) {
  if (mw == 1 && s == 4) return dispatch_nb_bf16<1, 4>(nb, g, ksplit, st);
  if (mw == 2 && s == 2) return dispatch_nb_bf16<2, 2>(nb, g, ksplit, st);
  if (mw == 2 && s == 4) return dispatch_nb_bf16<2, 4>(nb, g, ksplit, st);
  if (mw == 4 && s == 2) return dispatch_nb_bf16<4, 2>(nb, g, ksplit, st);
  set_error("unsupported bf16 product tile (mw=%d, s=%d)", mw, s);
  return CPHIFI_INVALID_ARG;
}

}  // namespace

int gemm_bk(Elt elt, int s) { return (elt == Elt::BF16 ? 32 : 4) * s; }

bool gemm_cfg_valid(Elt elt, int mw, int s) {
  if (elt == Elt::BF16)
    return (mw == 1 && s == 4) || (mw == 2 && s == 2) || (mw == 2 && s == 4) ||
           (mw == 4 && s == 2);
  return (mw == 1 && (s == 4 || s == 8)) || (mw == 2 && (s == 4 || s == 8)) ||
         (mw == 4 && s == 4);
}

GemmPlan make_gemm_plan(Elt elt, int64_t n, int mw, int s, int ksplit_req, int num_cu) {
  GemmPlan gp;
  gp.mw = mw;
  gp.s = s;
  const int64_t rows_per_wg = 4LL * mw * 16;
  const int64_t nrowblk = (n + rows_per_wg - 1) / rows_per_wg;
  const int64_t bk = gemm_bk(elt, s);
  int64_t ks = ksplit_req;
  if (ks <= 0) {
    // about three resident workgroups per CU, k ranges of at least 8 chunks
    const int64_t target = 3LL * (num_cu > 0 ? num_cu : 256);
    ks = (target + nrowblk - 1) / nrowblk;
    ks = std::min<int64_t>(ks, std::max<int64_t>(1, n / (8 * bk)));
  }
  ks = std::max<int64_t>(1, std::min<int64_t>(ks, kMaxSplit));
  int64_t kper = (n + ks - 1) / ks;
  kper = (kper + bk - 1) / bk * bk;
  gp.kper = kper;
  gp.ksplit = (int)((n + kper - 1) / kper);
  return gp;
}

GemmPlan choose_gemm(Elt elt, bool /*trans*/, int64_t n, int /*r*/, int num_cu) {
  if (elt == Elt::BF16) return make_gemm_plan(elt, n, 2, 4, 0, num_cu);
  return make_gemm_plan(elt, n, 2, 8, 0, num_cu);
}

static bool plan_ok(Elt elt, const GemmPlan& gp, int64_t n, int r) {
  return r >= 1 && r <= kMaxRank && n >= 1 && gp.ksplit >= 1 && gp.ksplit <= kMaxSplit &&
         gemm_cfg_valid(elt, gp.mw, gp.s) && gp.kper % gemm_bk(elt, gp.s) == 0 &&
         (int64_t)gp.ksplit * gp.kper >= n && (int64_t)(gp.ksplit - 1) * gp.kper < n;
}

int launch_gemm(Elt elt, bool trans, const GemmPlan& gp, const void* U, int64_t ldu,
                int64_t n, const double* X, int64_t ldx, int r, const double* xscale,
                void* part, const int32_t* done, hipStream_t st) {
  if (!plan_ok(elt, gp, n, r) || elt == Elt::BF16 || ldu < n || ldx < r) {
    set_error("launch_gemm: bad shape (n=%lld r=%d ksplit=%d kper=%lld mw=%d s=%d)",
              (long long)n, r, gp.ksplit, (long long)gp.kper, gp.mw, gp.s);
    return CPHIFI_INVALID_ARG;
  }
  const int nb = (r + 15) / 16;
  GArgs g{};
  g.U = U;
  g.ldu = ldu;
  g.n = n;
  g.X = X;
  g.ldx = ldx;
  g.r = r;
  g.xscale = xscale;
  g.part = part;
  g.kper = gp.kper;
  g.ldp = nb * 16;
  g.done = done;
  if (elt == Elt::F64)
    return trans ? dispatch_cfg_k4<double, true>(gp.mw, gp.s, nb, g, gp.ksplit, st)
                 : dispatch_cfg_k4<double, false>(gp.mw, gp.s, nb, g, gp.ksplit, st);
  return trans ? dispatch_cfg_k4<float, true>(gp.mw, gp.s, nb, g, gp.ksplit, st)
               : dispatch_cfg_k4<float, false>(gp.mw, gp.s, nb, g, gp.ksplit, st);
}

int launch_split_bf16(const double* X, int64_t ldx, int r, const double* xscale, int64_t n,
                      __bf16* xt_hi, __bf16* xt_lo, int64_t ldxt, const int32_t* done,
                      hipStream_t st) {
  const int nb = (r + 15) / 16;
  const int64_t total = (int64_t)nb * 16 * ldxt;
  const int blocks = (int)std::min<int64_t>(4096, (total + 255) / 256);
  hipLaunchKernelGGL(split_bf16_kernel, dim3(blocks), dim3(256), 0, st, X, ldx, r, xscale, n,
                     nb * 16, xt_hi, xt_lo, ldxt, done);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

// BF16 entry: X must already be split into xt_hi / xt_lo (launch_split_bf16).
int launch_gemm_bf16(const GemmPlan& gp, const __bf16* U, int64_t ldu, int64_t n,
                     const double* X, int64_t ldx, int r, const double* xscale, void* part,
                     __bf16* xt_hi, __bf16* xt_lo, int64_t ldxt, const int32_t* done,
                     hipStream_t st) {
  const int nb = (r + 15) / 16;
  const int64_t bk = gemm_bk(Elt::BF16, gp.s);
  const int64_t nround = (n + bk - 1) / bk * bk;
  if (!plan_ok(Elt::BF16, gp, n, r) || ldu % 8 != 0 || ldu < nround || ldxt < nround ||
      ldxt % 8 != 0 || ldx < r) {
    set_error("launch_gemm_bf16: bad shape (n=%lld r=%d ldu=%lld ldxt=%lld)", (long long)n, r,
              (long long)ldu, (long long)ldxt);
    return CPHIFI_INVALID_ARG;
  }
  GArgs g{};
  g.U = U;
  g.ldu = ldu;
  g.n = n;
  g.X = X;
  g.ldx = ldx;
  g.r = r;
  g.xscale = xscale;
  g.part = part;
  g.kper = gp.kper;
  g.ldp = nb * 16;
  g.done = done;
  g.xt_hi = xt_hi;
  g.xt_lo = xt_lo;
  g.ldxt = ldxt;
  return dispatch_cfg_bf16(gp.mw, gp.s, nb, g, gp.ksplit, st);
}

}  // namespace cphifi
