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

#include <cstdlib>
#include <mutex>
#include <string>
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
// VW: elements per vector load of the n x n operand along k (NN form only;
// requires ldu % VW == 0 and a 16-byte aligned U).
template <typename TA, int NB, int MW, int S, bool TRANS, int VW>
__global__ __launch_bounds__(256) void gemm_k4_kernel(GArgs g) {
  using AccT = typename std::conditional<std::is_same<TA, double>::value, d4, f4>::type;
  typedef TA VecT __attribute__((ext_vector_type(VW)));
  static_assert(S % VW == 0, "S must be a multiple of the vector width");
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
  const int64_t ldu = g.ldu;
  const int64_t mbase = (int64_t)blockIdx.x * (4 * MW * 16) + (int64_t)wave * (MW * 16);
  const int64_t kbeg = (int64_t)blockIdx.y * g.kper;
  const int64_t kend = min(n, kbeg + g.kper);
  const TA* __restrict__ U = (const TA*)g.U;

  // Lane-invariant parts of the addresses, computed once.
  const TA* abase[MW];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb) {
    const int64_t rc = min(mbase + mb * 16 + li, n - 1);
    abase[mb] = TRANS ? U + (int64_t)(kk * S) * ldu + rc : U + rc * ldu + kk * S;
  }
  const double* __restrict__ X = g.X;
  int xoff[XPT];   // offset of the staged element inside a chunk of X rows
  int xlds[XPT];   // its LDS slot
  int xkid[XPT];   // its row inside the chunk
  bool xon[XPT];   // inside the staged tile and a real column of X
#pragma unroll
  for (int j = 0; j < XPT; ++j) {
    const int e = tid + j * 256;
    const int kidx = e / NC, c = e % NC;
    xkid[j] = kidx;
    xoff[j] = kidx * (int)g.ldx + c;
    xlds[j] = kidx * LDX + c;
    xon[j] = e < XE && c < g.r;
  }

  AccT acc[MW][NB];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = AccT{0, 0, 0, 0};

  const int64_t span = kend - kbeg;
  const int64_t nfull = span > 0 ? span / BK : 0;
  const bool has_tail = span > 0 && (span % BK) != 0;
  const int64_t nchunk = nfull + (has_tail ? 1 : 0);

  auto loadA = [&](TA (&dst)[MW][S], int64_t k0) {
#pragma unroll
    for (int mb = 0; mb < MW; ++mb) {
      if (TRANS) {
        const TA* p = abase[mb] + k0 * ldu;
#pragma unroll
        for (int s = 0; s < S; ++s) dst[mb][s] = p[(int64_t)s * ldu];
      } else {
        const TA* p = abase[mb] + k0;
#pragma unroll
        for (int v = 0; v < S / VW; ++v) {
          const VecT t = *(const VecT*)(p + v * VW);
#pragma unroll
          for (int w = 0; w < VW; ++w) dst[mb][v * VW + w] = t[w];
        }
      }
    }
  };
  auto loadA_tail = [&](TA (&dst)[MW][S], int64_t k0) {
#pragma unroll
    for (int mb = 0; mb < MW; ++mb)
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int64_t k = k0 + kk * S + s;
        const int64_t dk = min(k, n - 1) - kk * S;  // relative to abase's k offset
        const TA v = TRANS ? abase[mb][dk * ldu] : abase[mb][dk];
        dst[mb][s] = (k < kend) ? v : TA(0);
      }
  };
  auto stageX = [&](TA (&xr)[XPT], int64_t k0, bool tail) {
    const double* xp = X + k0 * g.ldx;
#pragma unroll
    for (int j = 0; j < XPT; ++j) {
      double v = 0.0;
      const bool on = xon[j] && (!tail || k0 + xkid[j] < kend);
      if (on) {
        v = xp[xoff[j]];
        if (g.xscale != nullptr) v *= g.xscale[k0 + xkid[j]];
      }
      xr[j] = (TA)v;
    }
  };
  auto storeX = [&](int buf, const TA (&xr)[XPT]) {
#pragma unroll
    for (int j = 0; j < XPT; ++j)
      if (tid + j * 256 < XE) xs[buf][xlds[j]] = xr[j];
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
  // Next chunk: X rows first, then the n x n operand.  vmcnt retires in
  // order, so waiting for the X rows (to fill LDS) leaves the larger A
  // prefetch in flight across the barrier and into the next compute.
  auto fetch = [&](TA (&xr)[XPT], TA (&dst)[MW][S], int64_t c) {
    const int64_t k0 = kbeg + c * BK;
    const bool tail = c == nfull;
    stageX(xr, k0, tail);
    if (tail)
      loadA_tail(dst, k0);
    else
      loadA(dst, k0);
  };

  if (nchunk > 0) {
    TA acur[MW][S], anext[MW][S];
    TA xr[XPT];
    fetch(xr, acur, 0);
    storeX(0, xr);
    __syncthreads();
    for (int64_t c = 0; c < nchunk; ++c) {
      const int buf = (int)(c & 1);
      const bool more = c + 1 < nchunk;
      if (more) fetch(xr, anext, c + 1);
      compute(acur, buf);
      if (more) storeX(buf ^ 1, xr);
      __syncthreads();
#pragma unroll
      for (int mb = 0; mb < MW; ++mb)
#pragma unroll
        for (int q = 0; q < S; ++q) acur[mb][q] = anext[mb][q];
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
    // X rows of the next chunk are fetched before its U rows: vmcnt retires in
    // order, so filling LDS does not wait for the larger U prefetch.
    u32x4 acur[MW][S], anext[MW][S];
    u32x4 xr[2][XPT];
    stageX(xr, kbeg);
    loadA(acur, kbeg);
    storeX(0, xr);
    __syncthreads();
    for (int64_t c = 0; c < nchunk; ++c) {
      const int buf = (int)(c & 1);
      const bool more = c + 1 < nchunk;
      if (more) {
        stageX(xr, kbeg + (c + 1) * BK);
        loadA(anext, kbeg + (c + 1) * BK);
      }
      compute(acur, buf);
      if (more) storeX(buf ^ 1, xr);
      __syncthreads();
#pragma unroll
      for (int mb = 0; mb < MW; ++mb)
#pragma unroll
        for (int q = 0; q < S; ++q) acur[mb][q] = anext[mb][q];
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
  constexpr int VW = TRANS ? 1 : (std::is_same<TA, double>::value ? 2 : 4);
  const bool vec_ok = !TRANS && g.ldu % VW == 0 &&
                      (reinterpret_cast<uintptr_t>(g.U) % 16) == 0;
  if (vec_ok)
    hipLaunchKernelGGL((gemm_k4_kernel<TA, NB, MW, S, TRANS, VW>), grid, dim3(256), 0, st, g);
  else
    hipLaunchKernelGGL((gemm_k4_kernel<TA, NB, MW, S, TRANS, 1>), grid, dim3(256), 0, st, g);
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

template <typename TA, int MW, int S, bool TRANS>
int occ_k4(int nb) {
  constexpr int VW = TRANS ? 1 : (std::is_same<TA, double>::value ? 2 : 4);
  int blocks = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (nb) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_k4_kernel<TA, 1, MW, S, TRANS, VW>, 256, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_k4_kernel<TA, 2, MW, S, TRANS, VW>, 256, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_k4_kernel<TA, 3, MW, S, TRANS, VW>, 256, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_k4_kernel<TA, 4, MW, S, TRANS, VW>, 256, 0); break;
  }
  return e == hipSuccess && blocks > 0 ? blocks : 1;
}

template <int MW, int S>
int occ_bf16(int nb) {
  int blocks = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (nb) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_bf16_kernel<1, MW, S>, 256, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_bf16_kernel<2, MW, S>, 256, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_bf16_kernel<3, MW, S>, 256, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_bf16_kernel<4, MW, S>, 256, 0); break;
  }
  return e == hipSuccess && blocks > 0 ? blocks : 1;
}

template <typename TA, bool TRANS>
int occ_cfg_k4(int mw, int s, int nb) {
  if (mw == 1 && s == 4) return occ_k4<TA, 1, 4, TRANS>(nb);
  if (mw == 1 && s == 8) return occ_k4<TA, 1, 8, TRANS>(nb);
  if (mw == 2 && s == 4) return occ_k4<TA, 2, 4, TRANS>(nb);
  if (mw == 2 && s == 8) return occ_k4<TA, 2, 8, TRANS>(nb);
  if (mw == 4 && s == 4) return occ_k4<TA, 4, 4, TRANS>(nb);
  return 1;
}

int occ_cfg_bf16(int mw, int s, int nb) {
  if (mw == 1 && s == 4) return occ_bf16<1, 4>(nb);
  if (mw == 2 && s == 2) return occ_bf16<2, 2>(nb);
  if (mw == 2 && s == 4) return occ_bf16<2, 4>(nb);
  if (mw == 4 && s == 2) return occ_bf16<4, 2>(nb);
  return 1;
}

}  // namespace

int gemm_occupancy(Elt elt, bool trans, int mw, int s, int r) {
  const int nb = (r + 15) / 16;
  switch (elt) {
    case Elt::F64: return trans ? occ_cfg_k4<double, true>(mw, s, nb) : occ_cfg_k4<double, false>(mw, s, nb);
    case Elt::F32: return trans ? occ_cfg_k4<float, true>(mw, s, nb) : occ_cfg_k4<float, false>(mw, s, nb);
    case Elt::BF16: return occ_cfg_bf16(mw, s, nb);
  }
  return 1;
}

int gemm_bk(Elt elt, int s) { return (elt == Elt::BF16 ? 32 : 4) * s; }

bool gemm_cfg_valid(Elt elt, int mw, int s) {
  if (elt == Elt::BF16)
    return (mw == 1 && s == 4) || (mw == 2 && s == 2) || (mw == 2 && s == 4) ||
           (mw == 4 && s == 2);
  return (mw == 1 && (s == 4 || s == 8)) || (mw == 2 && (s == 4 || s == 8)) ||
         (mw == 4 && s == 4);
}

GemmPlan make_gemm_plan(Elt elt, bool trans, int64_t n, int r, int mw, int s, int ksplit_req,
                        int num_cu) {
  GemmPlan gp;
  gp.mw = mw;
  gp.s = s;
  const int64_t rows_per_wg = 4LL * mw * 16;
  const int64_t nrowblk = (n + rows_per_wg - 1) / rows_per_wg;
  const int64_t bk = gemm_bk(elt, s);
  int64_t ks = ksplit_req;
  if (ks <= 0) {
    // One round of resident workgroups: split K until the grid fills the
    // co-resident slots (CUs x workgroups per CU) without spilling into a
    // second, partial round; keep at least 4 chunks per split.
    const int64_t slots =
        (int64_t)(num_cu > 0 ? num_cu : 256) * gemm_occupancy(elt, trans, mw, s, r);
    ks = std::max<int64_t>(1, slots / nrowblk);
    ks = std::min<int64_t>(ks, std::max<int64_t>(1, n / (4 * bk)));
  }
  ks = std::max<int64_t>(1, std::min<int64_t>(ks, kMaxSplit));
  int64_t kper = (n + ks - 1) / ks;
  kper = (kper + bk - 1) / bk * bk;
  gp.kper = kper;
  gp.ksplit = (int)((n + kper - 1) / kper);
  return gp;
}

namespace {

struct TileRule {
  int elt, trans, r_lo, r_hi;
  int64_t n_lo, n_hi;
  int mw, s, ksplit;
};

// Tile table written by the autotuner (paper_2603_25691_amd/tune.py), read
// once per process from the file named by CPHIFI_TILE_TABLE.
const std::vector<TileRule>& tile_table() {
  static std::once_flag once;
  static std::vector<TileRule> rules;
  std::call_once(once, [] {
    const char* path = std::getenv("CPHIFI_TILE_TABLE");
    if (path == nullptr) return;
    FILE* f = std::fopen(path, "r");
    if (f == nullptr) return;
    char line[256];
    while (std::fgets(line, sizeof(line), f)) {
      if (line[0] == '#') continue;
      char tag[16];
      TileRule t{};
      long long nlo = 0, nhi = 0;
      if (std::sscanf(line, "%15s %d %d %d %lld %lld %d %d %d", tag, &t.trans, &t.r_lo, &t.r_hi,
                      &nlo, &nhi, &t.mw, &t.s, &t.ksplit) != 9)
        continue;
      const std::string e(tag);
      t.elt = e == "f64" ? 0 : e == "f32" ? 1 : e == "bf16" ? 2 : -1;
      t.n_lo = nlo;
      t.n_hi = nhi;
      if (t.elt >= 0 && gemm_cfg_valid((Elt)t.elt, t.mw, t.s)) rules.push_back(t);
    }
    std::fclose(f);
  });
  return rules;
}

bool table_tile(Elt elt, bool trans, int64_t n, int r, int* mw, int* s, int* ks) {
  for (const TileRule& t : tile_table())
    if (t.elt == (int)elt && t.trans == (int)trans && r >= t.r_lo && r <= t.r_hi &&
        n >= t.n_lo && n <= t.n_hi) {
      *mw = t.mw;
      *s = t.s;
      *ks = t.ksplit;
      return true;
    }
  return false;
}

}  // namespace

// Tile for a product: the autotuner's table when one is loaded and covers
// (n, r), else defaults measured at n = 30658, r = 40 on MI355X.
GemmPlan choose_gemm(Elt elt, bool trans, int64_t n, int r, int num_cu) {
  int mw = 0, s = 0, ks = 0;
  if (table_tile(elt, trans && elt != Elt::BF16, n, r, &mw, &s, &ks))
    return make_gemm_plan(elt, trans && elt != Elt::BF16, n, r, mw, s, ks, num_cu);
  switch (elt) {
    case Elt::BF16: return make_gemm_plan(elt, false, n, r, 4, 2, 0, num_cu);
    case Elt::F32: return trans ? make_gemm_plan(elt, true, n, r, 4, 4, 0, num_cu)
                                : make_gemm_plan(elt, false, n, r, 2, 4, 0, num_cu);
    case Elt::F64: return trans ? make_gemm_plan(elt, true, n, r, 4, 4, 0, num_cu)
                                : make_gemm_plan(elt, false, n, r, 2, 8, 0, num_cu);
  }
  return make_gemm_plan(elt, trans, n, r, 2, 8, 0, num_cu);
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
