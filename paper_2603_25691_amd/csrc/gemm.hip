// Grid launches of the skinny products Y = op(U) * diag(xscale) * X (the tiles
// themselves, and their design, are in gemm_tiles.h): one workgroup per
// (row block, k-range), the tile table of the autotuner, occupancy-based
// split-K, and the hi/lo BF16 split of the n x r operand.
#include "cphifi_internal.h"
#include "gemm_tiles.h"

#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>

namespace cphifi {
namespace {

using tiles::GArgs;

// Two workgroups per CU (occupancy target of the register allocator).
template <typename TA, int NB, int MW, int S, bool TRANS, int VW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_k4_kernel(
    GArgs g) {
  if (g.done != nullptr && *g.done) return;
  __shared__ TA xs[tiles::k4_lds_elems<TA, NB, S>()];
  tiles::gemm_k4_tile<TA, NB, MW, S, TRANS, VW>(g, blockIdx.x, blockIdx.y, xs, threadIdx.x);
}

// FP64 products: 4x4x4 MFMA tile over NC4 groups of 4 columns.  The empty asm
// that clobbers a0 marks the kernel as using AGPRs, so the register allocator
// may keep the MFMA accumulators there and leave the VGPRs to the two sets of
// prefetched operands.
template <int NC4, int MW, int S, bool TRANS, int VW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_f64_kernel(
    GArgs g) {
  if (g.done != nullptr && *g.done) return;
  asm volatile("" ::: "a0");
  __shared__ double xs[tiles::k4x4_lds_elems<NC4, S>()];
  const int64_t kbeg = (int64_t)blockIdx.y * g.kper;
  tiles::gemm_f64x4_tile<NC4, MW, S, TRANS, VW, true>(g, blockIdx.x, kbeg, min(g.n, kbeg + g.kper),
                                                      blockIdx.y, xs, threadIdx.x);
}

// Stream-K form of the transposed FP64 product: the (row block, k chunk)
// iterations are dealt out evenly to exactly one round of resident
// workgroups, so no slot idles at the end (the split-K grid of 120 row blocks
// x 4 splits at n = 30658 fills 480 of 512 slots).  A workgroup runs the
// tile once per row block its range touches and writes that part into slab
// (its rank among the row block's contributors); the last contributor of a
// row block zeroes the slabs past their count, so every row has sk.ksplit
// slabs like a split-K product.
struct SkArgs {
  int64_t nrb, nch;  // row blocks, k chunks per row block
  int64_t wgs;       // workgroups (grid size)
  int ksplit;        // slabs every row ends up with
};

__device__ __forceinline__ int64_t sk_first(int64_t x, int64_t wgs, int64_t T) {
  // the workgroup whose range [w T / wgs, (w + 1) T / wgs) holds iteration x
  return ((x + 1) * wgs - 1) / T;
}

template <int NC4, int MW, int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_f64_sk_kernel(
    GArgs g, SkArgs sk) {
  if (g.done != nullptr && *g.done) return;
  asm volatile("" ::: "a0");
  __shared__ double xs[tiles::k4x4_lds_elems<NC4, S>()];
  constexpr int BK = 4 * S;
  constexpr int64_t ROWS = 4 * MW * 16;
  const int64_t T = sk.nrb * sk.nch;
  const int64_t w = blockIdx.x;
  const int64_t c1 = (w + 1) * T / sk.wgs;
  for (int64_t c = w * T / sk.wgs; c < c1;) {
    const int64_t b = c / sk.nch;
    const int64_t cend = min(c1, (b + 1) * sk.nch);
    const int64_t wf = sk_first(b * sk.nch, sk.wgs, T);
    const int64_t wl = sk_first((b + 1) * sk.nch - 1, sk.wgs, T);
    // the zeroing goes first: it keeps the loop state out of the tile's live range
    if (w == wl) {  // last contributor: zero the unused slabs of this row block
      const int64_t r0 = b * ROWS, r1 = min(g.n, r0 + ROWS);
      double* part = (double*)g.part;
      for (int64_t sl = wl - wf + 1; sl < sk.ksplit; ++sl)
        for (int64_t e = threadIdx.x; e < (r1 - r0) * g.ldp; e += 256)
          part[(sl * g.n + r0) * g.ldp + e] = 0.0;
    }
    tiles::gemm_f64x4_tile<NC4, MW, S, true, 1, true>(
        g, b, (c - b * sk.nch) * BK, min(g.n, (cend - b * sk.nch) * BK), w - wf, xs,
        threadIdx.x);
    c = cend;
  }
}

// U chunks in flight of the BF16 tile: three for the tiled layout (compiled
// for one wave per SIMD, so the buffers fit every tile shape), else two.  At
// n = 30658, r = 40 (4x2 tile) the third buffer took the product from 0.327
// to 0.320 ms.
constexpr int bf16_depth(bool tiled) { return tiled ? 3 : 2; }

template <int NB, int MW, int S, bool TILED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TILED ? 1 : 2, TILED ? 1 : 2))) void gemm_bf16_kernel(
    GArgs g) {
  if (g.done != nullptr && *g.done) return;
  __shared__ __attribute__((aligned(16))) __bf16 xs[tiles::bf16_lds_elems<NB, S>()];
  const int64_t kb = (int64_t)blockIdx.y * g.kper;
  tiles::gemm_bf16_tile<NB, MW, S, TILED, bf16_depth(TILED)>(
      g, blockIdx.x, kb, min(g.n, kb + g.kper), blockIdx.y, xs, threadIdx.x);
}

// Stream-K form of the tiled BF16 product: the (row block, k chunk) iterations
// dealt evenly to exactly one workgroup per CU (the split-K grid of 120 x 2 at
// n = 30658 leaves 16 CUs idle); a workgroup writes one partial slab per row
// block it touches, and the last contributor of a row block zeroes the slabs
// no one writes, so every row sums `ksplit` slabs as in the split-K form.
template <int NB, int MW, int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void gemm_bf16_sk_kernel(
    GArgs g, SkArgs sk) {
  if (g.done != nullptr && *g.done) return;
  __shared__ __attribute__((aligned(16))) __bf16 xs[tiles::bf16_lds_elems<NB, S>()];
  constexpr int BK = 32 * S;
  constexpr int64_t ROWS = 4 * MW * 16;
  const int64_t T = sk.nrb * sk.nch;
  const int64_t w = blockIdx.x;
  const int64_t c1 = (w + 1) * T / sk.wgs;
  for (int64_t c = w * T / sk.wgs; c < c1;) {
    const int64_t b = c / sk.nch;
    const int64_t cend = min(c1, (b + 1) * sk.nch);
    const int64_t wf = sk_first(b * sk.nch, sk.wgs, T);
    const int64_t wl = sk_first((b + 1) * sk.nch - 1, sk.wgs, T);
    if (w == wl) {  // last contributor: zero the unused slabs of this row block
      const int64_t r0 = b * ROWS, r1 = min(g.n, r0 + ROWS);
      float* part = (float*)g.part;
      for (int64_t sl = wl - wf + 1; sl < sk.ksplit; ++sl)
        for (int64_t e = threadIdx.x; e < (r1 - r0) * g.ldp; e += 256)
          part[(sl * g.n + r0) * g.ldp + e] = 0.0f;
    }
    tiles::gemm_bf16_tile<NB, MW, S, true, bf16_depth(true)>(
        g, b, (c - b * sk.nch) * BK, min(g.n, (cend - b * sk.nch) * BK), w - wf, xs,
        threadIdx.x);
    __syncthreads();  // the next row block's first chunk reuses the LDS
    c = cend;
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
    double v = 0.0;
    if (k < n && c < r) {
      v = X[k * ldx + c];
      if (xscale != nullptr) v *= xscale[k];
    }
    split_pair(v, &hi[e], &lo[e]);
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

// Column groups of 4 for r: rounded up to an even count (8 columns), which
// bounds the instantiations and stays within the partials' 16 ceil(r/16).
inline int f64_groups(int r) { return 2 * ((r + 7) / 8); }

template <int NC4, int MW, int S, bool TRANS>
int launch_f64(const GArgs& g, int ksplit, hipStream_t st) {
  const int64_t rows = 4 * MW * 16;
  dim3 grid((unsigned)((g.n + rows - 1) / rows), (unsigned)ksplit);
  constexpr int VW = TRANS ? 1 : 2;
  const bool vec_ok =
      !TRANS && g.ldu % 2 == 0 && (reinterpret_cast<uintptr_t>(g.U) % 16) == 0;
  if (vec_ok)
    hipLaunchKernelGGL((gemm_f64_kernel<NC4, MW, S, TRANS, VW>), grid, dim3(256), 0, st, g);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<NC4, MW, S, TRANS, 1>), grid, dim3(256), 0, st, g);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

template <int MW, int S, bool TRANS>
int dispatch_nc4_f64(int nc4, const GArgs& g, int ksplit, hipStream_t st) {
  switch (nc4) {
    case 2: return launch_f64<2, MW, S, TRANS>(g, ksplit, st);
    case 4: return launch_f64<4, MW, S, TRANS>(g, ksplit, st);
    case 6: return launch_f64<6, MW, S, TRANS>(g, ksplit, st);
    case 8: return launch_f64<8, MW, S, TRANS>(g, ksplit, st);
    case 10: return launch_f64<10, MW, S, TRANS>(g, ksplit, st);
    case 12: return launch_f64<12, MW, S, TRANS>(g, ksplit, st);
    case 14: return launch_f64<14, MW, S, TRANS>(g, ksplit, st);
    case 16: return launch_f64<16, MW, S, TRANS>(g, ksplit, st);
  }
  set_error("unsupported column group count %d", nc4);
  return CPHIFI_INVALID_ARG;
}

template <int NC4, int MW, int S>
int launch_f64_sk(const GemmPlan& gp, const GArgs& g, hipStream_t st) {
  SkArgs sk;
  sk.nrb = (g.n + 4 * MW * 16 - 1) / (4 * MW * 16);
  sk.nch = (g.n + 4 * S - 1) / (4 * S);
  sk.wgs = gp.sk;
  sk.ksplit = gp.ksplit;
  hipLaunchKernelGGL((gemm_f64_sk_kernel<NC4, MW, S>), dim3((unsigned)gp.sk), dim3(256), 0, st,
                     g, sk);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

template <int MW, int S>
int dispatch_nc4_f64_sk(int nc4, const GemmPlan& gp, const GArgs& g, hipStream_t st) {
  switch (nc4) {
    case 2: return launch_f64_sk<2, MW, S>(gp, g, st);
    case 4: return launch_f64_sk<4, MW, S>(gp, g, st);
    case 6: return launch_f64_sk<6, MW, S>(gp, g, st);
    case 8: return launch_f64_sk<8, MW, S>(gp, g, st);
    case 10: return launch_f64_sk<10, MW, S>(gp, g, st);
    case 12: return launch_f64_sk<12, MW, S>(gp, g, st);
    case 14: return launch_f64_sk<14, MW, S>(gp, g, st);
    case 16: return launch_f64_sk<16, MW, S>(gp, g, st);
  }
  set_error("unsupported column group count %d", nc4);
  return CPHIFI_INVALID_ARG;
}

int dispatch_f64_sk(const GemmPlan& gp, int nc4, const GArgs& g, hipStream_t st) {
  if (gp.mw == 4 && gp.s == 2) return dispatch_nc4_f64_sk<4, 2>(nc4, gp, g, st);
  if (gp.mw == 2 && gp.s == 4) return dispatch_nc4_f64_sk<2, 4>(nc4, gp, g, st);
  if (gp.mw == 1 && gp.s == 8) return dispatch_nc4_f64_sk<1, 8>(nc4, gp, g, st);
  set_error("unsupported stream-K FP64 tile (mw=%d, s=%d)", gp.mw, gp.s);
  return CPHIFI_INVALID_ARG;
}

template <bool TRANS>
int dispatch_cfg_f64(int mw, int s, int nc4, const GArgs& g, int ksplit, hipStream_t st) {
  if (mw == 1 && s == 4) return dispatch_nc4_f64<1, 4, TRANS>(nc4, g, ksplit, st);
  if (mw == 1 && s == 8) return dispatch_nc4_f64<1, 8, TRANS>(nc4, g, ksplit, st);
  if (mw == 2 && s == 4) return dispatch_nc4_f64<2, 4, TRANS>(nc4, g, ksplit, st);
  if (mw == 2 && s == 8) return dispatch_nc4_f64<2, 8, TRANS>(nc4, g, ksplit, st);
  if (mw == 4 && s == 2) return dispatch_nc4_f64<4, 2, TRANS>(nc4, g, ksplit, st);
  // (4, 4): the 16x16x4 MFMA tile (columns in blocks of 16)
  if (mw == 4 && s == 4) return dispatch_nb_k4<double, 4, 4, TRANS>((g.r + 15) / 16, g, ksplit, st);
  set_error("unsupported FP64 product tile (mw=%d, s=%d)", mw, s);
  return CPHIFI_INVALID_ARG;
}

template <int NB, int MW, int S, bool TILED>
int launch_bf16(const GArgs& g, int ksplit, hipStream_t st) {
  const int64_t rows = 4 * MW * 16;
  dim3 grid((unsigned)((g.n + rows - 1) / rows), (unsigned)ksplit);
  hipLaunchKernelGGL((gemm_bf16_kernel<NB, MW, S, TILED>), grid, dim3(256), 0, st, g);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

template <int MW, int S, bool TILED>
int dispatch_nb_bf16(int nb, const GArgs& g, int ksplit, hipStream_t st) {
  switch (nb) {
    case 1: return launch_bf16<1, MW, S, TILED>(g, ksplit, st);
    case 2: return launch_bf16<2, MW, S, TILED>(g, ksplit, st);
    case 3: return launch_bf16<3, MW, S, TILED>(g, ksplit, st);
    case 4: return launch_bf16<4, MW, S, TILED>(g, ksplit, st);
  }
  set_error("unsupported column block count %d", nb);
  return CPHIFI_INVALID_ARG;
}

template <bool TILED>
int dispatch_cfg_bf16(int mw, int s, int nb, const GArgs& g, int ksplit, hipStream_t st) {
  if (mw == 1 && s == 4) return dispatch_nb_bf16<1, 4, TILED>(nb, g, ksplit, st);
  if (mw == 2 && s == 2) return dispatch_nb_bf16<2, 2, TILED>(nb, g, ksplit, st);
  if (mw == 2 && s == 4) return dispatch_nb_bf16<2, 4, TILED>(nb, g, ksplit, st);
  if (mw == 4 && s == 2) return dispatch_nb_bf16<4, 2, TILED>(nb, g, ksplit, st);
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

template <int MW, int S, bool TRANS>
int occ_f64(int nc4) {
  constexpr int VW = TRANS ? 1 : 2;
  int blocks = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (nc4) {
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_f64_kernel<2, MW, S, TRANS, VW>, 256, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_f64_kernel<4, MW, S, TRANS, VW>, 256, 0); break;
    case 6: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_f64_kernel<6, MW, S, TRANS, VW>, 256, 0); break;
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_f64_kernel<8, MW, S, TRANS, VW>, 256, 0); break;
    case 10: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_f64_kernel<10, MW, S, TRANS, VW>, 256, 0); break;
    case 12: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_f64_kernel<12, MW, S, TRANS, VW>, 256, 0); break;
    case 14: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_f64_kernel<14, MW, S, TRANS, VW>, 256, 0); break;
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_f64_kernel<16, MW, S, TRANS, VW>, 256, 0); break;
  }
  return e == hipSuccess && blocks > 0 ? blocks : 1;
}

template <bool TRANS>
int occ_cfg_f64(int mw, int s, int nc4) {
  if (mw == 1 && s == 4) return occ_f64<1, 4, TRANS>(nc4);
  if (mw == 1 && s == 8) return occ_f64<1, 8, TRANS>(nc4);
  if (mw == 2 && s == 4) return occ_f64<2, 4, TRANS>(nc4);
  if (mw == 2 && s == 8) return occ_f64<2, 8, TRANS>(nc4);
  if (mw == 4 && s == 2) return occ_f64<4, 2, TRANS>(nc4);
  if (mw == 4 && s == 4) return occ_k4<double, 4, 4, TRANS>((2 * nc4 + 7) / 8);
  return 1;
}

template <int MW, int S>
int occ_bf16(int nb) {
  int blocks = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (nb) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_bf16_kernel<1, MW, S, true>, 256, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_bf16_kernel<2, MW, S, true>, 256, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_bf16_kernel<3, MW, S, true>, 256, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gemm_bf16_kernel<4, MW, S, true>, 256, 0); break;
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
    case Elt::F64:
      return trans ? occ_cfg_f64<true>(mw, s, f64_groups(r)) : occ_cfg_f64<false>(mw, s, f64_groups(r));
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
  if (elt == Elt::F64)
    return (mw == 1 && (s == 4 || s == 8)) || (mw == 2 && (s == 4 || s == 8)) ||
           (mw == 4 && (s == 2 || s == 4));
  return (mw == 1 && (s == 4 || s == 8)) || (mw == 2 && (s == 4 || s == 8)) ||
         (mw == 4 && s == 4);
}

// Stream-K for the transposed FP64 product unless CPHIFI_F64_STREAMK says otherwise.
constexpr bool kF64StreamKDefault = false;
constexpr bool kBf16StreamKDefault = false;

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
    // second, partial round; keep at least 4 chunks per split.  The BF16
    // product fills one workgroup per CU: fewer concurrent row streams read
    // HBM faster (n = 30658, r = 40, 4x2 tile: split 2, 240 workgroups,
    // 0.351 ms; split 4, 480 workgroups, 0.368 ms).
    const int occ = elt == Elt::BF16 ? 1 : gemm_occupancy(elt, trans, mw, s, r);
    const int64_t slots = (int64_t)(num_cu > 0 ? num_cu : 256) * occ;
    ks = std::max<int64_t>(1, slots / nrowblk);
    ks = std::min<int64_t>(ks, std::max<int64_t>(1, n / (4 * bk)));
  }
  ks = std::max<int64_t>(1, std::min<int64_t>(ks, kMaxSplit));
  int64_t kper = (n + ks - 1) / ks;
  kper = (kper + bk - 1) / bk * bk;
  gp.kper = kper;
  gp.ksplit = (int)((n + kper - 1) / kper);
  // Stream-K for the transposed FP64 4x4x4 tile when the split-K grid leaves
  // resident slots idle (CPHIFI_F64_STREAMK=0 / 1 forces it off / on).
  const bool x4 = elt == Elt::F64 && trans && ((mw == 4 && s == 2) || (mw == 2 && s == 4) ||
                                              (mw == 1 && s == 8));
  if (x4 && ksplit_req <= 0) {
    const char* env = std::getenv("CPHIFI_F64_STREAMK");
    const int occ = gemm_occupancy(elt, trans, mw, s, r);
    const int64_t slots = (int64_t)(num_cu > 0 ? num_cu : 256) * occ;
    const int64_t grid = nrowblk * gp.ksplit;
    const bool want = env != nullptr ? std::atoi(env) != 0 : kF64StreamKDefault;
    const int64_t nch = (n + bk - 1) / bk;
    const int64_t T = nrowblk * nch;
    if (want && grid < slots && T >= slots) {
      const int64_t W = slots;
      int ksp = 1;
      for (int64_t b = 0; b < nrowblk; ++b) {
        const int64_t wf = ((b * nch + 1) * W - 1) / T;
        const int64_t wl = (((b + 1) * nch) * W - 1) / T;
        ksp = std::max<int>(ksp, (int)(wl - wf + 1));
      }
      if (ksp <= kMaxSplit) {
        gp.sk = (int)W;
        gp.ksplit = ksp;
        gp.kper = nch * bk;
      }
    }
  }
  return gp;
}

namespace {

struct TileRule {
  int elt, trans, r_lo, r_hi;
  int64_t n_lo, n_hi;
  int mw, s, ksplit;
};

// Tile tables written by the autotuner (paper_2603_25691_amd/tune.py): each
// file is parsed once per process; the default table is the file named by
// CPHIFI_TILE_TABLE.
std::vector<TileRule> read_table(const char* path) {
  std::vector<TileRule> rules;
  FILE* f = path != nullptr ? std::fopen(path, "r") : nullptr;
  if (f == nullptr) return rules;
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
  return rules;
}

const std::vector<TileRule>& tile_table(const char* path) {
  static std::mutex mu;
  static std::map<std::string, std::vector<TileRule>> cache;
  const char* p = path != nullptr ? path : std::getenv("CPHIFI_TILE_TABLE");
  const std::string key = p != nullptr ? p : "";
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it == cache.end()) it = cache.emplace(key, read_table(p)).first;
  return it->second;
}

bool table_tile(Elt elt, bool trans, int64_t n, int r, int* mw, int* s, int* ks) {
  return gemm_table_lookup(nullptr, elt, trans, n, r, mw, s, ks);
}

}  // namespace

bool gemm_table_lookup(const char* path, Elt elt, bool trans, int64_t n, int r, int* mw, int* s,
                       int* ks) {
  for (const TileRule& t : tile_table(path))
    if (t.elt == (int)elt && t.trans == (int)trans && r >= t.r_lo && r <= t.r_hi &&
        n >= t.n_lo && n <= t.n_hi) {
      *mw = t.mw;
      *s = t.s;
      *ks = t.ksplit;
      return true;
    }
  return false;
}

// Tile for a product: the autotuner's table when one is loaded and covers
// (n, r), else defaults measured at n = 30658, r = 40 on MI355X.
// Stream-K form of a tiled BF16 product plan (one workgroup per CU: the
// split-K grid of these plans leaves CUs idle, e.g. 240 of 256 at n = 30658);
// CPHIFI_BF16_STREAMK=1 turns it on.  Off by default: at n = 30658, r = 40 it
// ran 0.346-0.358 ms against 0.330-0.350 ms for the 240-workgroup split-K
// grid (this HBM-bound product reads faster from fewer concurrent row
// streams).  Only the 4 x 2 tile, only without an explicit split.
GemmPlan bf16_stream_k(const GemmPlan& gp, int64_t n, int num_cu) {
  const char* env = std::getenv("CPHIFI_BF16_STREAMK");
  const bool want = env != nullptr ? std::atoi(env) != 0 : kBf16StreamKDefault;
  if (!want || gp.sk > 0 || gp.mw != 4 || gp.s != 2) return gp;
  const int64_t rows = 4LL * gp.mw * 16;
  const int64_t nrowblk = (n + rows - 1) / rows;
  const int64_t bk = gemm_bk(Elt::BF16, gp.s);
  const int64_t nch = (n + bk - 1) / bk;
  const int64_t T = nrowblk * nch;
  const int64_t W = num_cu > 0 ? num_cu : 256;
  if (nrowblk * gp.ksplit >= W || T < W) return gp;
  int ksp = 1;
  for (int64_t b = 0; b < nrowblk; ++b) {
    const int64_t wf = ((b * nch + 1) * W - 1) / T;
    const int64_t wl = (((b + 1) * nch) * W - 1) / T;
    ksp = std::max<int>(ksp, (int)(wl - wf + 1));
  }
  if (ksp > kMaxSplit) return gp;
  GemmPlan out = gp;
  out.sk = (int)W;
  out.ksplit = ksp;
  out.kper = nch * bk;
  return out;
}

GemmPlan choose_gemm(Elt elt, bool trans, int64_t n, int r, int num_cu) {
  int mw = 0, s = 0, ks = 0;
  if (table_tile(elt, trans && elt != Elt::BF16, n, r, &mw, &s, &ks))
    return make_gemm_plan(elt, trans && elt != Elt::BF16, n, r, mw, s, ks, num_cu);
  // (tiles that fit two workgroups per CU without spilling at this r)
  switch (elt) {
    case Elt::BF16: return make_gemm_plan(elt, false, n, r, 4, 2, 0, num_cu);
    case Elt::F32:
      // Measured at n = 30658, r = 40 (rows padded to 256 floats): transposed
      // 4x4 0.94 ms; NN 4x4 0.99 ms against 1.09 ms for 2x4
      if (trans) return make_gemm_plan(elt, true, n, r, 4, 4, 0, num_cu);
      return n >= 4096 && r <= 48 ? make_gemm_plan(elt, false, n, r, 4, 4, 0, num_cu)
                                  : make_gemm_plan(elt, false, n, r, 2, 4, 0, num_cu);
    case Elt::F64: {
      // Measured at n = 30658, r = 40 on one MI355X (128-byte rows): NN 16x16x4
      // 4x4 tile 1.69 ms vs 4x4x4 4x2 1.72 ms (its 64-byte row chunks use half
      // a line per chunk); transposed 4x4x4 4x2 1.57 ms (every load 4 full
      // lines) vs 1.68 ms for the next best.  Non-spilling tiles for larger r.
      const int g4 = f64_groups(r);
      if (trans)
        return g4 <= 10 ? make_gemm_plan(elt, true, n, r, 4, 2, 0, num_cu)
               : g4 <= 14 ? make_gemm_plan(elt, true, n, r, 2, 4, 0, num_cu)
                          : make_gemm_plan(elt, true, n, r, 1, 8, 0, num_cu);
      return r <= 48 ? make_gemm_plan(elt, false, n, r, 4, 4, 0, num_cu)
                     : make_gemm_plan(elt, false, n, r, 2, 4, 0, num_cu);
    }
  }
  return make_gemm_plan(elt, trans, n, r, 2, 8, 0, num_cu);
}

static bool plan_ok(Elt elt, const GemmPlan& gp, int64_t n, int r) {
  if (gp.sk > 0)
    return (elt == Elt::F64 || elt == Elt::BF16) && r >= 1 && r <= kMaxRank && n >= 1 &&
           gp.ksplit >= 1 && gp.ksplit <= kMaxSplit && gemm_cfg_valid(elt, gp.mw, gp.s);
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
  if (elt == Elt::F64 && gp.sk > 0) {
    if (!trans) {
      set_error("launch_gemm: stream-K plan for the row-major product");
      return CPHIFI_INVALID_ARG;
    }
    return dispatch_f64_sk(gp, f64_groups(r), g, st);
  }
  if (elt == Elt::F64)
    return trans ? dispatch_cfg_f64<true>(gp.mw, gp.s, f64_groups(r), g, gp.ksplit, st)
                 : dispatch_cfg_f64<false>(gp.mw, gp.s, f64_groups(r), g, gp.ksplit, st);
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
// tiled: U in the 16 x 64 tile layout (tiles::bf16_tiled_off, ldu % 64 == 0).
int launch_gemm_bf16(const GemmPlan& gp, const __bf16* U, int64_t ldu, int64_t n,
                     const double* X, int64_t ldx, int r, const double* xscale, void* part,
                     __bf16* xt_hi, __bf16* xt_lo, int64_t ldxt, const int32_t* done,
                     hipStream_t st, bool tiled) {
  const int nb = (r + 15) / 16;
  const int64_t bk = gemm_bk(Elt::BF16, gp.s);
  const int64_t nround = (n + bk - 1) / bk * bk;
  if (!plan_ok(Elt::BF16, gp, n, r) || ldu % (tiled ? 64 : 8) != 0 || ldu < nround ||
      ldxt < nround || ldxt % 8 != 0 || ldx < r) {
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
  if (gp.sk > 0) {
    if (!tiled || gp.mw != 4 || gp.s != 2) {
      set_error("launch_gemm_bf16: the stream-K form needs the tiled layout and the 4x2 tile");
      return CPHIFI_INVALID_ARG;
    }
    SkArgs sk{};
    sk.nrb = (n + 255) / 256;  // rows of the 4x2 tile: 4 waves x 4 blocks x 16
    sk.nch = (n + bk - 1) / bk;
    sk.wgs = gp.sk;
    sk.ksplit = gp.ksplit;
    switch (nb) {
      case 1: hipLaunchKernelGGL((gemm_bf16_sk_kernel<1, 4, 2>), dim3((unsigned)gp.sk), dim3(256), 0, st, g, sk); break;
      case 2: hipLaunchKernelGGL((gemm_bf16_sk_kernel<2, 4, 2>), dim3((unsigned)gp.sk), dim3(256), 0, st, g, sk); break;
      case 3: hipLaunchKernelGGL((gemm_bf16_sk_kernel<3, 4, 2>), dim3((unsigned)gp.sk), dim3(256), 0, st, g, sk); break;
      default: hipLaunchKernelGGL((gemm_bf16_sk_kernel<4, 4, 2>), dim3((unsigned)gp.sk), dim3(256), 0, st, g, sk); break;
    }
    CPHIFI_CHECK_LAUNCH();
    return CPHIFI_OK;
  }
  return tiled ? dispatch_cfg_bf16<true>(gp.mw, gp.s, nb, g, gp.ksplit, st)
               : dispatch_cfg_bf16<false>(gp.mw, gp.s, nb, g, gp.ksplit, st);
}

}  // namespace cphifi
