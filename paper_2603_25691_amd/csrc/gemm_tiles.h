// Workgroup tiles of the skinny products Y = op(U) * diag(xscale) * X with U
// n x n and X n x r (r <= 64) on gfx950 MFMA: the K X, K Yhat1, U_K^T R and
// U_K T products of the two-step matrix-free product (Section 4.4.1) and of
// the preconditioner apply (eq. fx).  Each tile is one workgroup's share of one
// product -- a block of output rows over one k-range -- so the same code runs
// as a plain grid (gemm.hip) and as work items of the persistent batched
// solver (batch.hip).
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
//  * split-K writes deterministic partial sums (one slab per k-range) that the
//    consumer adds in a fixed order (no atomics).
#pragma once

#include "cphifi_internal.h"

#include <type_traits>

namespace cphifi {
namespace tiles {

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

// LDS elements of a 16x16x4 tile (two staged chunks of BK rows of X).
template <typename TA, int NB, int S>
constexpr int k4_lds_elems() {
  return 2 * (4 * S) * (NB * 16 + 16 / S);
}
// LDS elements of a BF16 tile (two chunks, hi and lo parts, NC rows of BK+8).
template <int NB, int S>
constexpr int bf16_lds_elems() {
  return 2 * 2 * (NB * 16) * (32 * S + 8);
}
// Output rows of one tile.
constexpr int tile_rows(int mw) { return 4 * mw * 16; }

// ------------------------------------------------- FP64 / FP32 (16x16x4) tile
// Rows [bx*tile_rows(MW), ...) over k in [by*kper, (by+1)*kper) into partial
// slab `by`; tid is the thread index (threadIdx.x, or item_tid() inside a
// persistent kernel).  VW: elements per vector load of the n x n operand along k (NN
// form only; requires ldu % VW == 0 and a 16-byte aligned U).  xs: LDS of
// k4_lds_elems<TA, NB, S>() elements.
template <typename TA, int NB, int MW, int S, bool TRANS, int VW>
__device__ __forceinline__ void gemm_k4_tile(const GArgs& g, int64_t bx, int64_t by, TA* xs,
                                             int tid) {
  using AccT = typename std::conditional<std::is_same<TA, double>::value, d4, f4>::type;
  typedef TA VecT __attribute__((ext_vector_type(VW)));
  static_assert(S % VW == 0, "S must be a multiple of the vector width");
  constexpr int BK = 4 * S;
  constexpr int NC = NB * 16;
  constexpr int LDX = NC + 16 / S;  // pad spreads the 4 k-groups over distinct banks
  constexpr int XE = BK * NC;       // staged elements per chunk
  constexpr int XB = BK * LDX;      // LDS elements per buffer
  constexpr int XPT = (XE + 255) / 256;

  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, kk = lane >> 4;
  const int64_t n = g.n;
  const int64_t ldu = g.ldu;
  const int64_t mbase = bx * (4 * MW * 16) + (int64_t)wave * (MW * 16);
  const int64_t kbeg = by * g.kper;
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
      if (tid + j * 256 < XE) xs[buf * XB + xlds[j]] = xr[j];
  };
  auto compute = [&](const TA (&a)[MW][S], int buf) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      TA b[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) b[nb] = xs[buf * XB + (kk * S + s) * LDX + nb * 16 + li];
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

  // Chunk loop unrolled twice with ping-pong operand registers a0 / a1: the
  // next chunk's loads go to the other set, so they stay in flight across
  // this chunk's MFMAs (a register copy would let the compiler sink them).
  // The steady state prefetches unconditionally (no branch for the waitcnt
  // insertion to merge conservatively) and runs only while both chunks it
  // prefetches are full ones; the remaining chunks, the k tail among them,
  // go through the general fetch.
  auto fetch_full = [&](TA (&xr)[XPT], TA (&dst)[MW][S], int64_t c) {
    const int64_t k0 = kbeg + c * BK;
    stageX(xr, k0, false);
    loadA(dst, k0);
  };
  if (nchunk > 0) {
    TA a0[MW][S], a1[MW][S];
    TA xr[XPT];
    fetch(xr, a0, 0);
    storeX(0, xr);
    __syncthreads();
    int64_t c = 0;
    while (c + 2 < nfull) {  // chunks c + 1 and c + 2 are full ones
      fetch_full(xr, a1, c + 1);
      __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the MFMAs
      compute(a0, (int)(c & 1));
      storeX((int)((c + 1) & 1), xr);
      __syncthreads();
      ++c;
      fetch_full(xr, a0, c + 1);
      __builtin_amdgcn_sched_barrier(0);
      compute(a1, (int)(c & 1));
      storeX((int)((c + 1) & 1), xr);
      __syncthreads();
      ++c;
    }
    for (;;) {  // at most three chunks left; a0 holds chunk c
      bool more = c + 1 < nchunk;
      if (more) fetch(xr, a1, c + 1);
      compute(a0, (int)(c & 1));
      if (more) storeX((int)((c + 1) & 1), xr);
      __syncthreads();
      if (!more) break;
      ++c;
      more = c + 1 < nchunk;
      if (more) fetch(xr, a0, c + 1);
      compute(a1, (int)(c & 1));
      if (more) storeX((int)((c + 1) & 1), xr);
      __syncthreads();
      if (!more) break;
      ++c;
    }
  }

  TA* part = (TA*)g.part + by * n * g.ldp;
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

// --------------------------------------------------- FP64 4x4x4 (4-block) tile
// The FP64 16x16x4 MFMA needs N in multiples of 16 (r = 40 pads to 48, 17 %
// wasted), and one wave can start one only every ~128 cycles, so the pipe
// (64 cycles per instruction) is full only while both waves of a SIMD issue.
// v_mfma_f64_4x4x4_4b runs four independent 4x4x4 products per instruction at
// the same flop rate (16 cycles each) and a single wave can issue them back to
// back.  Its lanes: block b = (lane / 4) % 4; A_b[i][k] in lane 16 k + 4 b + i,
// B_b[k][j] in lane 16 k + 4 b + j, D_b[i][j] in lane 16 i + 4 b + j.  Here the
// four blocks are four groups of 4 output rows sharing one 4-column group of X:
// lane (li = lane % 16, kk = lane / 16) supplies A = U[row li][k kk] -- the same
// operand as the 16x16x4 tile -- and B = X[k kk][4 c + lane % 4]; the result
// of column group c sits at row 4 ((lane / 4) % 4) + lane / 16, column
// 4 c + lane % 4.  NC4 column groups cover 4 NC4 >= r columns.
__device__ __forceinline__ double mfma4x4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

template <int NC4, int S>
constexpr int k4x4_lds_elems() {
  return 2 * (4 * S) * (4 * NC4 + 16 / S);
}

// Rows [bx*tile_rows(MW), ...) over k in [kbeg, kend) (kbeg a multiple of
// 4 S) into partial slab `slab`.  NT: the n x n operand's loads carry the
// non-temporal hint (it is streamed once per product; 1.59 -> 1.54 ms at
// n = 30658, r = 40).
template <int NC4, int MW, int S, bool TRANS, int VW, bool NT = false>
__device__ __forceinline__ void gemm_f64x4_tile(const GArgs& g, int64_t bx, int64_t kbeg,
                                                int64_t kend, int64_t slab, double* xs,
                                                int tid) {
  typedef double VecT __attribute__((ext_vector_type(VW)));
  static_assert(S % VW == 0, "S must be a multiple of the vector width");
  constexpr int BK = 4 * S;
  constexpr int NC = 4 * NC4;
  constexpr int LDX = NC + 16 / S;  // pad spreads the 4 k-groups over distinct banks
  constexpr int XE = BK * NC;
  constexpr int XB = BK * LDX;
  constexpr int XPT = (XE + 255) / 256;

  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, kk = lane >> 4;
  const int jj = lane & 3;                                // column within a group
  const int orow = 4 * ((lane >> 2) & 3) + (lane >> 4);  // output row within 16
  const int64_t n = g.n;
  const int64_t ldu = g.ldu;
  const int64_t mbase = bx * (4 * MW * 16) + (int64_t)wave * (MW * 16);
  const double* __restrict__ U = (const double*)g.U;

  const double* abase[MW];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb) {
    const int64_t rc = min(mbase + mb * 16 + li, n - 1);
    abase[mb] = TRANS ? U + (int64_t)(kk * S) * ldu + rc : U + rc * ldu + kk * S;
  }
  const double* __restrict__ X = g.X;
  int xoff[XPT], xlds[XPT], xkid[XPT];
  bool xon[XPT];
#pragma unroll
  for (int j = 0; j < XPT; ++j) {
    const int e = tid + j * 256;
    const int kidx = e / NC, c = e % NC;
    xkid[j] = kidx;
    xoff[j] = kidx * (int)g.ldx + c;
    xlds[j] = kidx * LDX + c;
    xon[j] = e < XE && c < g.r;
  }

  double acc[MW][NC4];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb)
#pragma unroll
    for (int c = 0; c < NC4; ++c) acc[mb][c] = 0.0;

  const int64_t span = kend - kbeg;
  const int64_t nfull = span > 0 ? span / BK : 0;
  const bool has_tail = span > 0 && (span % BK) != 0;
  const int64_t nchunk = nfull + (has_tail ? 1 : 0);

  auto loadA = [&](double (&dst)[MW][S], int64_t k0) {
#pragma unroll
    for (int mb = 0; mb < MW; ++mb) {
      if (TRANS) {
        const double* p = abase[mb] + k0 * ldu;
#pragma unroll
        for (int s = 0; s < S; ++s)
          dst[mb][s] = NT ? __builtin_nontemporal_load(p + (int64_t)s * ldu) : p[(int64_t)s * ldu];
      } else {
        const double* p = abase[mb] + k0;
#pragma unroll
        for (int v = 0; v < S / VW; ++v) {
          const VecT t = *(const VecT*)(p + v * VW);
#pragma unroll
          for (int w = 0; w < VW; ++w) dst[mb][v * VW + w] = t[w];
        }
      }
    }
  };
  auto loadA_tail = [&](double (&dst)[MW][S], int64_t k0) {
#pragma unroll
    for (int mb = 0; mb < MW; ++mb)
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int64_t k = k0 + kk * S + s;
        const int64_t dk = min(k, n - 1) - kk * S;
        const double v = TRANS ? abase[mb][dk * ldu] : abase[mb][dk];
        dst[mb][s] = (k < kend) ? v : 0.0;
      }
  };
  auto stageX = [&](double (&xr)[XPT], int64_t k0, bool tail) {
    const double* xp = X + k0 * g.ldx;
#pragma unroll
    for (int j = 0; j < XPT; ++j) {
      double v = 0.0;
      const bool on = xon[j] && (!tail || k0 + xkid[j] < kend);
      if (on) {
        v = xp[xoff[j]];
        if (g.xscale != nullptr) v *= g.xscale[k0 + xkid[j]];
      }
      xr[j] = v;
    }
  };
  auto storeX = [&](int buf, const double (&xr)[XPT]) {
#pragma unroll
    for (int j = 0; j < XPT; ++j)
      if (tid + j * 256 < XE) xs[buf * XB + xlds[j]] = xr[j];
  };
  auto compute = [&](const double (&a)[MW][S], int buf) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      double b[NC4];
#pragma unroll
      for (int c = 0; c < NC4; ++c) b[c] = xs[buf * XB + (kk * S + s) * LDX + 4 * c + jj];
#pragma unroll
      for (int mb = 0; mb < MW; ++mb)
#pragma unroll
        for (int c = 0; c < NC4; ++c) acc[mb][c] = mfma4x4(a[mb][s], b[c], acc[mb][c]);
    }
  };
  auto fetch = [&](double (&xr)[XPT], double (&dst)[MW][S], int64_t c) {
    const int64_t k0 = kbeg + c * BK;
    const bool tail = c == nfull;
    stageX(xr, k0, tail);
    if (tail)
      loadA_tail(dst, k0);
    else
      loadA(dst, k0);
  };
  auto fetch_full = [&](double (&xr)[XPT], double (&dst)[MW][S], int64_t c) {
    const int64_t k0 = kbeg + c * BK;
    stageX(xr, k0, false);
    loadA(dst, k0);
  };
  // Same chunk loop as gemm_k4_tile (ping-pong registers, branch-free steady
  // state over full chunks, tail-aware epilogue).
  if (nchunk > 0) {
    double a0[MW][S], a1[MW][S];
    double xr[XPT];
    fetch(xr, a0, 0);
    storeX(0, xr);
    __syncthreads();
    int64_t c = 0;
    while (c + 2 < nfull) {
      fetch_full(xr, a1, c + 1);
      __builtin_amdgcn_sched_barrier(0);
      compute(a0, (int)(c & 1));
      storeX((int)((c + 1) & 1), xr);
      __syncthreads();
      ++c;
      fetch_full(xr, a0, c + 1);
      __builtin_amdgcn_sched_barrier(0);
      compute(a1, (int)(c & 1));
      storeX((int)((c + 1) & 1), xr);
      __syncthreads();
      ++c;
    }
    for (;;) {
      bool more = c + 1 < nchunk;
      if (more) fetch(xr, a1, c + 1);
      compute(a0, (int)(c & 1));
      if (more) storeX((int)((c + 1) & 1), xr);
      __syncthreads();
      if (!more) break;
      ++c;
      more = c + 1 < nchunk;
      if (more) fetch(xr, a0, c + 1);
      compute(a1, (int)(c & 1));
      if (more) storeX((int)((c + 1) & 1), xr);
      __syncthreads();
      if (!more) break;
      ++c;
    }
  }

  double* part = (double*)g.part + slab * n * g.ldp;
#pragma unroll
  for (int mb = 0; mb < MW; ++mb) {
    const int64_t row = mbase + mb * 16 + orow;
    if (row < n) {
#pragma unroll
      for (int c = 0; c < NC4; ++c) part[row * g.ldp + 4 * c + jj] = acc[mb][c];
    }
  }
}

// ------------------------------------------------------- BF16 (16x16x32) tile
// Element offset of U[i][k] in the tiled BF16 layout: 16-row x 64-column
// tiles of 2 KB, stored row-block by row-block with the column tiles of a
// row block consecutive, each tile row-major.  A wave's 16-row MFMA block
// then reads one contiguous 2 KB tile per 64 columns instead of 16 rows x
// 128 bytes strided by the row pitch (a plain read of the operand in this
// pattern ran at 5.96 TB/s against 5.44 TB/s row-major on MI355X).
// ldu is a multiple of 64; the row blocks cover round_up(n, 16) rows.
__host__ __device__ __forceinline__ int64_t bf16_tiled_off(int64_t i, int64_t k, int64_t ldu) {
  return ((i >> 4) * (ldu >> 6) + (k >> 6)) * 1024 + (i & 15) * 64 + (k & 63);
}

// U is a zero-padded bf16 copy (row stride ldu >= round_up(n, BK)), row-major
// or (TILED) in the layout of bf16_tiled_off; the n x r operand arrives
// pre-split as hi + lo bf16 parts, transposed to c-major rows of stride ldxt,
// so the product carries ~16 significant bits of X while U stays at bf16.
// Accumulation is FP32.  xs: LDS of bf16_lds_elems<NB, S>().
// Rows [bx*tile_rows(MW), ...) over k in [kbeg, kend) (kbeg a multiple of the
// chunk, 32 S) into partial slab `slab`.
template <int NB, int MW, int S, bool TILED = false, int DEPTH = 2>
__device__ __forceinline__ void gemm_bf16_tile(const GArgs& g, int64_t bx, int64_t kbeg,
                                               int64_t kend, int64_t slab, __bf16* xs,
                                               int tid) {
  static_assert(DEPTH == 2 || DEPTH == 3, "U chunks in flight: 2 or 3");
  constexpr int BK = 32 * S;
  constexpr int NC = NB * 16;
  constexpr int LDK = BK + 8;           // bf16 elements per LDS row (bank spread)
  constexpr int V8 = BK / 8;            // 16-byte vectors per staged row
  constexpr int XV = NC * V8;           // 16-byte vectors per chunk and part
  constexpr int XPT = (XV + 255) / 256;
  constexpr int XP = NC * LDK;          // LDS elements per part
  constexpr int XB = 2 * XP;            // LDS elements per buffer (hi, lo)

  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, kk = lane >> 4;
  const int64_t n = g.n;
  const int64_t mbase = bx * (4 * MW * 16) + (int64_t)wave * (MW * 16);
  const __bf16* __restrict__ U = (const __bf16*)g.U;

  // Offset of the lane's first element of a chunk starting at k0 = 0: its row
  // and its column offset kk * 8 S.  Tiled, chunks start at multiples of 64
  // and a lane's 8 S elements of a chunk stay in one tile row, so a chunk at
  // k0 adds (k0 / 64) tiles of 1024 elements.
  static_assert(!TILED || BK % 64 == 0, "tiled BF16 chunks span whole tiles");
  int64_t rowc[MW];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb) {
    const int64_t row = min(mbase + mb * 16 + li, n - 1);
    rowc[mb] = TILED ? bf16_tiled_off(row, kk * (8 * S), g.ldu) : row * g.ldu + kk * (8 * S);
  }

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
        dst[mb][s] = *(const u32x4*)(U + rowc[mb] + (TILED ? (k0 >> 6) * 1024 : k0) + 8 * s);
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
        *(u32x4*)(&xs[buf * XB + c * LDK + 8 * v]) = xr[0][j];
        *(u32x4*)(&xs[buf * XB + XP + c * LDK + 8 * v]) = xr[1][j];
      }
    }
  };
  auto compute = [&](const u32x4 (&a)[MW][S], int buf) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int off = (nb * 16 + li) * LDK + kk * (8 * S) + 8 * s;
        const bf16x8 bh = __builtin_bit_cast(bf16x8, *(const u32x4*)(&xs[buf * XB + off]));
        const bf16x8 bl = __builtin_bit_cast(bf16x8, *(const u32x4*)(&xs[buf * XB + XP + off]));
#pragma unroll
        for (int mb = 0; mb < MW; ++mb) {
          const bf16x8 av = __builtin_bit_cast(bf16x8, a[mb][s]);
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bh, acc[mb][nb], 0, 0, 0);
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bl, acc[mb][nb], 0, 0, 0);
        }
      }
    }
  };

  // X rows of the next chunk are fetched before its U rows: vmcnt retires in
  // order, so filling LDS does not wait for the larger U prefetch.  The chunk
  // loop is unrolled twice with ping-pong U registers a0 / a1, so the next
  // chunk's loads stay in flight across this chunk's MFMAs; the steady state
  // prefetches unconditionally and the last one or two chunks are peeled.
  auto fetch = [&](u32x4 (&xr)[2][XPT], u32x4 (&dst)[MW][S], int64_t c) {
    stageX(xr, kbeg + c * BK);
    loadA(dst, kbeg + c * BK);
  };
  if (DEPTH == 3 && nchunk > 0) {
    // Three U buffers: chunk c + 2 is loading while chunk c is multiplied (X
    // stays one chunk ahead through LDS).  Steady state in groups of three
    // steps, rotating the buffers; then at most four peeled steps.
    u32x4 a0[MW][S], a1[MW][S], a2[MW][S];
    u32x4 xr[2][XPT];
    fetch(xr, a0, 0);
    storeX(0, xr);
    if (nchunk > 1) loadA(a1, kbeg + BK);
    __syncthreads();
    int64_t c = 0;
    auto step = [&](const u32x4 (&cur)[MW][S], u32x4 (&ahead)[MW][S]) {
      stageX(xr, kbeg + (c + 1) * BK);  // X of c + 1, then U of c + 2
      loadA(ahead, kbeg + (c + 2) * BK);
      __builtin_amdgcn_sched_barrier(0);
      compute(cur, (int)(c & 1));
      storeX((int)((c + 1) & 1), xr);
      __syncthreads();
      ++c;
    };
    while (c + 5 <= nchunk) {
      step(a0, a2);
      step(a1, a0);
      step(a2, a1);
    }
    auto tail = [&](const u32x4 (&cur)[MW][S], u32x4 (&ahead)[MW][S]) {
      if (c >= nchunk) return;
      const bool more = c + 1 < nchunk;
      if (more) stageX(xr, kbeg + (c + 1) * BK);
      if (c + 2 < nchunk) loadA(ahead, kbeg + (c + 2) * BK);
      compute(cur, (int)(c & 1));
      if (more) {
        storeX((int)((c + 1) & 1), xr);
        __syncthreads();
      }
      ++c;
    };
    tail(a0, a2);
    tail(a1, a0);
    tail(a2, a1);
    tail(a0, a2);
  } else if (nchunk > 0) {
    u32x4 a0[MW][S], a1[MW][S];
    u32x4 xr[2][XPT];
    fetch(xr, a0, 0);
    storeX(0, xr);
    __syncthreads();
    int64_t c = 0;
    while (c + 2 < nchunk) {
      fetch(xr, a1, c + 1);
      __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the MFMAs
      compute(a0, (int)(c & 1));
      storeX((int)((c + 1) & 1), xr);
      __syncthreads();
      ++c;
      fetch(xr, a0, c + 1);
      __builtin_amdgcn_sched_barrier(0);
      compute(a1, (int)(c & 1));
      storeX((int)((c + 1) & 1), xr);
      __syncthreads();
      ++c;
    }
    if (c + 1 < nchunk) {
      fetch(xr, a1, c + 1);
      compute(a0, (int)(c & 1));
      storeX((int)((c + 1) & 1), xr);
      __syncthreads();
      ++c;
      compute(a1, (int)(c & 1));
    } else {
      compute(a0, (int)(c & 1));
    }
  }

  float* part = (float*)g.part + slab * n * g.ldp;
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

}  // namespace tiles
}  // namespace cphifi
