// Batched mixed-precision solver: many independent unaligned RKHS-mode
// subproblems (Section 4.4) of uneven n and r, solved together by ONE
// persistent kernel launch that is captured, with its reset kernel, in a HIP
// graph.
//
// Method per member (the same as cphifi_ui_solve at MIXED_BF16): FP64 iterative
// refinement of (F^T F + lambda I kron K + rho I) w = b carried out in the
// eigenbasis of K (w = U_K xbar, the rotation of Section 3.3): the FP64
// residual of the rotated system rbar = U^T b - Abar xbar, inner PCG solves of
// Abar_lp dbar = rbar with the BF16-rounded eigenvectors and the r x r middle
// step of eq. (fx) as preconditioner, xbar += dbar; at the end W = U xbar and
// its FP64 residual in the original form certifies it.
//
// The launch starts from the observed values y: the per-solve setup of
// Section 4.4.2 (V = Z^T Z, eig(V) by Jacobi, the inverse diagonal D) and the
// observed MTTKRP B of the right-hand side b = K B (Section 4) run inside it,
// b itself is never formed: bbar = U^T b = D_K U^T B, and the certificate is
// b - A W = K (B - Yhat1 - lambda W) - rho W with ||b|| = ||bbar||.
//
// Execution model.  Each member runs a small state machine (mode):
//   SETUP -> ROT_B [-> ROT_W] -> RES0 -> INNER ... INNER -> RES -> INNER ...
//         -> RES -> FINAL -> CERT -> DONE   (or back to RES if CERT misses tol)
// and the kernel advances every member by one step per *round*.  A round has
// eight phases; in each phase every active member contributes work items
// according to its mode:
//
//   phase  INNER (one PCG iteration)     RES (rotated FP64 residual)   CERT (FP64 residual of W)
//   A      BF16 U (D_K p)                FP64 U (D_K xbar)             FP64 K W
//   OBS    gather-dot-scatter (eqs. vl, yhat1)
//   ROWS   split segments + hi/lo BF16 split of Yhat1; split segments; T = B - Yhat1 - lambda W
//   B      BF16 U^T Yhat1                FP64 U^T Yhat1                FP64 K T
//   FIN    q = D_K(Y + lambda p) + rho p rbar = bbar - Abar xbar       rf = K T - rho W
//   UPD    alpha; dbar, r update         -                             -
//   PREC   z = ((r U_V) had D) U_V^T     z (when refining on)          -
//   CTRL   beta; p update + split;       relres test; p = z + split    certificate test
//          at the stop xbar += dbar
// SETUP uses A (V, one item), OBS (the MTTKRP gather), ROWS (split segments),
// B (eig(V), one item) and FIN (D and dK clamped, W = 0 unless warm);
// ROT_B / ROT_W (D_K U^T B, U^T W0 for a warm start) and FINAL (W = U xbar)
// use phases A and FIN; RES0 (rbar = bbar) has no products.
//
// Work items of a phase (product tiles, wave tasks of the gather, row chunks
// of the vector steps) are handed out by an atomic counter; phases are
// separated by a bounded grid barrier; reductions write one partial per item
// and every consumer adds them in a fixed order, so results do not depend on
// the schedule.  Per-member scalars stay on the device.  Every wait is bounded:
// a barrier that times out raises an error flag on which every workgroup
// leaves, so the launch always drains.
#include "cphifi_internal.h"
#include "gemm_tiles.h"
#include "jacobi.h"
#include "obs_tile.h"
#include "plan.h"

#include <cmath>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <vector>

using namespace cphifi;

#define TRY_RC(x)                    \
  do {                               \
    const int s_ = (x);              \
    if (s_ != CPHIFI_OK) return s_;  \
  } while (0)

namespace {

constexpr int kMaxBatch = 256;     // members per batch (one thread each in the round setup)
constexpr int kRC = 128;           // rows per vector work item
constexpr int kTPW = 8;            // gather tasks per wave in one work item
constexpr int kSlots = 8;          // phases per round
constexpr int64_t kMaxN = 65536;   // also keeps a vector phase's partials within red[]
static_assert(kMaxN <= (int64_t)kRC * kMaxVecBlocks, "partials of a vector phase fit red[]");
// Members have r <= 48 (three 16-column MFMA blocks): the largest tiles then
// fit the register budget of two workgroups per CU.
constexpr int kBatchRank = 48;
constexpr int kSmemBytes = 65536;  // LDS shared by the phases (largest: B of a member, J r <= 8192)

static_assert(tiles::bf16_lds_elems<3, 2>() * 2 <= kSmemBytes, "bf16 tile LDS");
static_assert(tiles::k4_lds_elems<double, 3, 4>() * 8 <= kSmemBytes, "f64 NN tile LDS");
static_assert(tiles::k4_lds_elems<double, 3, 4>() * 8 <= kSmemBytes, "f64 T tile LDS");
static_assert((kBatchRank * kBatchRank + 4 * kWave) * 8 <= kSmemBytes, "preconditioner LDS");
static_assert(2 * kBatchRank * kRC * 2 <= kSmemBytes, "split transpose LDS");
static_assert(sizeof(JacobiLds<kBatchRank>) <= kSmemBytes, "Jacobi LDS");

enum : int32_t {
  M_SETUP = 0,  // V, eig(V), D, the observed MTTKRP B; W = 0 unless warm
  M_ROT_B = 1,  // bbar = U^T b = D_K U^T B; ||b||^2 = ||bbar||^2
  M_ROT_W = 2,  // xbar = U^T W (warm start)
  M_RES0 = 3,   // rbar = bbar (xbar = 0)
  M_RES = 4,    // rbar = bbar - Abar xbar (FP64)
  M_INNER = 5,  // one inner PCG iteration
  M_FINAL = 6,  // W = U xbar
  M_CERT = 7,   // FP64 residual of W
  M_DONE = 8,
  M_RESC = 9    // rbar = U^T rf (a certificate missed: its residual continues)
};
enum : int { S_A = 0, S_OBS = 1, S_ROWS = 2, S_B = 3, S_FIN = 4, S_UPD = 5, S_PREC = 6, S_CTRL = 7 };

// Constants of one member (device copy; never written by the kernel).
struct BSub {
  int64_t n, ldk, ldl, I, J;
  int32_t r, ldp, nb, ocls;  // ocls: lane layout class of the gather (from r)
  int32_t nrc, ntask, ntaskw, nmulti;  // ntaskw: gather work items
  int32_t orow, own;                   // gather by lane rows (short segments); one
                                       // sample per time point (A read per segment)
  const double* K;
  const double* UK;
  const double* dK;   // eigenvalues of K as given (clamped at 0 into dKc)
  const double* y;    // observed values (bound per solve)
  const double* Vin;  // caller's V = Z^T Z, or null: formed from A and B
  double* W;
  const int32_t* obs_i;
  const int32_t* obs_j;
  const double* A;
  const double* B;
  const float *A32, *B32;  // FP32 copies (the inner gather computes in FP32)
  const int32_t *tseg, *tbeg, *tend, *tslot, *tfirst, *mptr, *rowm, *obs_ptr;
  void* part;
  double* tpart;
  double *V, *UV, *dV, *D, *dKc;
  const __bf16 *ulp, *utlp;
  __bf16 *xthi, *xtlo;
  double *X, *R, *Z, *P, *Q, *XH, *Y1, *RF;
  double *BB, *XA;  // bbar = U^T b, accumulated xbar
  double* BM;       // the observed MTTKRP B
  double *red0, *red1, *red2;
  int32_t bf_mw, bf_ks, bf_nrb, fn_ks, fn_nrb, fn_vw, ft_mw, ft_ks, ft_nrb, pad0;
  int64_t bf_kper, fn_kper, ft_kper;
  double lam, rho, gamma, tol, inner_tol2;
  int32_t maxit, max_refine, warm;
  int32_t adapt;  // default inner tolerance: loosened on steps that cannot reach tol
};

template <typename P>
__device__ __forceinline__ P global_word(uint64_t w) {
  return (P)(__attribute__((address_space(1))) char*)(uintptr_t)w;
}

// A member's constants, read through the constant address space: the kernel
// never writes them, and scalar loads keep them out of vector registers.
__device__ __forceinline__ BSub load_sub(const BSub* sub, int b) {
  static_assert(sizeof(BSub) % 8 == 0, "BSub is copied in 8-byte words");
  typedef __attribute__((address_space(4))) const uint64_t cword;
  const cword* src = (const cword*)(sub + b);
  uint64_t w[sizeof(BSub) / 8];
#pragma unroll
  for (int k = 0; k < (int)(sizeof(BSub) / 8); ++k) w[k] = src[k];
  BSub s;
  __builtin_memcpy(&s, w, sizeof(BSub));
  // Every pointer refers to global memory; rebuilding it as a global-space
  // pointer lets the compiler use global (not flat) loads and stores.
  s.K = global_word<decltype(s.K)>(w[offsetof(BSub, K) / 8]);
  s.UK = global_word<decltype(s.UK)>(w[offsetof(BSub, UK) / 8]);
  s.dK = global_word<decltype(s.dK)>(w[offsetof(BSub, dK) / 8]);
  s.y = global_word<decltype(s.y)>(w[offsetof(BSub, y) / 8]);
  s.Vin = global_word<decltype(s.Vin)>(w[offsetof(BSub, Vin) / 8]);
  s.W = global_word<decltype(s.W)>(w[offsetof(BSub, W) / 8]);
  s.obs_i = global_word<decltype(s.obs_i)>(w[offsetof(BSub, obs_i) / 8]);
  s.obs_j = global_word<decltype(s.obs_j)>(w[offsetof(BSub, obs_j) / 8]);
  s.A = global_word<decltype(s.A)>(w[offsetof(BSub, A) / 8]);
  s.B = global_word<decltype(s.B)>(w[offsetof(BSub, B) / 8]);
  s.A32 = global_word<decltype(s.A32)>(w[offsetof(BSub, A32) / 8]);
  s.B32 = global_word<decltype(s.B32)>(w[offsetof(BSub, B32) / 8]);
  s.tseg = global_word<decltype(s.tseg)>(w[offsetof(BSub, tseg) / 8]);
  s.tbeg = global_word<decltype(s.tbeg)>(w[offsetof(BSub, tbeg) / 8]);
  s.tend = global_word<decltype(s.tend)>(w[offsetof(BSub, tend) / 8]);
  s.tslot = global_word<decltype(s.tslot)>(w[offsetof(BSub, tslot) / 8]);
  s.tfirst = global_word<decltype(s.tfirst)>(w[offsetof(BSub, tfirst) / 8]);
  s.mptr = global_word<decltype(s.mptr)>(w[offsetof(BSub, mptr) / 8]);
  s.rowm = global_word<decltype(s.rowm)>(w[offsetof(BSub, rowm) / 8]);
  s.obs_ptr = global_word<decltype(s.obs_ptr)>(w[offsetof(BSub, obs_ptr) / 8]);
  s.part = global_word<decltype(s.part)>(w[offsetof(BSub, part) / 8]);
  s.tpart = global_word<decltype(s.tpart)>(w[offsetof(BSub, tpart) / 8]);
  s.V = global_word<decltype(s.V)>(w[offsetof(BSub, V) / 8]);
  s.UV = global_word<decltype(s.UV)>(w[offsetof(BSub, UV) / 8]);
  s.dV = global_word<decltype(s.dV)>(w[offsetof(BSub, dV) / 8]);
  s.D = global_word<decltype(s.D)>(w[offsetof(BSub, D) / 8]);
  s.dKc = global_word<decltype(s.dKc)>(w[offsetof(BSub, dKc) / 8]);
  s.ulp = global_word<decltype(s.ulp)>(w[offsetof(BSub, ulp) / 8]);
  s.utlp = global_word<decltype(s.utlp)>(w[offsetof(BSub, utlp) / 8]);
  s.xthi = global_word<decltype(s.xthi)>(w[offsetof(BSub, xthi) / 8]);
  s.xtlo = global_word<decltype(s.xtlo)>(w[offsetof(BSub, xtlo) / 8]);
  s.X = global_word<decltype(s.X)>(w[offsetof(BSub, X) / 8]);
  s.R = global_word<decltype(s.R)>(w[offsetof(BSub, R) / 8]);
  s.Z = global_word<decltype(s.Z)>(w[offsetof(BSub, Z) / 8]);
  s.P = global_word<decltype(s.P)>(w[offsetof(BSub, P) / 8]);
  s.Q = global_word<decltype(s.Q)>(w[offsetof(BSub, Q) / 8]);
  s.XH = global_word<decltype(s.XH)>(w[offsetof(BSub, XH) / 8]);
  s.Y1 = global_word<decltype(s.Y1)>(w[offsetof(BSub, Y1) / 8]);
  s.RF = global_word<decltype(s.RF)>(w[offsetof(BSub, RF) / 8]);
  s.BB = global_word<decltype(s.BB)>(w[offsetof(BSub, BB) / 8]);
  s.XA = global_word<decltype(s.XA)>(w[offsetof(BSub, XA) / 8]);
  s.BM = global_word<decltype(s.BM)>(w[offsetof(BSub, BM) / 8]);
  s.red0 = global_word<decltype(s.red0)>(w[offsetof(BSub, red0) / 8]);
  s.red1 = global_word<decltype(s.red1)>(w[offsetof(BSub, red1) / 8]);
  s.red2 = global_word<decltype(s.red2)>(w[offsetof(BSub, red2) / 8]);
  return s;
}

// Mutable scalars of one member.
struct BState {
  int32_t mode, k, it, total_inner, status, force;  // force: refine although rel <= tol
  int32_t true_res;  // a certificate missed: every later step certifies first
  double bb, bbar, rel, cert, tol2, rz[2];           // ||b||^2, ||bbar||^2, relres, ...
  double rel_prev;  // the rotated residual before rel (0: none yet)
};

// Batch-wide control words.
constexpr int kBatchMaxGrid = 2048;  // workgroups of a launch (one barrier flag each)

struct BCtl {
  uint32_t fc[4];  // work-item counters of the last four phases
  int32_t err;     // a wait timed out: every workgroup leaves
  int32_t rounds;  // rounds executed by the last launch
  // Real-time clock ticks (100 MHz) spent in each phase, seen by workgroup 0
  // from one barrier exit to the next: [kSlots] phases, then the round setup.
  uint64_t ticks[kSlots + 1];
  // Grid-barrier arrival flags, one 64-byte line per workgroup: the number of
  // barriers the workgroup has reached (the host reads only the words above).
  uint32_t flag[kBatchMaxGrid * 16];
};
constexpr size_t kCtlHostBytes = offsetof(BCtl, flag);

struct BArgs {
  const BSub* sub;
  BState* st;
  BCtl* ctl;
  int32_t count;
  int32_t max_rounds;
  int64_t spin_limit;
};

// ------------------------------------------------------------ small helpers
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic sum over the 256 threads; result in every thread.
__device__ __forceinline__ double block_sum(double v, double* s_red) {
  v = wave_sum(v);
  const int wave = item_tid() >> 6, lane = item_tid() & 63;
  __syncthreads();
  if (lane == 0) s_red[wave] = v;
  __syncthreads();
  if (item_tid() == 0) s_red[4] = ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];
  __syncthreads();
  return s_red[4];
}

// Sum of red[0..cnt) in one fixed order (the same in every caller).
__device__ __forceinline__ double sum_partials(const double* red, int cnt, double* s_red) {
  double v = 0.0;
  for (int i = item_tid(); i < cnt; i += blockDim.x) v += red[i];
  return block_sum(v, s_red);
}

template <typename PT>
__device__ __forceinline__ double part_sum(const void* part, int ks, int64_t n, int ldp, int64_t s,
                                           int c) {
  const PT* p = (const PT*)part;
  double v = 0.0;
  for (int sp = 0; sp < ks; ++sp) v += (double)p[((int64_t)sp * n + s) * ldp + c];
  return v;
}

// Writes the transposed split tile th/tl ([c][row], kRC rows) of rows
// [s0, s0 + rows) into the c-major hi/lo operand of the BF16 product.
__device__ __forceinline__ void store_split(const BSub& S, int64_t s0, int rows, const __bf16* th,
                            const __bf16* tl) {
  __syncthreads();
  for (int e = item_tid(); e < S.r * kRC; e += blockDim.x) {
    const int c = e / kRC, sr = e % kRC;
    if (sr < rows) {
      const int64_t o = (int64_t)c * S.ldl + s0 + sr;
      S.xthi[o] = th[c * kRC + sr];
      S.xtlo[o] = tl[c * kRC + sr];
    }
  }
}

// ------------------------------------------------------------- work counts
__device__ __forceinline__ int item_count(const BSub& S, int mode, int slot) {
  const int fn = S.fn_nrb * S.fn_ks, ft = S.ft_nrb * S.ft_ks, bf = S.bf_nrb * S.bf_ks;
  const int rows = (S.nmulti > 0 && !S.orow) ? S.nrc : 0;  // split segments to add
  switch (mode) {
    case M_SETUP:
      switch (slot) {
        case S_A:
        case S_B:
        case S_CTRL: return 1;
        case S_OBS: return S.ntaskw;
        case S_ROWS: return rows;
        case S_FIN: return S.nrc;
        default: return 0;
      }
    case M_ROT_B:
    case M_ROT_W:
      return slot == S_A ? fn : slot == S_FIN ? S.nrc : slot == S_CTRL ? 1 : 0;
    case M_FINAL:
      return slot == S_A ? ft : slot == S_FIN ? S.nrc : slot == S_CTRL ? 1 : 0;
    case M_RES0:
      return (slot == S_FIN || slot == S_PREC || slot == S_CTRL) ? S.nrc : 0;
    case M_RESC:
      return slot == S_A ? fn : (slot == S_FIN || slot == S_PREC || slot == S_CTRL) ? S.nrc : 0;
    case M_RES:
      switch (slot) {
        case S_A: return ft;
        case S_OBS: return S.ntaskw;
        case S_ROWS: return rows;
        case S_B: return fn;
        case S_UPD: return 0;
        default: return S.nrc;  // FIN, PREC, CTRL
      }
    case M_CERT:
      switch (slot) {
        case S_A:
        case S_B: return fn;
        case S_OBS: return S.ntaskw;
        case S_ROWS: return S.nrc;  // T = B - Yhat1 - lambda W
        case S_FIN: return S.nrc;
        case S_CTRL: return 1;
        default: return 0;
      }
    case M_INNER:
      switch (slot) {
        case S_A:
        case S_B: return bf;
        case S_OBS: return S.ntaskw;
        case S_ROWS: return S.orow ? 0 : S.nrc;  // lane-row gathers split their own rows
        case S_PREC: return 0;                   // fused into S_UPD
        default: return S.nrc;                   // FIN, UPD, CTRL
      }
  }
  return 0;
}

// ---------------------------------------------------------------- products
// Products: BF16 U (D_K p) / U^T Y (inner), FP64 K X, FP64 U^T X (NN on the
// stored U^T), FP64 U X and U (D_K X) (transposed form).
enum : int { G_BF_U = 0, G_BF_UT = 1, G_K = 2, G_UKN = 3, G_UKT = 4 };

template <int NB>
__device__ __forceinline__ void gemm_item_nb(const BSub& S, int kind, const double* X, int64_t i, char* smem) {
  tiles::GArgs g{};
  g.n = S.n;
  g.r = S.r;
  g.ldp = S.ldp;
  g.part = S.part;
  g.X = X;
  g.ldx = S.r;
  if (kind == G_BF_U || kind == G_BF_UT) {
    g.U = kind == G_BF_U ? (const void*)S.ulp : (const void*)S.utlp;
    g.ldu = S.ldl;
    g.kper = S.bf_kper;
    g.xt_hi = S.xthi;
    g.xt_lo = S.xtlo;
    g.ldxt = S.ldl;
    const int64_t bx = i % S.bf_nrb, by = i / S.bf_nrb;
    // the member plans hold U and U^T in the tiled BF16 layout
    if (S.bf_mw == 4)
      tiles::gemm_bf16_tile<NB, 4, 2, true>(g, bx, by * g.kper, min(g.n, (by + 1) * g.kper), by,
                                              (__bf16*)smem, item_tid());
    else
      tiles::gemm_bf16_tile<NB, 2, 2, true>(g, bx, by * g.kper, min(g.n, (by + 1) * g.kper), by,
                                              (__bf16*)smem, item_tid());
  } else if (kind == G_UKT) {
    g.U = S.UK;
    g.ldu = S.ldk;
    g.kper = S.ft_kper;
    const int64_t bx = i % S.ft_nrb, by = i / S.ft_nrb;
    tiles::gemm_k4_tile<double, NB, 2, 4, true, 1>(g, bx, by, (double*)smem, item_tid());
  } else {
    g.U = kind == G_K ? S.K : S.UK;
    g.ldu = S.ldk;
    g.kper = S.fn_kper;
    const int64_t bx = i % S.fn_nrb, by = i / S.fn_nrb;
    if (S.fn_vw == 2)
      tiles::gemm_k4_tile<double, NB, 2, 4, false, 2>(g, bx, by, (double*)smem, item_tid());
    else
      tiles::gemm_k4_tile<double, NB, 2, 4, false, 1>(g, bx, by, (double*)smem, item_tid());
  }
}

__device__ __forceinline__ void gemm_item(const BSub& S, int kind, const double* X, int64_t i, char* smem) {
  switch (S.nb) {
    case 1: gemm_item_nb<1>(S, kind, X, i, smem); break;
    case 2: gemm_item_nb<2>(S, kind, X, i, smem); break;
    default: gemm_item_nb<3>(S, kind, X, i, smem); break;
  }
}

// ------------------------------------------------------ gather-dot-scatter
// Work item i: wave w takes tasks [(4 i + w) kTPW, ...) of the member's list,
// or, for short segments, segments [(4 i + w) kSegPerWave, ...) by lane rows.
// The arithmetic type is that of the partials (FP32 after the BF16 products).
template <int L, int CPL, int FORM, int MODE, typename PT, bool BL>
__device__ __forceinline__ void obs_item_b(const BSub& S, int64_t i, int mode, const PT* Bl) {
  const int64_t wv = 4 * i + (item_tid() >> 6);
  const int64_t t0 = wv * kTPW;
  const int64_t t1 = min((int64_t)S.ntask, t0 + kTPW);
  tiles::TaskView tv{S.tseg, S.tbeg, S.tend, S.tslot, S.tfirst, S.ntask};
  tiles::ObsDev d{};
  d.a.n = S.n;
  d.a.r = S.r;
  d.a.obs_i = S.obs_i;
  d.a.obs_j = S.obs_j;
  d.a.A = S.A;
  d.a.B = S.B;
  d.a.A32 = S.A32;
  d.a.B32 = S.B32;
  d.a.Zhat = nullptr;
  d.a.y = MODE == 1 ? S.y : nullptr;
  d.a.part = MODE == 1 ? nullptr : S.part;
  // split-K depth of the product A that made Xhat
  d.a.ksplit = mode == M_INNER ? S.bf_ks : mode == M_RES ? S.ft_ks : S.fn_ks;
  d.a.ldp = S.ldp;
  d.a.Xhat = nullptr;
  d.a.out = MODE == 1 ? S.BM : S.Y1;
  d.a.tpart = S.tpart;
  d.a.done = nullptr;
  d.I = S.I;
  d.J = S.J;
  if (S.orow) {
    if (mode == M_INNER) {  // Yhat1 only feeds the BF16 U^T Yhat1 product
      d.a.xt_hi = S.xthi;
      d.a.xt_lo = S.xtlo;
      d.a.ldxt = S.ldl;
    }
    constexpr int ROWS = 64 / L;
    for (int k = 0; k < kSegPerWave; k += ROWS) {
      const int64_t s0 = wv * kSegPerWave + k;
      if (s0 >= S.n) break;
      tiles::obs_rows<L, CPL, FORM, MODE, PT, BL, PT>(d, S.obs_ptr, s0,
                                                   (int)min((int64_t)ROWS, S.n - s0),
                                                   item_tid() & 63, Bl);
    }
    return;
  }
  for (int64_t task = t0; task < t1; ++task)
    tiles::obs_task<L, CPL, FORM, MODE, PT, BL, PT>(tv, d, task, item_tid() & 63, Bl);
}

// B (J x r, at most kSmemBytes as FP64; checked at batch creation) goes to LDS
// first, so every observation reads its factor row from LDS instead of L2.
__device__ __forceinline__ const double* factor_b(const BSub& S, double) { return S.B; }
__device__ __forceinline__ const float* factor_b(const BSub& S, float) { return S.B32; }

template <int L, int CPL, int FORM, int MODE, typename PT>
__device__ __forceinline__ void obs_item_c(const BSub& S, int64_t i, int mode, char* smem) {
  const int64_t len = (int64_t)S.J * S.r;
  if (len * (int64_t)sizeof(double) <= kSmemBytes) {
    PT* Bl = (PT*)smem;
    const PT* src = factor_b(S, PT(0));
    for (int64_t e = item_tid(); e < len; e += blockDim.x) Bl[e] = src[e];
    __syncthreads();
    obs_item_b<L, CPL, FORM, MODE, PT, true>(S, i, mode, Bl);
  }
}

template <int L, int CPL>
__device__ __forceinline__ void obs_item_l(const BSub& S, int64_t i, int mode, char* smem) {
  const bool f = mode == M_INNER;  // BF16 products leave float partials
  if (mode == M_SETUP) {            // the observed MTTKRP B (FP64)
    if (S.own)
      obs_item_c<L, CPL, tiles::kOwner, 1, double>(S, i, mode, smem);
    else
      obs_item_c<L, CPL, tiles::kImplicit, 1, double>(S, i, mode, smem);
  } else if (S.own) {
    if (f)
      obs_item_c<L, CPL, tiles::kOwner, 0, float>(S, i, mode, smem);
    else
      obs_item_c<L, CPL, tiles::kOwner, 0, double>(S, i, mode, smem);
  } else {
    if (f)
      obs_item_c<L, CPL, tiles::kImplicit, 0, float>(S, i, mode, smem);
    else
      obs_item_c<L, CPL, tiles::kImplicit, 0, double>(S, i, mode, smem);
  }
}

__device__ __forceinline__ void obs_item(const BSub& S, int64_t i, int mode, char* smem) {
  switch (S.ocls) {
    case 0: obs_item_l<4, 2>(S, i, mode, smem); break;
    case 1: obs_item_l<4, 3>(S, i, mode, smem); break;
    case 2: obs_item_l<4, 5>(S, i, mode, smem); break;
    case 3: obs_item_l<8, 5>(S, i, mode, smem); break;
    default: obs_item_l<16, 4>(S, i, mode, smem); break;
  }
}

// Rows of segments split over several gather tasks: the gather's output row
// (Yhat1, or the MTTKRP B in SETUP) = sum of their partial rows (fixed order).
// INNER also writes the hi/lo BF16 operand of the U^T Yhat1 product for the
// chunk's rows; CERT forms T = B - Yhat1 - lambda W for the K T product.
__device__ __forceinline__ void rows_item(const BSub& S, int64_t i, int mode, char* smem) {
  const bool split = mode == M_INNER;
  const bool cert = mode == M_CERT;
  double* out = mode == M_SETUP ? S.BM : S.Y1;
  const int64_t s0 = i * kRC;
  const int rows = (int)min((int64_t)kRC, S.n - s0);
  const int r = S.r;
  __bf16* th = (__bf16*)smem;
  __bf16* tl = th + kBatchRank * kRC;
  for (int e = item_tid(); e < rows * r; e += blockDim.x) {
    const int sr = e / r, c = e % r;
    const int64_t s = s0 + sr;
    const int32_t m = (S.nmulti > 0 && !S.orow) ? S.rowm[s] : -1;
    double v;
    if (m >= 0) {
      v = 0.0;
      for (int32_t k = S.mptr[m]; k < S.mptr[m + 1]; ++k) v += S.tpart[(int64_t)k * r + c];
      if (!split && !cert) out[s * r + c] = v;
    } else {
      if (!split && !cert) continue;
      v = S.Y1[s * r + c];
    }
    if (cert) {
      const int64_t o = s * r + c;
      S.Q[o] = S.BM[o] - v - S.lam * S.W[o];
    } else if (split) {
      split_pair(v, &th[c * kRC + sr], &tl[c * kRC + sr]);
    }
  }
  if (split) store_split(S, s0, rows, th, tl);
}

// V = (A^T A) had (B^T B) of one member (or the caller's V), one work item.
__device__ __forceinline__ void gram_item(const BSub& S) {
  const int r = S.r;
  for (int e = item_tid(); e < r * r; e += blockDim.x) {
    const int a = e / r, b = e % r;
    if (S.Vin != nullptr) {
      S.V[e] = S.Vin[e];
    } else if (a <= b) {
      const double v = gram_entry(S.A, S.I, S.B, S.J, r, a, b);
      S.V[a * r + b] = v;
      S.V[b * r + a] = v;
    }
  }
}

// ------------------------------------------------------------ vector steps
// Elements per thread whose loads are issued together in the row phases
// (member pointers may alias, so the compiler cannot hoist a later
// element's loads above an earlier element's stores by itself).
constexpr int kEU = 4;

__device__ __forceinline__ void fin_item(const BSub& S, int mode, int64_t i, double* s_red) {
  const int r = S.r;
  const int64_t e0 = i * kRC * r, e1 = min(S.n, (i + 1) * kRC) * r;
  double loc = 0.0;
  if (mode == M_INNER) {  // q = D_K (Y + lambda p) + rho p, every inner iteration
    const int64_t stride = (int64_t)kEU * blockDim.x;
    for (int64_t e = e0 + item_tid(); e < e1; e += stride) {
      double y[kEU], pe[kEU], dk[kEU];
#pragma unroll
      for (int u = 0; u < kEU; ++u) {
        const int64_t ee = e + (int64_t)u * blockDim.x;
        const bool on = ee < e1;
        const int64_t eo = on ? ee : e;
        const int64_t s = eo / r;
        y[u] = part_sum<float>(S.part, S.bf_ks, S.n, S.ldp, s, (int)(eo % r));
        pe[u] = S.P[eo];
        dk[u] = S.dKc[s];
      }
#pragma unroll
      for (int u = 0; u < kEU; ++u) {
        const int64_t ee = e + (int64_t)u * blockDim.x;
        if (ee < e1) {
          const double v = dk[u] * (y[u] + S.lam * pe[u]) + S.rho * pe[u];
          S.Q[ee] = v;
          loc += pe[u] * v;
        }
      }
    }
    const double t = block_sum(loc, s_red);
    if (item_tid() == 0) S.red0[i] = t;
    return;
  }
  for (int64_t e = e0 + item_tid(); e < e1; e += blockDim.x) {
    const int64_t s = e / r;
    const int c = (int)(e % r);
    switch (mode) {
      case M_RES: {  // rbar = bbar - (D_K (Y + lambda xbar) + rho xbar)
        const double y = part_sum<double>(S.part, S.fn_ks, S.n, S.ldp, s, c);
        const double xa = S.XA[e];
        const double q = S.dKc[s] * (y + S.lam * xa) + S.rho * xa;
        const double v = S.BB[e] - q;
        S.R[e] = v;
        S.X[e] = 0.0;
        loc += v * v;
        break;
      }
      case M_RES0: {  // rbar = bbar
        const double v = S.BB[e];
        S.R[e] = v;
        S.X[e] = 0.0;
        loc += v * v;
        break;
      }
      case M_RESC: {  // rbar = U^T rf
        const double v = part_sum<double>(S.part, S.fn_ks, S.n, S.ldp, s, c);
        S.R[e] = v;
        S.X[e] = 0.0;
        loc += v * v;
        break;
      }
      case M_CERT: {  // rf = b - A W = K (B - Yhat1 - lambda W) - rho W
        const double v = part_sum<double>(S.part, S.fn_ks, S.n, S.ldp, s, c) - S.rho * S.W[e];
        S.RF[e] = v;
        loc += v * v;
        break;
      }
      case M_ROT_B: {  // bbar = U^T b = U^T K B = D_K U^T B
        const double v = S.dKc[s] * part_sum<double>(S.part, S.fn_ks, S.n, S.ldp, s, c);
        S.BB[e] = v;
        if (!S.warm) S.XA[e] = 0.0;
        loc += v * v;
        break;
      }
      case M_ROT_W: {  // xbar = U^T W (and D_K xbar, as in accumulate_rows)
        const double v = part_sum<double>(S.part, S.fn_ks, S.n, S.ldp, s, c);
        S.XA[e] = v;
        S.XH[e] = S.dKc[s] * v;
        break;
      }
      case M_FINAL:  // W = U xbar
        S.W[e] = part_sum<double>(S.part, S.ft_ks, S.n, S.ldp, s, c);
        break;
      default: {  // M_SETUP: dK clamped at 0, D (eq. fx), W = 0 unless warm
        const double dk = S.dK[s];
        if (c == 0) S.dKc[s] = fmax(dk, 0.0);
        S.D[e] = precond_entry(dk, S.dV[c], S.gamma, S.lam, S.rho);
        if (!S.warm) S.W[e] = 0.0;
        break;
      }
    }
  }
  double* red = nullptr;
  switch (mode) {
    case M_RES:
    case M_RES0:
    case M_RESC:
    case M_CERT:
    case M_ROT_B: red = S.red1; break;
    default: break;
  }
  if (red != nullptr) {
    const double t = block_sum(loc, s_red);
    if (item_tid() == 0) red[i] = t;
  }
}

// Refinement decision after a rotated residual (RES, RES0), identical in every
// caller: refine on while the residual misses tol (or a certificate asked for
// one more step) and steps remain.
__device__ __forceinline__ bool refine_on(const BSub& S, const BState* st, double* s_red,
                                          double* rel_out) {
  const double rr = sum_partials(S.red1, S.nrc, s_red);
  const double bb = st->bbar;
  const double rel = bb > 0.0 ? sqrt(rr / bb) : (rr > 0.0 ? INFINITY : 0.0);
  *rel_out = rel;
  return isfinite(rel) && (rel > S.tol || st->force) && st->k < S.max_refine;
}

// Inner stopping test of iteration `it`, identical in every caller: p^T A p
// not positive or not finite, ||r||^2 <= tol2, or the iteration cap.
__device__ __forceinline__ bool inner_stop(const BSub& S, const BState* st, int it, double* s_red, bool* finite) {
  const double pq = sum_partials(S.red0, S.nrc, s_red);
  const double rr = sum_partials(S.red1, S.nrc, s_red);
  *finite = isfinite(pq) && isfinite(rr);
  return !(pq > 0.0) || !*finite || rr <= st->tol2 || it + 1 >= S.maxit;
}

// z = ((r U_V) had D) U_V^T for the chunk's rows (eq. fx in the eigenbasis of
// K); partial r^T z.  The two r x r products run on the FP64 4x4x4 MFMA
// (v_mfma_f64_4x4x4_4b; block b = (lane / 4) % 4, A_b[i][k] in lane
// 16 k + 4 b + i, B_b[k][j] in lane 16 k + 4 b + j, D_b[i][j] in lane
// 16 i + 4 b + j): a wave takes 16 rows at a time, the four blocks being four
// groups of 4 rows that share one group of 4 columns; r is padded to a
// multiple of 4 with zeros (at most kBatchRank).  With UPD (inner iteration)
// the rows are first updated, x += alpha p and r -= alpha q, while they are
// staged, and r^T r is summed as well: update and preconditioner share one
// pass over the rows.
constexpr int kPC4 = kBatchRank / 4;      // column groups at most
constexpr int kPLT = kBatchRank + 1;      // row stride of a wave's 16-row tile
static_assert((kBatchRank * kBatchRank + 4 * 16 * kPLT) * 8 <= kSmemBytes, "precond LDS");

template <bool UPD>
__device__ __forceinline__ void prec_rows(const BSub& S, int64_t i, char* smem, double* s_red,
                                          double alpha = 0.0) {
  const int r = S.r;
  const int nc4 = (r + 3) / 4, rp = 4 * nc4;
  double* uv = (double*)smem;  // rp x rp
  const int wave = item_tid() >> 6, lane = item_tid() & 63;
  double* wt = uv + kBatchRank * kBatchRank + wave * (16 * kPLT);
  for (int e = item_tid(); e < rp * rp; e += blockDim.x) {
    const int j = e / rp, c = e % rp;
    uv[e] = (j < r && c < r) ? S.UV[j * r + c] : 0.0;
  }
  __syncthreads();
  const int li = lane & 15, kk = lane >> 4, jj = lane & 3;
  const int orow = 4 * ((lane >> 2) & 3) + kk;
  const int64_t s0 = i * kRC, s1 = min(S.n, s0 + kRC);
  double loc = 0.0, loc_rr = 0.0;
  for (int64_t row0 = s0 + 16 * wave; row0 < s1; row0 += 64) {
    for (int e = lane; e < 16 * rp; e += 64) {
      const int ri = e / rp, c = e % rp;
      const int64_t s = row0 + ri;
      double v = 0.0;
      if (s < s1 && c < r) {
        const int64_t o = s * r + c;
        if (UPD) {
          S.X[o] += alpha * S.P[o];
          v = S.R[o] - alpha * S.Q[o];
          S.R[o] = v;
          loc_rr += v * v;
        } else {
          v = S.R[o];
        }
      }
      wt[ri * kPLT + c] = v;
    }
    __builtin_amdgcn_wave_barrier();
    double acc[kPC4];
#pragma unroll
    for (int c = 0; c < kPC4; ++c) acc[c] = 0.0;
    for (int ks = 0; ks < nc4; ++ks) {  // (r U_V)
      const double a = wt[li * kPLT + 4 * ks + kk];
#pragma unroll
      for (int c = 0; c < kPC4; ++c)
        if (c < nc4)
          acc[c] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, uv[(4 * ks + kk) * rp + 4 * c + jj],
                                                      acc[c], 0, 0, 0);
    }
    const int64_t s = row0 + orow;
    const bool ron = s < s1;
    double tv[kPC4];  // r at this lane's output elements, for r^T z
#pragma unroll
    for (int c = 0; c < kPC4; ++c) {
      const int col = 4 * c + jj;
      tv[c] = c < nc4 ? wt[orow * kPLT + col] : 0.0;
      if (c < nc4) acc[c] *= (ron && col < r) ? S.D[s * r + col] : 0.0;
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = 0; c < kPC4; ++c)
      if (c < nc4) wt[orow * kPLT + 4 * c + jj] = acc[c];
    __builtin_amdgcn_wave_barrier();
    double z[kPC4];
#pragma unroll
    for (int c = 0; c < kPC4; ++c) z[c] = 0.0;
    for (int ks = 0; ks < nc4; ++ks) {  // (. U_V^T)
      const double a = wt[li * kPLT + 4 * ks + kk];
#pragma unroll
      for (int c = 0; c < kPC4; ++c)
        if (c < nc4)
          z[c] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, uv[(4 * c + jj) * rp + 4 * ks + kk], z[c],
                                                    0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < kPC4; ++c) {
      const int col = 4 * c + jj;
      if (c < nc4 && ron && col < r) {
        S.Z[s * r + col] = z[c];
        loc += tv[c] * z[c];
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (UPD) {
    const double rr = block_sum(loc_rr, s_red);
    if (item_tid() == 0) S.red1[i] = rr;
  }
  const double tot = block_sum(loc, s_red);
  if (item_tid() == 0) S.red2[i] = tot;
}

// Inner iteration, after the FIN phase: alpha = r^T z / p^T q, then the
// fused row update and preconditioner apply (partials r^T r -> red1, r^T z ->
// red2).  A step length that is not positive and finite leaves the rows as
// they are; the control phase then ends the inner solve.
__device__ __forceinline__ void upd_item(const BSub& S, const BState* st, int it, int64_t i,
                                         char* smem, double* s_red) {
  const double pq = sum_partials(S.red0, S.nrc, s_red);
  const double rz = st->rz[it & 1];
  if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rz)) return;
  prec_rows<true>(S, i, smem, s_red, rz / pq);
}

// p = z + beta p for the chunk's rows and the hi/lo split of D_K p.
__device__ __forceinline__ void p_rows(const BSub& S, int64_t i, double beta, char* smem) {
  const int r = S.r;
  const int64_t s0 = i * kRC;
  const int rows = (int)min((int64_t)kRC, S.n - s0);
  __bf16* th = (__bf16*)smem;
  __bf16* tl = th + kBatchRank * kRC;
  const int ne = rows * r;
  for (int e = item_tid(); e < ne; e += kEU * blockDim.x) {
    double z[kEU], pp[kEU], dk[kEU];
#pragma unroll
    for (int u = 0; u < kEU; ++u) {
      const int ee = min(e + u * (int)blockDim.x, ne - 1);
      const int64_t s = s0 + ee / r, o = s0 * r + ee;
      z[u] = S.Z[o];
      pp[u] = S.P[o];
      dk[u] = S.dKc[s];
    }
#pragma unroll
    for (int u = 0; u < kEU; ++u) {
      const int ee = e + u * (int)blockDim.x;
      if (ee < ne) {
        const int sr = ee / r, c = ee % r;
        const double pv = z[u] + beta * pp[u];
        S.P[s0 * r + ee] = pv;
        split_pair(dk[u] * pv, &th[c * kRC + sr], &tl[c * kRC + sr]);
      }
    }
  }
  store_split(S, s0, rows, th, tl);
}

__device__ __forceinline__ void finish_member(BState* st, int32_t mode, int32_t status) {
  st->mode = mode;
  if (mode == M_DONE) st->status = status;
}

// xbar += dbar for the chunk's rows (the inner solve's correction), and
// D_K xbar into XH for the rotated residual's product U (D_K xbar) (scaled
// here rather than while the product stages X, where waiting for the scale
// loads would hold back its prefetch of U).
__device__ __forceinline__ void accumulate_rows(const BSub& S, int64_t i) {
  const int r = S.r;
  const int64_t e0 = i * kRC * r, e1 = min(S.n, (i + 1) * kRC) * r;
  for (int64_t e = e0 + item_tid(); e < e1; e += blockDim.x) {
    const double v = S.XA[e] + S.X[e];
    S.XA[e] = v;
    S.XH[e] = S.dKc[e / r] * v;
  }
}

__device__ __forceinline__ void ctrl_item(const BSub& S, BState* st, int mode, int it, int64_t i,
                                          char* smem, double* s_red) {
  const bool lead = i == 0 && item_tid() == 0;
  switch (mode) {
    case M_INNER: {
      bool finite = true;
      bool stop = inner_stop(S, st, it, s_red, &finite);
      double rz_new = 0.0;
      if (!stop) {
        rz_new = sum_partials(S.red2, S.nrc, s_red);
        if (!(rz_new > 0.0) || !isfinite(rz_new)) {
          stop = true;
          finite = isfinite(rz_new);
        }
      }
      if (stop) {
        if (finite) accumulate_rows(S, i);
        if (lead) {
          st->total_inner += it + 1;
          st->k += 1;
          st->force = 0;
          // As in the single solve: when the last step's contraction predicts
          // convergence, W = U xbar is certified at once (M_FINAL, M_CERT)
          // instead of forming the rotated residual first (M_RES).
          const bool predict = st->true_res || (st->rel_prev > 0.0 &&
                               st->rel * (st->rel / st->rel_prev) <= kCertifyFirst * S.tol);
          if (!finite)
            finish_member(st, M_DONE, CPHIFI_NUMERIC);
          else
            finish_member(st, predict ? M_FINAL : M_RES, 0);
        }
        return;
      }
      p_rows(S, i, rz_new / st->rz[it & 1], smem);
      if (lead) {
        st->rz[(it + 1) & 1] = rz_new;
        st->it = it + 1;
      }
      return;
    }
    case M_RES:
    case M_RES0:
    case M_RESC: {
      double rel = 0.0;
      const bool on = refine_on(S, st, s_red, &rel);
      double rz0 = 0.0;
      if (on) {
        rz0 = sum_partials(S.red2, S.nrc, s_red);
        if (rz0 > 0.0 && isfinite(rz0)) p_rows(S, i, 0.0, smem);
      }
      if (lead) {
        st->rel_prev = st->rel;
        st->rel = rel;
        if (!isfinite(rel) || (on && !isfinite(rz0))) {
          finish_member(st, M_DONE, CPHIFI_NUMERIC);
        } else if (on && rz0 > 0.0) {
          const double rr = rel * rel * st->bbar;
          const bool loose = S.adapt && rel * kInnerLoose > S.tol;
          st->tol2 = (loose ? fmax(S.inner_tol2, kInnerLoose * kInnerLoose) : S.inner_tol2) * rr;
          st->rz[0] = rz0;
          st->it = 0;
          finish_member(st, M_INNER, 0);
        } else if (on) {
          finish_member(st, M_DONE, CPHIFI_BREAKDOWN);  // r^T M^{-1} r <= 0
        } else {
          finish_member(st, M_FINAL, 0);
        }
      }
      return;
    }
    case M_CERT: {
      const double rr = sum_partials(S.red1, S.nrc, s_red);
      if (lead) {
        const double bb = st->bb;
        const double cert = bb > 0.0 ? sqrt(rr / bb) : (rr > 0.0 ? INFINITY : 0.0);
        st->cert = cert;
        if (!isfinite(cert)) {
          finish_member(st, M_DONE, CPHIFI_NUMERIC);
        } else if (cert <= S.tol) {
          if (!(st->rel <= S.tol)) st->rel = cert;  // certified without a rotated residual
          finish_member(st, M_DONE, CPHIFI_OK);
        } else if (st->k >= S.max_refine) {
          finish_member(st, M_DONE, CPHIFI_NOT_CONVERGED);
        } else {
          // the certificate missed: its residual, rotated, is the next right-hand
          // side, and so for every later step (the rotated residual disagrees
          // with the original system's)
          st->force = 1;
          st->true_res = 1;
          finish_member(st, M_RESC, 0);
        }
      }
      return;
    }
    case M_ROT_B: {  // ||b||^2 = ||bbar||^2 (U_K orthogonal)
      const double bb = sum_partials(S.red1, S.nrc, s_red);
      if (lead) {
        st->bbar = bb;
        st->bb = bb;
        if (!isfinite(bb)) {
          finish_member(st, M_DONE, CPHIFI_NUMERIC);
        } else if (bb == 0.0 && !S.warm) {
          st->rel = st->cert = 0.0;  // b = 0: w = 0 is exact
          finish_member(st, M_DONE, CPHIFI_OK);
        } else {
          finish_member(st, S.warm ? M_ROT_W : M_RES0, 0);
        }
      }
      return;
    }
    case M_ROT_W:
      if (lead) finish_member(st, M_RES, 0);
      return;
    case M_FINAL:
      if (lead) finish_member(st, M_CERT, 0);
      return;
    default:  // M_SETUP
      if (lead) finish_member(st, M_ROT_B, 0);
      return;
  }
}

__device__ __forceinline__ void run_item(const BSub& S, BState* st, int slot, int mode, int it,
                                         int64_t i, char* smem, double* s_red) {
  switch (slot) {
    case S_A:
      switch (mode) {
        case M_INNER: gemm_item(S, G_BF_U, nullptr, i, smem); break;
        case M_RES: gemm_item(S, G_UKT, S.XH, i, smem); break;  // U (D_K xbar)
        case M_CERT: gemm_item(S, G_K, S.W, i, smem); break;
        case M_ROT_B: gemm_item(S, G_UKN, S.BM, i, smem); break;
        case M_SETUP: gram_item(S); break;
        case M_ROT_W: gemm_item(S, G_UKN, S.W, i, smem); break;
        case M_FINAL: gemm_item(S, G_UKT, S.XA, i, smem); break;
        case M_RESC: gemm_item(S, G_UKN, S.RF, i, smem); break;
      }
      break;
    case S_OBS: obs_item(S, i, mode, smem); break;
    case S_ROWS: rows_item(S, i, mode, smem); break;
    case S_B:
      switch (mode) {
        case M_INNER: gemm_item(S, G_BF_UT, nullptr, i, smem); break;
        case M_RES: gemm_item(S, G_UKN, S.Y1, i, smem); break;
        case M_SETUP:  // eq. eigV
          jacobi_sym<kBatchRank>(S.V, S.r, S.UV, S.dV, *(JacobiLds<kBatchRank>*)smem,
                                 item_tid());
          break;
        default: gemm_item(S, G_K, S.Q, i, smem); break;  // M_CERT: K T
      }
      break;
    case S_FIN: fin_item(S, mode, i, s_red); break;
    case S_UPD: upd_item(S, st, it, i, smem, s_red); break;
    case S_PREC: {  // M_RES, M_RES0, M_RESC (the inner iteration's is fused into S_UPD)
      double rel = 0.0;
      if (refine_on(S, st, s_red, &rel)) prec_rows<false>(S, i, smem, s_red);
      break;
    }
    default: ctrl_item(S, st, mode, it, i, smem, s_red); break;
  }
}

// Bounded grid barrier on per-workgroup arrival flags: thread 0 releases the
// workgroup's writes and stores the barrier count in its own line; the first
// wave polls every workgroup's flag (a few per lane) until all have reached
// it, then thread 0 acquires the others' writes.  No shared counter, so the
// arrivals do not queue on one atomic.  Returns false when a wait timed out
// (here or in any other workgroup); the caller then leaves the kernel.
__device__ __forceinline__ bool grid_sync(BCtl* ctl, uint32_t epoch, int64_t spin_limit, int* s_ok) {
  __syncthreads();
  if (threadIdx.x < 64) {
    if (threadIdx.x == 0) {
      // release this workgroup's writes device-wide (a release fence: the L2
      // write-back only, no invalidation)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&ctl->flag[blockIdx.x * 16], epoch, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    int ok = 1;
    for (int64_t spin = 0;; ++spin) {
      bool mine = true;
      for (int g = threadIdx.x; g < (int)gridDim.x; g += 64)
        mine = mine && __hip_atomic_load(&ctl->flag[g * 16], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) >= epoch;
      if (__all(mine)) break;
      if ((spin & 63) == 63 &&
          __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        ok = 0;
        break;
      }
      if (spin >= spin_limit) {
        if (threadIdx.x == 0)
          __hip_atomic_store(&ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (threadIdx.x == 0) {
      // acquire the other workgroups' writes (an acquire fence: invalidation only)
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      *s_ok = ok;
    }
  }
  __syncthreads();
  return *s_ok != 0;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void batch_kernel(
    BArgs a) {
  __shared__ __attribute__((aligned(16))) char smem[kSmemBytes];
  __shared__ int s_pref[kSlots][kMaxBatch + 1];
  __shared__ int s_mode[kMaxBatch];
  __shared__ int s_it[kMaxBatch];
  __shared__ int s_wtot[kSlots][4];
  __shared__ double s_red[8];
  __shared__ int s_item;
  __shared__ int s_ok;
  __shared__ uint64_t s_tick[kSlots + 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int count = a.count;
  const bool clock0 = blockIdx.x == 0 && tid == 0;  // keeps the phase clock
  if (tid <= kSlots) s_tick[tid] = 0;
  uint64_t t_last = clock0 ? __builtin_amdgcn_s_memrealtime() : 0;
  uint32_t nbar = 0;  // barriers passed
  uint32_t pi = 0;    // phases run
  int round = 0;
  for (; round < a.max_rounds; ++round) {
    if (__hip_atomic_load(&a.ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    // Snapshot of the members' modes and the item prefix sums of each phase.
    int cnt[kSlots];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) cnt[s] = 0;
    if (tid < count) {
      const int m = a.st[tid].mode;
      s_mode[tid] = m;
      s_it[tid] = a.st[tid].it;
      if (m != M_DONE) {
        const BSub& S = a.sub[tid];
#pragma unroll
        for (int s = 0; s < kSlots; ++s) cnt[s] = item_count(S, m, s);
      }
    }
    int incl[kSlots];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      int v = cnt[s];
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
      }
      incl[s] = v;
      if (lane == 63) s_wtot[s][wave] = v;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      int base = 0;
      for (int w = 0; w < wave; ++w) base += s_wtot[s][w];
      if (tid < count) s_pref[s][tid] = base + incl[s] - cnt[s];
      if (tid == count - 1) s_pref[s][count] = base + incl[s];
    }
    __syncthreads();
    if (clock0) {
      const uint64_t t = __builtin_amdgcn_s_memrealtime();
      s_tick[kSlots] += t - t_last;
      t_last = t;
    }
    if (s_pref[S_CTRL][count] == 0) break;  // every member is done

    for (int slot = 0; slot < kSlots; ++slot) {
      const int total = s_pref[slot][count];
      if (total == 0) continue;
      if (blockIdx.x == 0 && tid == 0)
        __hip_atomic_store(&a.ctl->fc[(pi + 2) & 3], 0u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      // Products and the gather take their items from a counter (their costs
      // differ by member); the row steps' items are uniform and dealt
      // round-robin, with no atomic per item.
      const bool dyn = slot == S_A || slot == S_B || slot == S_OBS;
      int item = blockIdx.x;
      while (item < total) {
        // member b: last one whose range starts at or before the item
        int lo = 0, hi = count - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_pref[slot][mid] <= item)
            lo = mid;
          else
            hi = mid - 1;
        }
        // uniform member index
        const int b = __builtin_amdgcn_readfirstlane(lo);
        const BSub S = load_sub(a.sub, b);
        run_item(S, &a.st[b], slot, __builtin_amdgcn_readfirstlane(s_mode[b]),
                 __builtin_amdgcn_readfirstlane(s_it[b]),
                 __builtin_amdgcn_readfirstlane(item - s_pref[slot][b]), smem, s_red);
        if (dyn) {
          __syncthreads();
          if (tid == 0)
            s_item = (int)gridDim.x + (int)__hip_atomic_fetch_add(&a.ctl->fc[pi & 3], 1u,
                                                                   __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT);
          __syncthreads();
          item = s_item;
        } else {
          item += (int)gridDim.x;
        }
      }
      ++pi;
      ++nbar;
      if (!grid_sync(a.ctl, nbar, a.spin_limit, &s_ok)) return;
      if (clock0) {
        const uint64_t t = __builtin_amdgcn_s_memrealtime();
        s_tick[slot] += t - t_last;
        t_last = t;
      }
    }
  }
  if (clock0) {
    a.ctl->rounds = round;
    for (int j = 0; j <= kSlots; ++j) a.ctl->ticks[j] = s_tick[j];
  }
}

// Start state of a launch: control words cleared, every member at SETUP.
__global__ void batch_reset_kernel(BArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int j = 0; j < 4; ++j) a.ctl->fc[j] = 0;
    a.ctl->err = 0;
    a.ctl->rounds = 0;
    for (int j = 0; j <= kSlots; ++j) a.ctl->ticks[j] = 0;
  }
  for (int g = threadIdx.x; g < kBatchMaxGrid; g += blockDim.x) a.ctl->flag[g * 16] = 0u;
  for (int b = threadIdx.x; b < a.count; b += blockDim.x) {
    BState s{};
    s.mode = M_SETUP;
    s.status = CPHIFI_NOT_CONVERGED;
    a.st[b] = s;
  }
}

}  // namespace

// ------------------------------------------------------------------- host
struct cphifi_batch {
  int count = 0;
  hipStream_t st = nullptr;
  std::vector<cphifi_plan*> plans;
  BSub* d_sub = nullptr;
  BState* d_st = nullptr;
  BCtl* d_ctl = nullptr;
  BSub* h_sub = nullptr;    // pinned mirrors
  BState* h_st = nullptr;
  BCtl* h_ctl = nullptr;
  int grid = 0;
  int max_rounds = 0;
  int64_t spin_limit = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

struct BatchLayout {
  size_t sub, st, ctl, head;
  std::vector<size_t> member, member_bytes;
  size_t total;
};

// A member's plan: the batched kernel runs its own product tiles on U_K as
// given, so the plan needs no transposed copy of U_K.
cphifi_ui_desc member_desc(const cphifi_ui_desc& d) {
  cphifi_ui_desc m = d;
  // the batched kernel runs its own refinement: no copies for the single-solve path
  m.flags |= CPHIFI_FLAG_NO_UKT_COPY | CPHIFI_FLAG_FP64_RESIDUALS;
  return m;
}

int batch_layout(int count, const cphifi_ui_desc* descs, BatchLayout* L) {
  if (count < 1 || count > kMaxBatch) {
    set_error("batch count %d outside 1..%d", count, kMaxBatch);
    return CPHIFI_INVALID_ARG;
  }
  if (descs == nullptr) {
    set_error("descs is NULL");
    return CPHIFI_INVALID_ARG;
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align_up(off, kAlign);
    const size_t o = off;
    off += std::max<size_t>(bytes, 1);
    return o;
  };
  L->sub = take(sizeof(BSub) * count);
  L->st = take(sizeof(BState) * count);
  L->ctl = take(sizeof(BCtl));
  L->head = align_up(off, kAlign);
  L->member.resize(count);
  L->member_bytes.resize(count);
  for (int b = 0; b < count; ++b) {
    size_t bytes = 0;
    const cphifi_ui_desc d = member_desc(descs[b]);
    const int rc = cphifi_ui_workspace_bytes(&d, &bytes);
    if (rc != CPHIFI_OK) return rc;
    L->member[b] = take(bytes);
    L->member_bytes[b] = bytes;
  }
  L->total = align_up(off, kAlign);
  return CPHIFI_OK;
}

// Tile of one product kind for the batch: the tile table (when it covers
// (n, r)) gives the split-K depth and, for BF16, the rows per wave; else the
// k-range of an item is about 2048.
void batch_tile(const char* table, Elt elt, bool trans, int64_t n, int r, int* mw, int* ks,
                int64_t* kper, int* nrb) {
  int tmw = 0, ts = 0, tks = 0;
  const bool hit = gemm_table_lookup(table, elt, trans, n, r, &tmw, &ts, &tks);
  const int nb = (r + 15) / 16;
  int64_t bk;
  if (elt == Elt::BF16) {
    *mw = (hit && tmw < 4) ? 2 : 4;
    bk = gemm_bk(Elt::BF16, 2);
  } else if (trans) {
    *mw = 2;
    bk = gemm_bk(Elt::F64, 4);
  } else {
    *mw = 2;
    bk = gemm_bk(Elt::F64, 4);
  }
  int64_t want = hit && tks > 0 ? tks : (n + 2047) / 2048;
  want = std::max<int64_t>(1, std::min<int64_t>(want, kMaxSplit));
  int64_t kp = (n + want - 1) / want;
  kp = (kp + bk - 1) / bk * bk;
  *kper = kp;
  *ks = (int)((n + kp - 1) / kp);
  const int64_t rows = tiles::tile_rows(*mw);
  *nrb = (int)((n + rows - 1) / rows);
}

int obs_class(int r) {
  if (r <= 8) return 0;
  if (r <= 12) return 1;
  if (r <= 20) return 2;
  if (r <= 40) return 3;
  return 4;
}

void destroy_batch(cphifi_batch* bt) {
  if (bt == nullptr) return;
  for (cphifi_plan* p : bt->plans)
    if (p) (void)cphifi_ui_plan_destroy(p);
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  if (bt->h_sub) (void)hipHostFree(bt->h_sub);
  if (bt->h_st) (void)hipHostFree(bt->h_st);
  if (bt->h_ctl) (void)hipHostFree(bt->h_ctl);
  delete bt;
}

BArgs make_args(const cphifi_batch* bt) {
  BArgs a{};
  a.sub = bt->d_sub;
  a.st = bt->d_st;
  a.ctl = bt->d_ctl;
  a.count = bt->count;
  a.max_rounds = bt->max_rounds;
  a.spin_limit = bt->spin_limit;
  return a;
}

// The graph of one batched solve: the reset kernel, then the persistent
// kernel.  It is captured on a private stream (the caller's may be the null
// stream, which cannot be captured) and launched on the batch's stream.
int build_graph(cphifi_batch* bt) {
  if (bt->exec != nullptr) return CPHIFI_OK;
  const BArgs a = make_args(bt);
  hipStream_t cs = nullptr;
  CPHIFI_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(256), 0, cs, a);
    hipLaunchKernelGGL(batch_kernel, dim3(bt->grid), dim3(256), 0, cs, a);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess && g == nullptr) e = hipErrorInvalidValue;
    if (e == hipSuccess) {
      bt->graph = g;
      e = hipGraphInstantiate(&bt->exec, g, nullptr, nullptr, 0);
    }
  }
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    bt->exec = nullptr;
    set_error("graph capture of the batched solve failed: %s", hipGetErrorString(e));
    return CPHIFI_HIP_ERROR;
  }
  return CPHIFI_OK;
}

}  // namespace

extern "C" {

int cphifi_batch_workspace_bytes(int count, const cphifi_ui_desc* descs, size_t* bytes) {
  clear_error();
  if (bytes == nullptr) {
    set_error("bytes is NULL");
    return CPHIFI_INVALID_ARG;
  }
  BatchLayout L;
  const int rc = batch_layout(count, descs, &L);
  if (rc != CPHIFI_OK) return rc;
  *bytes = L.total;
  return CPHIFI_OK;
}

int cphifi_batch_create(cphifi_batch** out, int count, const cphifi_ui_desc* descs,
                        const cphifi_ui_inputs* inputs, void* workspace, size_t workspace_bytes,
                        void* stream, const char* tile_table) {
  clear_error();
  if (out == nullptr || inputs == nullptr) {
    set_error("out / inputs is NULL");
    return CPHIFI_INVALID_ARG;
  }
  *out = nullptr;
  BatchLayout L;
  TRY_RC(batch_layout(count, descs, &L));
  if (workspace == nullptr || workspace_bytes < L.total ||
      (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) {
    set_error("workspace must be >= %zu bytes and 256-byte aligned (got %zu)", L.total,
              workspace_bytes);
    return CPHIFI_INVALID_ARG;
  }
  for (int b = 0; b < count; ++b) {
    const cphifi_ui_desc& d = descs[b];
    if (d.precision != CPHIFI_MIXED_BF16) {
      set_error("member %d: the batched solver runs the MIXED_BF16 form only", b);
      return CPHIFI_UNSUPPORTED;
    }
    if (inputs[b].Zhat != nullptr) {
      set_error("member %d: the batched solver takes the implicit (A, B) form only", b);
      return CPHIFI_UNSUPPORTED;
    }
    if (d.flags & (CPHIFI_FLAG_TOEPLITZ_K | CPHIFI_FLAG_FIBER_COLLAPSE)) {
      set_error("member %d: the batched solver has no structured (Toeplitz / fiber) forms", b);
      return CPHIFI_UNSUPPORTED;
    }
    if (d.r > kBatchRank) {
      set_error("member %d: r = %lld exceeds the batched limit %d", b, (long long)d.r,
                kBatchRank);
      return CPHIFI_UNSUPPORTED;
    }
    if (d.n > kMaxN) {
      set_error("member %d: n = %lld exceeds the batched limit %lld", b, (long long)d.n,
                (long long)kMaxN);
      return CPHIFI_UNSUPPORTED;
    }
    if ((int64_t)d.J * d.r * (int64_t)sizeof(double) > kSmemBytes) {
      set_error("member %d: J r = %lld exceeds the batched gather's LDS copy of B (%d)", b,
                (long long)d.J * d.r, kSmemBytes / (int)sizeof(double));
      return CPHIFI_UNSUPPORTED;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  cphifi_batch* bt = new cphifi_batch();
  bt->count = count;
  bt->st = st;
  bt->plans.assign(count, nullptr);
  char* ws = (char*)workspace;
  bt->d_sub = (BSub*)(ws + L.sub);
  bt->d_st = (BState*)(ws + L.st);
  bt->d_ctl = (BCtl*)(ws + L.ctl);
  auto fail = [&](int code) {
    destroy_batch(bt);
    return code;
  };
  if (hipHostMalloc((void**)&bt->h_sub, sizeof(BSub) * count, hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&bt->h_st, sizeof(BState) * count, hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&bt->h_ctl, sizeof(BCtl), hipHostMallocDefault) != hipSuccess) {
    set_error("hipHostMalloc of the batch mirrors failed");
    return fail(CPHIFI_HIP_ERROR);
  }
  std::memset(bt->h_sub, 0, sizeof(BSub) * count);
  int num_cu = 256;
  {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cu > 0)
      num_cu = cu;
  }
  int max_rounds = 0;
  for (int b = 0; b < count; ++b) {
    const cphifi_ui_desc d = member_desc(descs[b]);
    const cphifi_ui_inputs& in = inputs[b];
    int rc = cphifi_ui_plan_create(&bt->plans[b], &d, &in, ws + L.member[b], L.member_bytes[b],
                                   stream);
    if (rc == CPHIFI_OK) rc = cphifi_ui_setup(bt->plans[b]);
    if (rc != CPHIFI_OK) {
      const std::string msg = cphifi_last_error();
      destroy_batch(bt);
      set_error("member %d: %s", b, msg.c_str());
      return rc;
    }
    cphifi_plan* p = bt->plans[b];
    if (p->a32 == nullptr || p->b32 == nullptr) {  // made by every MIXED_BF16 (A, B) plan
      set_error("member %d: no FP32 copies of A and B", b);
      return fail(CPHIFI_UNSUPPORTED);
    }
    // zero padding rows / columns of the BF16 split operand once
    const size_t xt_bytes = sizeof(__bf16) * (size_t)p->ldp * p->L.ldl;
    if (hipMemsetAsync(p->xthi, 0, xt_bytes, st) != hipSuccess ||
        hipMemsetAsync(p->xtlo, 0, xt_bytes, st) != hipSuccess) {
      set_error("clearing the split operand failed");
      return fail(CPHIFI_HIP_ERROR);
    }
    BSub& S = bt->h_sub[b];
    S.n = p->n;
    S.ldk = p->ldk;
    S.ldl = p->L.ldl;
    S.I = p->I;
    S.J = p->J;
    S.r = (int32_t)p->r;
    S.ldp = p->ldp;
    S.nb = (int32_t)((p->r + 15) / 16);
    S.ocls = obs_class((int)p->r);
    S.nrc = (int32_t)((p->n + kRC - 1) / kRC);
    S.ntask = p->tasks.ntask;
    S.orow = p->tasks.rows ? 1 : 0;
    S.own = p->tasks.owner ? 1 : 0;
    S.ntaskw = S.orow ? (int32_t)((p->n + 4 * kSegPerWave - 1) / (4 * kSegPerWave))
                      : (p->tasks.ntask + 4 * kTPW - 1) / (4 * kTPW);
    S.obs_ptr = in.obs_ptr;
    S.nmulti = p->tasks.nmulti;
    S.K = in.K;
    S.UK = in.UK;
    S.dK = in.dK;
    S.Vin = in.V;
    S.obs_i = in.obs_i;
    S.obs_j = in.obs_j;
    S.A = in.A;
    S.B = in.B;
    S.A32 = p->a32;
    S.B32 = p->b32;
    S.tseg = p->tasks.seg;
    S.tbeg = p->tasks.beg;
    S.tend = p->tasks.end;
    S.tslot = p->tasks.slot;
    S.tfirst = p->tasks.first;
    S.mptr = p->tasks.mptr;
    S.rowm = p->rowm;
    S.part = p->part;
    S.tpart = p->tpart;
    S.V = p->V;
    S.UV = p->UV;
    S.dV = p->dV;
    S.D = p->D;
    S.dKc = p->dKc;
    S.ulp = (const __bf16*)p->ulp;
    S.utlp = (const __bf16*)p->utlp;
    S.xthi = p->xthi;
    S.xtlo = p->xtlo;
    S.X = p->vec[V_XB];
    S.R = p->vec[V_R2];
    S.Z = p->vec[V_Z2];
    S.P = p->vec[V_P2];
    S.Q = p->vec[V_Q2];
    S.XH = p->vec[V_XHAT];
    S.Y1 = p->vec[V_Y1];
    S.RF = p->vec[V_RF];
    S.BB = p->vec[V_T2];
    S.XA = p->vec[V_TMP];
    S.BM = p->vec[V_B];
    S.red0 = p->red[0];
    S.red1 = p->red[1];
    S.red2 = p->red[2];
    int mw = 0;
    batch_tile(tile_table, Elt::BF16, false, p->n, (int)p->r, &S.bf_mw, &S.bf_ks, &S.bf_kper,
               &S.bf_nrb);
    batch_tile(tile_table, Elt::F64, false, p->n, (int)p->r, &mw, &S.fn_ks, &S.fn_kper,
               &S.fn_nrb);
    batch_tile(tile_table, Elt::F64, true, p->n, (int)p->r, &S.ft_mw, &S.ft_ks, &S.ft_kper,
               &S.ft_nrb);
    const bool aligned = (reinterpret_cast<uintptr_t>(in.K) % 16) == 0 &&
                         (reinterpret_cast<uintptr_t>(in.UK) % 16) == 0;
    S.fn_vw = (p->ldk % 2 == 0 && aligned) ? 2 : 1;
    S.lam = d.lambda;
    S.rho = d.rho;
    S.gamma = p->gamma;
    S.tol = d.tol;
    const double itol = d.inner_tol > 0.0 ? d.inner_tol : kInnerTol;
    S.inner_tol2 = itol * itol;
    S.adapt = d.inner_tol > 0.0 ? 0 : 1;
    S.maxit = eff_maxit(d);
    S.max_refine = d.max_refine > 0 ? d.max_refine : 30;
    S.warm = (d.flags & CPHIFI_FLAG_WARM_START) ? 1 : 0;
    max_rounds = std::max(max_rounds, (S.max_refine + 1) * (S.maxit + 3) + 8);
  }
  bt->max_rounds = max_rounds;
  {
    const char* e = std::getenv("CPHIFI_BATCH_SPIN_LIMIT");
    bt->spin_limit = (e != nullptr && std::atoll(e) > 0) ? std::atoll(e) : (1LL << 23);
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel, 256, 0) !=
          hipSuccess ||
      per_cu < 1) {
    set_error("occupancy query of the batched kernel failed");
    return fail(CPHIFI_HIP_ERROR);
  }
  bt->grid = std::min(num_cu * per_cu, kBatchMaxGrid);
  {
    const char* e = std::getenv("CPHIFI_BATCH_GRID");
    if (e != nullptr && std::atoi(e) > 0) bt->grid = std::min(bt->grid, std::atoi(e));
  }
  if (hipMemcpyAsync(bt->d_sub, bt->h_sub, sizeof(BSub) * count, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    set_error("uploading the batch description failed");
    return fail(CPHIFI_HIP_ERROR);
  }
  *out = bt;
  return CPHIFI_OK;
}

int cphifi_batch_plan(cphifi_batch* bt, int member, cphifi_plan** out) {
  clear_error();
  if (bt == nullptr || out == nullptr || member < 0 || member >= bt->count) {
    set_error("bad batch, member or out");
    return CPHIFI_INVALID_ARG;
  }
  *out = bt->plans[member];
  return CPHIFI_OK;
}

int cphifi_batch_rhs(cphifi_batch* bt, const double* const* y, double* const* b) {
  clear_error();
  if (bt == nullptr || y == nullptr || b == nullptr) {
    set_error("bad batch, y or b");
    return CPHIFI_INVALID_ARG;
  }
  for (int i = 0; i < bt->count; ++i) {
    const int rc = cphifi_ui_rhs(bt->plans[i], y[i], b[i]);
    if (rc != CPHIFI_OK) return rc;
  }
  return CPHIFI_OK;
}

int cphifi_batch_bind(cphifi_batch* bt, const double* const* y, double* const* W) {
  clear_error();
  if (bt == nullptr || y == nullptr || W == nullptr) {
    set_error("bad batch, y or W");
    return CPHIFI_INVALID_ARG;
  }
  for (int i = 0; i < bt->count; ++i)
    if ((y[i] == nullptr && bt->plans[i]->q > 0) || W[i] == nullptr) {
      set_error("member %d: y / W is NULL", i);
      return CPHIFI_INVALID_ARG;
    }
  CPHIFI_HIP(hipStreamSynchronize(bt->st));  // the mirror may still be in flight
  for (int i = 0; i < bt->count; ++i) {
    bt->h_sub[i].y = y[i];
    bt->h_sub[i].W = W[i];
  }
  CPHIFI_HIP(hipMemcpyAsync(bt->d_sub, bt->h_sub, sizeof(BSub) * bt->count,
                            hipMemcpyHostToDevice, bt->st));
  return CPHIFI_OK;
}

int cphifi_batch_graph(cphifi_batch* bt, void** graph_exec) {
  clear_error();
  if (bt == nullptr || graph_exec == nullptr) {
    set_error("bad batch or graph_exec");
    return CPHIFI_INVALID_ARG;
  }
  TRY_RC(build_graph(bt));
  *graph_exec = (void*)bt->exec;
  return CPHIFI_OK;
}

int cphifi_batch_info(cphifi_batch* bt, cphifi_solve_info* infos) {
  clear_error();
  if (bt == nullptr || infos == nullptr) {
    set_error("bad batch or infos");
    return CPHIFI_INVALID_ARG;
  }
  CPHIFI_HIP(hipMemcpyAsync(bt->h_st, bt->d_st, sizeof(BState) * bt->count,
                            hipMemcpyDeviceToHost, bt->st));
  CPHIFI_HIP(hipMemcpyAsync(bt->h_ctl, bt->d_ctl, kCtlHostBytes, hipMemcpyDeviceToHost, bt->st));
  CPHIFI_HIP(hipStreamSynchronize(bt->st));
  const bool timed_out = bt->h_ctl->err != 0;
  int worst = CPHIFI_OK;
  for (int i = 0; i < bt->count; ++i) {
    const BState& s = bt->h_st[i];
    cphifi_solve_info& f = infos[i];
    f.iters = s.total_inner;
    f.refine_steps = s.k;
    f.relres_true = s.cert;
    f.relres_recursive = s.rel;
    f.gemm_ms = 0.0;
    f.gemm_launches = 0;
    int status = s.mode == M_DONE ? s.status : CPHIFI_NOT_CONVERGED;
    if (timed_out) status = CPHIFI_HIP_ERROR;
    f.status = status;
    if (status == CPHIFI_HIP_ERROR)
      worst = CPHIFI_HIP_ERROR;
    else if (status == CPHIFI_NUMERIC && worst != CPHIFI_HIP_ERROR)
      worst = CPHIFI_NUMERIC;
    else if (status != CPHIFI_OK && worst == CPHIFI_OK)
      worst = status;
  }
  if (timed_out) set_error("a grid barrier of the batched kernel timed out");
  return worst;
}

int cphifi_batch_solve(cphifi_batch* bt, const double* const* y, double* const* W,
                       cphifi_solve_info* infos) {
  clear_error();
  if (bt == nullptr) {
    set_error("batch is NULL");
    return CPHIFI_INVALID_ARG;
  }
  if (y != nullptr || W != nullptr) TRY_RC(cphifi_batch_bind(bt, y, W));
  for (int i = 0; i < bt->count; ++i)
    if ((bt->h_sub[i].y == nullptr && bt->plans[i]->q > 0) || bt->h_sub[i].W == nullptr) {
      set_error("member %d has no bound y / W", i);
      return CPHIFI_INVALID_ARG;
    }
  TRY_RC(build_graph(bt));
  CPHIFI_HIP(hipGraphLaunch(bt->exec, bt->st));
  if (infos == nullptr) return CPHIFI_OK;
  return cphifi_batch_info(bt, infos);
}

int cphifi_batch_rounds(cphifi_batch* bt, int* rounds, int* grid) {
  clear_error();
  if (bt == nullptr || rounds == nullptr || grid == nullptr) {
    set_error("bad arguments");
    return CPHIFI_INVALID_ARG;
  }
  CPHIFI_HIP(hipMemcpyAsync(bt->h_ctl, bt->d_ctl, kCtlHostBytes, hipMemcpyDeviceToHost, bt->st));
  CPHIFI_HIP(hipStreamSynchronize(bt->st));
  *rounds = bt->h_ctl->rounds;
  *grid = bt->grid;
  return CPHIFI_OK;
}

int cphifi_batch_phase_ms(cphifi_batch* bt, double* ms) {
  clear_error();
  if (bt == nullptr || ms == nullptr) {
    set_error("bad arguments");
    return CPHIFI_INVALID_ARG;
  }
  CPHIFI_HIP(hipMemcpyAsync(bt->h_ctl, bt->d_ctl, kCtlHostBytes, hipMemcpyDeviceToHost, bt->st));
  CPHIFI_HIP(hipStreamSynchronize(bt->st));
  for (int j = 0; j <= kSlots; ++j) ms[j] = 1e-5 * (double)bt->h_ctl->ticks[j];  // 100 MHz
  return CPHIFI_OK;
}

int cphifi_batch_destroy(cphifi_batch* bt) {
  clear_error();
  if (bt == nullptr) return CPHIFI_OK;
  (void)hipStreamSynchronize(bt->st);
  destroy_batch(bt);
  return CPHIFI_OK;
}

}  // extern "C"
