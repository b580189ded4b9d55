// Plan state shared by the translation units of the solver: the workspace
// layout of one subproblem and the plan object behind cphifi_plan*.
#pragma once

#include "cphifi_internal.h"
#include "small.h"

namespace cphifi {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

enum VecSlot {
  V_R = 0, V_Z, V_P, V_Q,           // outer / FP64 PCG vectors
  V_XHAT, V_Y1, V_T2, V_B,          // product intermediates, internal right-hand side
  V_RF, V_RB, V_XB,                 // refinement residual, its eigenbasis image, correction
  V_R2, V_Z2, V_P2, V_Q2,           // eigenbasis PCG vectors
  V_TMP,
  NVEC
};

struct Layout {
  size_t vec[NVEC];
  size_t part, tpart;
  size_t tseg, tbeg, tend, tslot, tfirst, mseg, mptr, rowm;
  size_t red[3];
  size_t sc, sc2, hist;
  size_t V, UV, dV, D, dKc;
  size_t ulp, utlp, xthi, xtlo, ukt, a32, b32, ut32;
  size_t toep, fptr, fidx, fgram;  // structured forms (Toeplitz K, fiber collapse)
  size_t total;
  int64_t ldl;
  int64_t ntask_max, nslot_max, nmulti_max;
  int hist_len;
};

inline int64_t eff_ldk(const cphifi_ui_desc& d) { return d.ldk > 0 ? d.ldk : d.n; }
// Plans of this size or larger keep a transposed copy of U_K (see
// CPHIFI_FLAG_NO_UKT_COPY).
constexpr int64_t kUktMinN = 4096;
// FP64 plans that run the persistent PCG (small.hip): asked for, or small
// enough that it is the faster form.  Measured per solve against the graph
// replays: n = 208, r = 5 / 8: 1.25 / 1.25 against 2.20 / 1.90 ms; n = 151 /
// 199, r = 10: 1.54 / 1.49 against 1.99 / 2.08 ms; n = 500, r = 5: 1.20
// against 1.51 ms; slower at n = 500, r = 8 (1.86 / 1.80), n = 269, r = 10
// (2.65 / 2.18), r = 16 or n = 1000 (up to 2.4x).  They keep the copy of U_K
// too (the preconditioner reads rows of U and of U^T).
constexpr int kSmallDefaultMaxR = 8;
constexpr int64_t kSmallDefaultMaxNR = 2560;
constexpr int kSmallDefaultWideR = 12;     // with one row per wave:
constexpr int64_t kSmallDefaultWideN = 256;  // n <= 4 x 64 workgroups
inline bool small_plan(const cphifi_ui_desc& d) {
  constexpr int32_t kOff = CPHIFI_FLAG_EIGENBASIS | CPHIFI_FLAG_TOEPLITZ_K |
                           CPHIFI_FLAG_FIBER_COLLAPSE | CPHIFI_FLAG_NO_UKT_COPY |
                           CPHIFI_FLAG_TIME_KERNELS | CPHIFI_FLAG_NO_PERSISTENT;
  const bool wanted = (d.flags & CPHIFI_FLAG_PERSISTENT) ||
                      (d.r <= kSmallDefaultMaxR && d.n * d.r <= kSmallDefaultMaxNR) ||
                      (d.r <= kSmallDefaultWideR && d.n <= kSmallDefaultWideN);
  return d.precision == CPHIFI_FP64 && wanted && !(d.flags & kOff) &&
         small_path_fits(d.n, (int)d.r);
}
inline bool keeps_ukt(const cphifi_ui_desc& d) {
  return (d.n >= kUktMinN && !(d.flags & CPHIFI_FLAG_NO_UKT_COPY)) || small_plan(d);
}
// MIXED_BF16 plans of this size or larger keep an FP32 copy of U_K^T for the
// early refinement residuals (see CPHIFI_FLAG_FP64_RESIDUALS): there an FP64
// pass over U_K costs ~1.5 ms (n = 30658), an FP32 one about half.
constexpr int64_t kUt32MinN = 4096;
inline bool keeps_ut32(const cphifi_ui_desc& d) {
  return d.precision == CPHIFI_MIXED_BF16 && d.n >= kUt32MinN &&
         !(d.flags & CPHIFI_FLAG_FP64_RESIDUALS);
}
inline int eff_maxit(const cphifi_ui_desc& d) { return d.maxit > 0 ? d.maxit : 500; }

// Workspace layout of one subproblem (offsets into the caller's buffer).
Layout make_layout(const cphifi_ui_desc& d);

}  // namespace cphifi

using namespace cphifi;  // the plan is a global type behind the C ABI

constexpr int kPollRing = 16;  // PCG iterations the host may enqueue ahead
constexpr int64_t kGraphMaxN = 4096;  // FP64 plans below this n replay captured iterations
constexpr int kNoWork = -2;    // timing tag of a launch issued after convergence

struct cphifi_plan {
  cphifi_ui_desc d{};
  cphifi_ui_inputs in{};
  hipStream_t st = nullptr;
  int64_t n = 0, r = 0, q = 0, ldk = 0, I = 0, J = 0;
  int ldp = 16;
  double gamma = 0.0;
  int num_cu = 256;
  Layout L{};
  char* ws = nullptr;
  double* vec[NVEC]{};
  void* part = nullptr;
  double* tpart = nullptr;
  ObsTasks tasks{};
  int32_t* rowm = nullptr;  // [n] multi-task segment index of each row, or -1
  double* red[3]{};
  DevScalars* sc = nullptr;
  DevScalars* sc2 = nullptr;
  double* hist = nullptr;
  double *V = nullptr, *UV = nullptr, *dV = nullptr, *D = nullptr, *dKc = nullptr;
  Elt lp = Elt::F64;
  double* ukt = nullptr; // U_K transposed (eigenvector k = column k), or NULL
  float* a32 = nullptr;  // mixed forms, implicit factors: FP32 copies of A and B
  float* b32 = nullptr;  //   (the low-precision gather computes in FP32)
  void* ulp = nullptr;   // U_K rounded: U (BF16 form only; 16 x 64 tiles)
  void* utlp = nullptr;  // U_K rounded: U^T, eigenvector k = row k (FP32 row-major,
                         // BF16 in 16 x 64 tiles)
  float* ut32 = nullptr; // BF16 plans: U^T in FP32 as well, for the early
                         // refinement residuals (keeps_ut32), or NULL
  __bf16 *xthi = nullptr, *xtlo = nullptr;
  double* toep = nullptr;      // FLAG_TOEPLITZ_K: the first row c of K
  int32_t* fptr = nullptr;     // FLAG_FIBER_COLLAPSE: fibers of time s are
  int32_t* fidx = nullptr;     //   fidx[fptr[s] .. fptr[s+1]) (their sample index)
  double* fgram = nullptr;     //   and G = B^T B
  int32_t fmax = 0;            //   most fibers at one time point
  bool small = false;          // FLAG_PERSISTENT taken: the persistent PCG (small.hip)
  hipGraphExec_t pcg_graph = nullptr;  // captured FP64 PCG iterations (paper form)
  GemmPlan gp64n{}, gp64t{}, gplpn{}, gplpt{};  // NN / transposed product plans
  GemmPlan gp32n{}, gp32t{};                    // the same on ut32
  int last_ksplit = 1;  // split-K depth of the partials the last product wrote
  DevScalars* h_sc = nullptr;  // host mirror (mapped, coherent) ...
  DevScalars* d_sc = nullptr;  // ... and its device address
  // Convergence flag that the device writes into host memory every PCG
  // iteration, and one event per in-flight iteration: the host waits for an
  // iteration some steps behind the one it enqueues, so the stream never runs
  // dry while the host decides whether to stop.
  int32_t* h_flag = nullptr;  // host-mapped, coherent
  int32_t* d_flag = nullptr;  // its device address
  hipEvent_t pev[kPollRing]{};
  // Side stream of the whole-subproblem solve: the setup's eig(V) chain (V,
  // its Jacobi eigendecomposition, the eq. fx diagonal) runs there, forked
  // from and joined back into st, while st forms the right-hand side.
  hipStream_t side = nullptr;  // made on the plan's device (`device`)
  int device = 0;               // device current at plan creation
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  bool join_pending = false;  // st has not yet waited for join_ev
  bool timing = false;
  Elt timed_elt = Elt::F64;  // product type whose launches are timed ...
  bool timed_trans = false;  // ... and orientation (one kernel symbol)
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  // Per timed launch (event pair): the PCG step that issued it, 2 it for the
  // operator and 2 it + 1 for the preconditioner of iteration it, -1 outside
  // the iteration, kNoWork once known to have run after convergence (its
  // kernels returned at once, so it is left out of the timing).
  std::vector<int> ev_tag;
  int cur_tag = -1;
  bool setup_done = false;
};

// out (n x r) = K X in FP64 on the plan's stream (partials reduced).
int plan_times_K(cphifi_plan* p, const double* X, double* out);
