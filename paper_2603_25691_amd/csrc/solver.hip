// Plan, operators and solvers behind the C ABI of cphifi.h.
//
// The FP64 method is Section 4.4 of the paper: PCG on
//   (F^T F + lambda I kron K + rho I) vec(W) = vec(K B)
// with the two-step product (Section 4.4.1) and the eq. (fx) preconditioner
// (Section 4.4.2).  The mixed forms keep that FP64 system as the target of an
// iterative-refinement loop whose inner solves run in the eigenbasis of K
// (x = U_K xbar, the rotation the paper uses for the aligned PCG of Section
// 3.3): there the operator is D_K U^T G(U D_K xbar) + lambda D_K xbar + rho xbar,
// which stays symmetric positive definite when U is rounded to FP32 or BF16,
// and the preconditioner of eq. (fx) reduces to its r x r middle step.
#include "cphifi_internal.h"
#include "plan.h"
#include "small.h"

#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <functional>

namespace cphifi {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

}  // namespace cphifi

using namespace cphifi;

namespace cphifi {

Layout make_layout(const cphifi_ui_desc& d) {
  Layout L{};
  const int64_t n = d.n, r = d.r, q = d.q;
  const int64_t nr = n * r;
  const int64_t ldp = round_up(r, 16);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align_up(off, kAlign);
    const size_t o = off;
    off += std::max<size_t>(bytes, 1);
    return o;
  };
  for (int i = 0; i < NVEC; ++i) L.vec[i] = take(sizeof(double) * nr);
  // (the persistent PCG keeps its barrier counter and partial sums here)
  L.part = take(std::max(sizeof(double) * (size_t)kMaxSplit * n * ldp,
                         small_plan(d) ? small_scratch_bytes() : size_t(0)));
  L.ntask_max = n + q / kObsChunk + 1;
  L.nslot_max = 2 * (q / kObsChunk) + 2;
  L.nmulti_max = q / kObsChunk + 1;
  L.tpart = take(sizeof(double) * (size_t)L.nslot_max * r);
  L.tseg = take(sizeof(int32_t) * L.ntask_max);
  L.tbeg = take(sizeof(int32_t) * L.ntask_max);
  L.tend = take(sizeof(int32_t) * L.ntask_max);
  L.tslot = take(sizeof(int32_t) * L.ntask_max);
  L.tfirst = take(sizeof(int32_t) * L.ntask_max);
  L.mseg = take(sizeof(int32_t) * L.nmulti_max);
  L.mptr = take(sizeof(int32_t) * (L.nmulti_max + 1));
  L.rowm = take(sizeof(int32_t) * n);
  for (int i = 0; i < 3; ++i) L.red[i] = take(sizeof(double) * kMaxVecBlocks);
  L.sc = take(sizeof(DevScalars));
  L.sc2 = take(sizeof(DevScalars));
  L.hist_len = eff_maxit(d) + 2;
  L.hist = take(sizeof(double) * L.hist_len);
  L.V = take(sizeof(double) * r * r);
  L.UV = take(sizeof(double) * r * r);
  L.dV = take(sizeof(double) * r);
  L.D = take(sizeof(double) * nr);
  L.dKc = take(sizeof(double) * n);
  if (keeps_ukt(d)) L.ukt = take(sizeof(double) * (size_t)n * eff_ldk(d));
  if (d.flags & CPHIFI_FLAG_TOEPLITZ_K) L.toep = take(sizeof(double) * n);
  if ((d.flags & CPHIFI_FLAG_FIBER_COLLAPSE) && d.J > 0) {
    L.fptr = take(sizeof(int32_t) * (n + 1));
    L.fidx = take(sizeof(int32_t) * (q / d.J + 1));
    L.fgram = take(sizeof(double) * r * r);
  }
  L.ldl = round_up(n, kLowpAlign);
  if (d.precision != CPHIFI_FP64 && d.I > 0 && d.J > 0) {
    L.a32 = take(sizeof(float) * (size_t)d.I * r);
    L.b32 = take(sizeof(float) * (size_t)d.J * r);
  }
  if (d.precision == CPHIFI_MIXED_BF16) {
    // 16 x 64 tiles (the BF16 product's layout): whole 16-row blocks
    L.ulp = take(sizeof(__bf16) * (size_t)round_up(n, 16) * L.ldl);
    L.utlp = take(sizeof(__bf16) * (size_t)round_up(n, 16) * L.ldl);
    L.xthi = take(sizeof(__bf16) * (size_t)ldp * L.ldl);
    L.xtlo = take(sizeof(__bf16) * (size_t)ldp * L.ldl);
  } else if (d.precision == CPHIFI_MIXED_FP32) {
    L.utlp = take(sizeof(float) * (size_t)n * L.ldl);
  }
  if (keeps_ut32(d)) L.ut32 = take(sizeof(float) * (size_t)n * L.ldl);
  L.total = align_up(off, kAlign);
  return L;
}

}  // namespace cphifi

namespace {

// ------------------------------------------------------------------ timing
int timed_begin(cphifi_plan* p, Elt elt, bool trans, hipEvent_t* out) {
  *out = nullptr;
  if (!p->timing || elt != p->timed_elt || trans != p->timed_trans) return CPHIFI_OK;
  if (p->ev_used + 2 > p->ev.size()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      CPHIFI_HIP(hipEventCreate(&e));
      p->ev.push_back(e);
    }
    p->ev_tag.resize(p->ev.size() / 2);
  }
  p->ev_tag[p->ev_used / 2] = p->cur_tag;
  *out = p->ev[p->ev_used];
  CPHIFI_HIP(hipEventRecord(*out, p->st));
  return CPHIFI_OK;
}

int timed_end(cphifi_plan* p, hipEvent_t start) {
  if (start == nullptr) return CPHIFI_OK;
  CPHIFI_HIP(hipEventRecord(p->ev[p->ev_used + 1], p->st));
  p->ev_used += 2;
  return CPHIFI_OK;
}

int timing_collect(cphifi_plan* p, double* ms, int* count) {
  *ms = 0.0;
  *count = 0;
  if (!p->timing) return CPHIFI_OK;
  for (size_t i = 0; i + 1 < p->ev_used; i += 2) {
    if (p->ev_tag[i / 2] == kNoWork) continue;
    float t = 0.f;
    CPHIFI_HIP(hipEventElapsedTime(&t, p->ev[i], p->ev[i + 1]));
    *ms += t;
    ++*count;
  }
  p->ev_used = 0;
  return CPHIFI_OK;
}

#define TRY(x)                       \
  do {                               \
    const int s_ = (x);              \
    if (s_ != CPHIFI_OK) return s_;  \
  } while (0)

// ------------------------------------------------------------ n x n products
// part <- K X.  K is symmetric, so K X = K^T X: the transposed product,
// whose loads each cover four full 128-byte lines of K, runs faster than the
// row-major one at these shapes (1.57 vs 1.69 ms at n = 30658, r = 40).
int prod_K(cphifi_plan* p, const double* X, const int32_t* done) {
  if (p->toep != nullptr) {  // symmetric Toeplitz K: c only (untimed)
    return launch_toeplitz_product(p->toep, p->n, X, p->r, (int)p->r, (double*)p->part, p->ldp,
                                   p->num_cu, &p->last_ksplit, done, p->st);
  }
  hipEvent_t e0;
  TRY(timed_begin(p, Elt::F64, true, &e0));
  TRY(launch_gemm(Elt::F64, true, p->gp64t, p->in.K, p->ldk, p->n, X, p->r, (int)p->r, nullptr,
                  p->part, done, p->st));
  p->last_ksplit = p->gp64t.ksplit;
  return timed_end(p, e0);
}

// part <- U (diag(xscale) X) at element type elt.  UK holds U^T row-major
// (LAPACK column-major U), so in FP64/FP32 this is the transposed product.
int prod_U(cphifi_plan* p, Elt elt, const double* X, const double* xscale,
           const int32_t* done) {
  if (elt == Elt::BF16)
    TRY(launch_split_bf16(X, p->r, (int)p->r, xscale, p->n, p->xthi, p->xtlo, p->L.ldl, done,
                          p->st));
  hipEvent_t e0;
  TRY(timed_begin(p, elt, elt != Elt::BF16, &e0));
  switch (elt) {
    case Elt::F64:
      TRY(launch_gemm(Elt::F64, true, p->gp64t, p->in.UK, p->ldk, p->n, X, p->r, (int)p->r,
                      xscale, p->part, done, p->st));
      p->last_ksplit = p->gp64t.ksplit;
      break;
    case Elt::F32: {
      // the FP32 plan's own copy, or a BF16 plan's FP32 copy of U^T
      const bool own = p->lp == Elt::F32;
      const GemmPlan& gp = own ? p->gplpt : p->gp32t;
      const void* m = own ? p->utlp : (const void*)p->ut32;
      if (m == nullptr) {
        set_error("internal: FP32 product without an FP32 copy of U_K");
        return CPHIFI_INVALID_ARG;
      }
      TRY(launch_gemm(Elt::F32, true, gp, m, p->L.ldl, p->n, X, p->r, (int)p->r, xscale,
                      p->part, done, p->st));
      p->last_ksplit = gp.ksplit;
      break;
    }
    case Elt::BF16:
      TRY(launch_gemm_bf16(p->gplpn, (const __bf16*)p->ulp, p->L.ldl, p->n, X, p->r, (int)p->r,
                           xscale, p->part, p->xthi, p->xtlo, p->L.ldl, done, p->st, true));
      p->last_ksplit = p->gplpn.ksplit;
      break;
  }
  return timed_end(p, e0);
}

// part <- U^T X at element type elt (row-major NN product on U^T, or in FP64
// the transposed product on the plan's copy of U when it keeps one).
int prod_Ut(cphifi_plan* p, Elt elt, const double* X, const int32_t* done,
            bool presplit = false) {
  if (elt == Elt::BF16 && !presplit)
    TRY(launch_split_bf16(X, p->r, (int)p->r, nullptr, p->n, p->xthi, p->xtlo, p->L.ldl, done,
                          p->st));
  const bool tcopy = elt == Elt::F64 && p->ukt != nullptr;
  hipEvent_t e0;
  TRY(timed_begin(p, elt, tcopy, &e0));
  switch (elt) {
    case Elt::F64:
      if (tcopy) {
        TRY(launch_gemm(Elt::F64, true, p->gp64t, p->ukt, p->ldk, p->n, X, p->r, (int)p->r,
                        nullptr, p->part, done, p->st));
        p->last_ksplit = p->gp64t.ksplit;
      } else {
        TRY(launch_gemm(Elt::F64, false, p->gp64n, p->in.UK, p->ldk, p->n, X, p->r, (int)p->r,
                        nullptr, p->part, done, p->st));
        p->last_ksplit = p->gp64n.ksplit;
      }
      break;
    case Elt::F32: {
      const bool own = p->lp == Elt::F32;
      const GemmPlan& gp = own ? p->gplpn : p->gp32n;
      const void* m = own ? p->utlp : (const void*)p->ut32;
      if (m == nullptr) {
        set_error("internal: FP32 product without an FP32 copy of U_K");
        return CPHIFI_INVALID_ARG;
      }
      TRY(launch_gemm(Elt::F32, false, gp, m, p->L.ldl, p->n, X, p->r, (int)p->r, nullptr,
                      p->part, done, p->st));
      p->last_ksplit = gp.ksplit;
      break;
    }
    case Elt::BF16:
      TRY(launch_gemm_bf16(p->gplpn, (const __bf16*)p->utlp, p->L.ldl, p->n, X, p->r, (int)p->r,
                           nullptr, p->part, p->xthi, p->xtlo, p->L.ldl, done, p->st, true));
      p->last_ksplit = p->gplpn.ksplit;
      break;
  }
  return timed_end(p, e0);
}

// Split-K depth of the partials in p->part (set by the product that wrote them).
int ksplit_of(const cphifi_plan* p, Elt /*elt*/) { return p->last_ksplit; }

// Gather-dot-scatter over the observations: out <- G applied to the product
// held in part (gather mode), optionally storing Xhat.
// With split (lane-row form only), the rows go out as the hi/lo BF16 operand
// of the next product instead of to out.
int obs_gather(cphifi_plan* p, Elt elt, double* xhat, double* out, const int32_t* done,
               bool split = false) {
  if (p->fptr != nullptr) {  // every observed fiber complete: r^2 work per fiber
    if (split) {
      set_error("internal: the fiber-collapsed gather has no split output");
      return CPHIFI_INVALID_ARG;
    }
    return launch_fiber_gather(p->part, elt != Elt::F64, ksplit_of(p, elt), p->ldp, nullptr,
                               p->n, (int)p->r, p->fptr, p->fidx, p->in.A, p->fgram, xhat, out,
                               p->fmax, done, p->st);
  }
  ObsArgs a{};
  a.n = p->n;
  a.r = (int)p->r;
  a.obs_i = p->in.obs_i;
  a.obs_j = p->in.obs_j;
  a.A = p->in.A;
  a.B = p->in.B;
  a.A32 = p->a32;
  a.B32 = p->b32;
  a.Zhat = p->in.Zhat;
  a.y = nullptr;
  a.part = p->part;
  a.ksplit = ksplit_of(p, elt);
  a.ldp = p->ldp;
  a.Xhat = xhat;
  a.out = out;
  a.tpart = p->tpart;
  a.done = done;
  if (split) {
    a.xt_hi = p->xthi;
    a.xt_lo = p->xtlo;
    a.ldxt = p->L.ldl;
  }
  return launch_obs(ObsMode::Gather, elt != Elt::F64, p->tasks, a, p->I, p->J, p->st);
}

// ------------------------------------------------------------------ operators
// y = A x in FP64, paper form (Section 4.4.1); red <- partials of x . y.
int op_apply_paper(cphifi_plan* p, const double* x, double* y, double* red, int* nblk,
                   const int32_t* done) {
  TRY(prod_K(p, x, done));
  TRY(obs_gather(p, Elt::F64, p->vec[V_XHAT], p->vec[V_Y1], done));
  TRY(prod_K(p, p->vec[V_Y1], done));
  return launch_apply_finish(p->part, false, p->last_ksplit, p->ldp, p->n, (int)p->r,
                             p->vec[V_XHAT], x, nullptr, p->d.lambda, p->d.rho, y, red, nblk,
                             done, p->st);
}

// z = M^{-1} x in FP64 (eq. fx); red <- partials of x . z.
int op_precond_paper(cphifi_plan* p, const double* x, double* z, double* red, int* nblk,
                     const int32_t* done) {
  if (p->d.flags & CPHIFI_FLAG_NO_PRECOND) {
    TRY(launch_copy(z, x, p->n * p->r, p->st));
    return red ? launch_dot(x, z, p->n * p->r, red, nblk, done, p->st) : CPHIFI_OK;
  }
  TRY(prod_Ut(p, Elt::F64, x, done));
  TRY(launch_prec_mid(p->part, false, p->last_ksplit, p->ldp, nullptr, p->n, (int)p->r, p->UV,
                      p->D, p->vec[V_T2], nullptr, nullptr, nullptr, done, p->st));
  TRY(prod_U(p, Elt::F64, p->vec[V_T2], nullptr, done));
  return launch_reduce_partials(p->part, false, p->last_ksplit, p->ldp, p->n, (int)p->r, z, x,
                                red, nblk, done, p->st);
}

// ybar = D_K U^T G(U D_K xbar) + lambda D_K xbar + rho xbar at element type elt.
int op_apply_eig(cphifi_plan* p, Elt elt, const double* xb, double* yb, double* red, int* nblk,
                 const int32_t* done) {
  // BF16 with the lane-row gather: the gather writes the split operand of
  // U^T Yhat1 itself (the split of U (D_K xbar) before it has zeroed the
  // padding rows and columns of that operand).
  const bool fuse = elt == Elt::BF16 && p->tasks.rows && p->fptr == nullptr;
  if (elt == Elt::BF16) {
    TRY(prod_U(p, elt, xb, p->dKc, done));  // the split applies D_K
  } else {
    // D_K xbar first: the FP64 / FP32 tiles would multiply it in while
    // staging X, where the wait for the scale loads holds back the prefetch of
    // U (2.04 against 1.51 ms per FP64 product at n = 30658, r = 40).
    TRY(launch_scale_rows(p->vec[V_XHAT], xb, p->dKc, p->n, (int)p->r, done, p->st));
    TRY(prod_U(p, elt, p->vec[V_XHAT], nullptr, done));
  }
  TRY(obs_gather(p, elt, nullptr, p->vec[V_Y1], done, fuse));
  TRY(prod_Ut(p, elt, p->vec[V_Y1], done, fuse));
  return launch_apply_finish(p->part, elt != Elt::F64, ksplit_of(p, elt), p->ldp, p->n,
                             (int)p->r, nullptr, xb, p->dKc, p->d.lambda, p->d.rho, yb, red, nblk,
                             done, p->st);
}

// zbar = ((xbar U_V) had D) U_V^T: eq. (fx) in the eigenbasis of K.
int op_precond_eig(cphifi_plan* p, const double* xb, double* zb, double* red, int* nblk,
                   const int32_t* done) {
  return launch_prec_mid(nullptr, false, 1, p->ldp, xb, p->n, (int)p->r, p->UV, p->D, zb, xb,
                         red, nblk, done, p->st);
}

// out <- U^T x (elt) with the partials reduced in FP64.
int rotate_in(cphifi_plan* p, Elt elt, const double* x, double* out) {
  TRY(prod_Ut(p, elt, x, nullptr));
  return launch_reduce_partials(p->part, elt != Elt::F64, ksplit_of(p, elt), p->ldp, p->n,
                                (int)p->r, out, nullptr, nullptr, nullptr, nullptr, p->st);
}

// out <- U x (elt).
int rotate_out(cphifi_plan* p, Elt elt, const double* x, double* out) {
  TRY(prod_U(p, elt, x, nullptr, nullptr));
  return launch_reduce_partials(p->part, elt != Elt::F64, ksplit_of(p, elt), p->ldp, p->n,
                                (int)p->r, out, nullptr, nullptr, nullptr, nullptr, p->st);
}

using OpFn = std::function<int(const double*, double*, double*, int*, const int32_t*)>;

struct PcgVecs {
  double *R, *Z, *P, *Q;
};

struct PcgOut {
  int iters = 0;
  int status = CPHIFI_OK;
  double relres = 0.0;
};

// Host copy of *sc once the stream has drained (a kernel writes it into the
// mapped mirror: cheaper than a device-to-host copy of a few words).
int poll(cphifi_plan* p, DevScalars* sc) {
  TRY(launch_mirror(sc, p->d_sc, p->st));
  CPHIFI_HIP(hipStreamSynchronize(p->st));
  return CPHIFI_OK;
}

// Iterations the host keeps enqueued beyond the newest one whose convergence
// flag it has read (at most kPollRing - 1).
int check_every(const cphifi_plan* p) {
  const int e = p->d.check_every > 0 ? p->d.check_every : (p->n >= 4096 ? 1 : 8);
  return std::min(e, kPollRing - 1);
}

// Makes the plan's stream wait for the eig(V) chain that setup_plan left on
// the side stream.  Whatever reads V, U_V, d_V or D runs after this.
int join_setup(cphifi_plan* p) {
  if (!p->join_pending) return CPHIFI_OK;
  p->join_pending = false;
  CPHIFI_HIP(hipStreamWaitEvent(p->st, p->join_ev, 0));
  return CPHIFI_OK;
}

// Textbook PCG with device-resident scalars.  Every kernel of an iteration
// checks sc->done, so iterations can be enqueued ahead of the host's check:
// after enqueuing iteration it, the host waits for iteration it - every and
// reads the convergence flag that iteration's check wrote to host memory.
// The stream keeps `every` iterations of work queued meanwhile; those left
// over after convergence return at once.
// fused_eig: the preconditioner is the eigenbasis one (op_precond_eig); the
// iteration then runs the x/r update and the preconditioner as one kernel.
// graph: the iterations run as replays of a HIP graph that holds
// kGraphIters captured iterations (built on first use and kept in the plan);
// the kernels then take the iteration index from the device counter, and x
// lives in the plan's V_XB (the graph's pointers must not change between
// solves), copied from / to the caller's x around the loop.
constexpr int kGraphIters = 8;

int run_pcg(cphifi_plan* p, const OpFn& apply, const OpFn& precond, const double* b, double* x,
            bool have_x0, double tol, int maxit, const PcgVecs& v, DevScalars* sc,
            double* hist, int hist_len, PcgOut* out, bool fused_eig = false,
            bool graph = false) {
  const int64_t len = p->n * p->r;
  hipStream_t st = p->st;
  const hipStream_t st_caller = st;
  double* x_user = x;
  if (graph) {
    x = p->vec[V_XB];
    if (have_x0) TRY(launch_copy(x, x_user, len, st));
  }
  int nb_bb = 0, nb_rr = 0, nb_rz = 0, nb_pq = 0;
  double* red0 = p->red[0];
  double* red1 = p->red[1];
  double* red2 = p->red[2];
  // red0 <- ||b||^2 partials are consumed by pcg_init; keep them in red0 until then.
  TRY(launch_dot(b, b, len, red0, &nb_bb, nullptr, st));
  TRY(launch_copy(v.R, b, len, st));
  if (have_x0) {
    TRY(apply(x, v.Q, nullptr, nullptr, nullptr));
    TRY(launch_axpby(v.R, -1.0, v.Q, 1.0, len, nullptr, st));
  } else {
    TRY(launch_fill(x, 0.0, len, st));
  }
  TRY(launch_dot(v.R, v.R, len, red1, &nb_rr, nullptr, st));
  TRY(precond(v.R, v.Z, red2, &nb_rz, nullptr));
  TRY(launch_copy(v.P, v.Z, len, st));
  TRY(launch_pcg_init(sc, red0, nb_bb, red1, nb_rr, red2, nb_rz, tol, hist, hist_len, st));
  const int every = check_every(p);
  *(volatile int32_t*)p->h_flag = 0;
  const size_t first_pair = p->ev_used / 2;
  int it0 = 0;  // first iteration the loop below runs (after the graph replays)
  if (graph) {
    if (p->pcg_graph == nullptr) {
      // Capture kGraphIters iterations with device-counted iteration indices,
      // on a private stream (the caller's may be the null stream, which
      // cannot be captured); replays go to the caller's stream.
      hipGraph_t g = nullptr;
      hipStream_t cap = nullptr;
      CPHIFI_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      if (hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed) != hipSuccess) {
        (void)hipStreamDestroy(cap);
        set_error("PCG graph: hipStreamBeginCapture failed");
        return CPHIFI_HIP_ERROR;
      }
      p->st = cap;
      st = cap;
      int rc = CPHIFI_OK;
      for (int k = 0; k < kGraphIters && rc == CPHIFI_OK; ++k) {
        if ((rc = apply(v.P, v.Q, red0, &nb_pq, &sc->done)) != CPHIFI_OK ||
            (rc = launch_update_xr(x, v.R, v.P, v.Q, len, red0, nb_pq, red1, &nb_rr, sc, -1,
                                   st)) != CPHIFI_OK ||
            (rc = launch_check_conv(red1, nb_rr, sc, -1, hist, hist_len, p->d_flag, st)) !=
                CPHIFI_OK ||
            (rc = precond(v.R, v.Z, red2, &nb_rz, &sc->done)) != CPHIFI_OK)
          break;
        rc = launch_update_p(v.P, v.Z, len, red2, nb_rz, sc, -1, st);
      }
      const hipError_t ec = hipStreamEndCapture(cap, &g);
      p->st = st = st_caller;
      (void)hipStreamDestroy(cap);
      if (rc != CPHIFI_OK || ec != hipSuccess ||
          hipGraphInstantiateWithFlags(&p->pcg_graph, g, 0) != hipSuccess) {
        if (g != nullptr) (void)hipGraphDestroy(g);
        p->pcg_graph = nullptr;
        if (rc == CPHIFI_OK) set_error("PCG graph capture failed");
        return rc != CPHIFI_OK ? rc : CPHIFI_HIP_ERROR;
      }
      (void)hipGraphDestroy(g);
    }
    // Replays, one ahead of the host's check of the convergence flag.
    int launched = 0;
    bool stop = false;
    while (it0 + kGraphIters <= maxit) {
      CPHIFI_HIP(hipGraphLaunch(p->pcg_graph, st));
      CPHIFI_HIP(hipEventRecord(p->pev[launched % kPollRing], st));
      ++launched;
      it0 += kGraphIters;
      if (launched >= 2) {
        CPHIFI_HIP(hipEventSynchronize(p->pev[(launched - 2) % kPollRing]));
        if (*(volatile int32_t*)p->h_flag) {
          stop = true;
          break;
        }
      }
    }
    if (!stop && launched > 0) {
      CPHIFI_HIP(hipEventSynchronize(p->pev[(launched - 1) % kPollRing]));
      stop = *(volatile int32_t*)p->h_flag != 0;
    }
    if (stop) it0 = maxit;  // done: the loop below runs nothing
  }
  for (int it = it0; it < maxit; ++it) {
    p->cur_tag = 2 * it;
    TRY(apply(v.P, v.Q, red0, &nb_pq, &sc->done));
    if (fused_eig) {
      TRY(launch_update_prec(x, v.R, v.P, v.Q, p->n, (int)p->r, p->UV, p->D, v.Z, red0, nb_pq,
                             red1, red2, &nb_rr, sc, it, st));
      nb_rz = nb_rr;
    } else {
      TRY(launch_update_xr(x, v.R, v.P, v.Q, len, red0, nb_pq, red1, &nb_rr, sc, it, st));
    }
    TRY(launch_check_conv(red1, nb_rr, sc, it, hist, hist_len, p->d_flag, st));
    CPHIFI_HIP(hipEventRecord(p->pev[it % kPollRing], st));
    if (it - it0 >= every) {
      CPHIFI_HIP(hipEventSynchronize(p->pev[(it - every) % kPollRing]));
      if (*(volatile int32_t*)p->h_flag) break;
    }
    if (it + 1 == maxit) break;
    p->cur_tag = 2 * it + 1;
    if (!fused_eig) TRY(precond(v.R, v.Z, red2, &nb_rz, &sc->done));
    TRY(launch_update_p(v.P, v.Z, len, red2, nb_rz, sc, it, st));
  }
  p->cur_tag = -1;
  if (graph) TRY(launch_copy(x_user, x, len, st));
  TRY(poll(p, sc));
  const DevScalars& h = *p->h_sc;
  out->iters = h.done ? h.iters : maxit;
  // Launches of the iterations enqueued past convergence did no work.
  for (size_t i = first_pair; i < p->ev_used / 2; ++i)
    if (p->ev_tag[i] >= 2 * out->iters - 1) p->ev_tag[i] = kNoWork;
  out->status = h.done ? h.status : CPHIFI_NOT_CONVERGED;
  out->relres = h.bb > 0.0 ? std::sqrt(h.rr / h.bb) : 0.0;
  return CPHIFI_OK;
}

// ||b - A x|| / ||b|| with the FP64 paper-form product (residual certificate).
int true_relres(cphifi_plan* p, const double* b, const double* x, double* rel) {
  const int64_t len = p->n * p->r;
  int nb = 0, nbb = 0;
  TRY(op_apply_paper(p, x, p->vec[V_Q], nullptr, nullptr, nullptr));
  TRY(launch_copy(p->vec[V_RF], b, len, p->st));
  TRY(launch_axpby(p->vec[V_RF], -1.0, p->vec[V_Q], 1.0, len, nullptr, p->st));
  TRY(launch_dot(p->vec[V_RF], p->vec[V_RF], len, p->red[0], &nb, nullptr, p->st));
  TRY(launch_store_sum(p->red[0], nb, p->sc2, 0, p->st));
  TRY(launch_dot(b, b, len, p->red[1], &nbb, nullptr, p->st));
  TRY(launch_store_sum(p->red[1], nbb, p->sc2, 1, p->st));
  TRY(poll(p, p->sc2));
  const double rr = p->h_sc->scratch[0], bb = p->h_sc->scratch[1];
  *rel = bb > 0.0 ? std::sqrt(rr / bb) : (rr > 0.0 ? INFINITY : 0.0);
  return CPHIFI_OK;
}

// The same certificate for b = K Bm given through Bm (the observed MTTKRP):
// b - A W = K (Bm - Yhat1 - lambda W) - rho W with Yhat1 = G(K W), two passes
// over K as above; bb = ||b||^2 comes from the caller.
int true_relres_from_B(cphifi_plan* p, const double* Bm, const double* W, double bb,
                       double* rel) {
  const int64_t len = p->n * p->r;
  double* T = p->vec[V_Z];
  double* RF = p->vec[V_RF];
  int nb = 0;
  TRY(prod_K(p, W, nullptr));
  TRY(obs_gather(p, Elt::F64, nullptr, p->vec[V_Y1], nullptr));
  TRY(launch_copy(T, Bm, len, p->st));
  TRY(launch_axpby(T, -1.0, p->vec[V_Y1], 1.0, len, nullptr, p->st));
  TRY(launch_axpby(T, -p->d.lambda, W, 1.0, len, nullptr, p->st));
  TRY(prod_K(p, T, nullptr));
  TRY(launch_reduce_partials(p->part, false, p->last_ksplit, p->ldp, p->n, (int)p->r, RF,
                             nullptr, nullptr, nullptr, nullptr, p->st));
  TRY(launch_axpby(RF, -p->d.rho, W, 1.0, len, nullptr, p->st));
  TRY(launch_dot(RF, RF, len, p->red[0], &nb, nullptr, p->st));
  TRY(launch_store_sum(p->red[0], nb, p->sc2, 0, p->st));
  TRY(poll(p, p->sc2));
  const double rr = p->h_sc->scratch[0];
  *rel = bb > 0.0 ? std::sqrt(rr / bb) : (rr > 0.0 ? INFINITY : 0.0);
  return CPHIFI_OK;
}

}  // namespace

int plan_times_K(cphifi_plan* p, const double* X, double* out) {
  const bool t = p->timing;
  p->timing = false;
  const int rc = prod_K(p, X, nullptr);
  p->timing = t;
  TRY(rc);
  return launch_reduce_partials(p->part, false, p->last_ksplit, p->ldp, p->n, (int)p->r, out,
                                nullptr, nullptr, nullptr, nullptr, p->st);
}

namespace {

// The whole FP64 PCG of a small subproblem in one persistent launch
// (small.hip): no launch or host poll per iteration.
int run_small_pcg(cphifi_plan* p, const double* b, double* W, bool warm, int maxit,
                  PcgOut* out) {
  SmallArgs a{};
  a.n = p->n;
  a.ldk = p->ldk;
  a.r = (int)p->r;
  a.warm = warm ? 1 : 0;
  a.precond = (p->d.flags & CPHIFI_FLAG_NO_PRECOND) ? 0 : 1;
  a.maxit = maxit;
  a.hist_len = p->L.hist_len;
  a.lam = p->d.lambda;
  a.rho = p->d.rho;
  a.tol = p->d.tol;
  // CPHIFI_SMALL_SPIN_LIMIT shortens the barrier waits (tests of the fallback)
  const char* spin_env = std::getenv("CPHIFI_SMALL_SPIN_LIMIT");
  a.spin_limit = (spin_env != nullptr && std::atoll(spin_env) > 0) ? std::atoll(spin_env)
                                                                   : kSmallSpinLimit;
  a.K = p->in.K;
  a.UK = p->in.UK;
  a.UKT = p->ukt;
  a.UV = p->UV;
  a.D = p->D;
  a.obs_ptr = p->in.obs_ptr;
  a.obs_i = p->in.obs_i;
  a.obs_j = p->in.obs_j;
  a.A = p->in.A;
  a.B = p->in.B;
  a.Zhat = p->in.Zhat;
  a.b = b;
  a.X = W;
  a.R0 = p->vec[V_R];
  a.R1 = p->vec[V_R2];
  a.P0 = p->vec[V_P];
  a.P1 = p->vec[V_P2];
  a.Z = p->vec[V_Z];
  a.Q = p->vec[V_Q];
  a.Xh = p->vec[V_XHAT];
  a.Y1 = p->vec[V_Y1];
  a.T2 = p->vec[V_T2];
  a.scratch = p->part;
  a.hist = p->hist;
  a.out = (SmallOut*)p->sc2;  // the certificate's scalars are free until it runs
  // The kernel updates W in place: keep the starting point of a warm start
  // for the fallback below.
  if (warm) TRY(launch_copy(p->vec[V_XB], W, p->n * p->r, p->st));
  TRY(launch_small_pcg(a, p->st));
  SmallOut h{};
  CPHIFI_HIP(hipMemcpyAsync(&h, a.out, sizeof(h), hipMemcpyDeviceToHost, p->st));
  CPHIFI_HIP(hipStreamSynchronize(p->st));
  if (h.status == kSmallTimeout) {
    // Not every workgroup was resident (other work on the device): the
    // caller runs the multi-kernel loop instead, from the same start.
    if (warm) TRY(launch_copy(W, p->vec[V_XB], p->n * p->r, p->st));
    return kSmallTimeout;
  }
  out->iters = h.iters;
  out->status = h.status;
  out->relres = h.bb > 0.0 ? std::sqrt(h.rr / h.bb) : 0.0;
  return CPHIFI_OK;
}

int solve_fp64(cphifi_plan* p, const double* b, double* W, cphifi_solve_info* info) {
  const bool warm = (p->d.flags & CPHIFI_FLAG_WARM_START) != 0;
  const int maxit = eff_maxit(p->d);
  PcgOut o;
  bool small = p->small && p->ukt != nullptr && !p->timing;
  if (small) {
    const int rs = run_small_pcg(p, b, W, warm, maxit, &o);
    if (rs == kSmallTimeout)
      small = false;
    else
      TRY(rs);
  }
  if (small) {
    // done
  } else if (p->d.flags & CPHIFI_FLAG_EIGENBASIS) {
    // x = U xbar: PCG on the rotated system, then rotate back.
    TRY(rotate_in(p, Elt::F64, b, p->vec[V_RB]));
    if (warm) TRY(rotate_in(p, Elt::F64, W, p->vec[V_XB]));
    OpFn A = [p](const double* x, double* y, double* red, int* nb, const int32_t* done) {
      return op_apply_eig(p, Elt::F64, x, y, red, nb, done);
    };
    OpFn M = [p](const double* x, double* z, double* red, int* nb, const int32_t* done) {
      return op_precond_eig(p, x, z, red, nb, done);
    };
    TRY(run_pcg(p, A, M, p->vec[V_RB], p->vec[V_XB], warm, p->d.tol, maxit,
                PcgVecs{p->vec[V_R2], p->vec[V_Z2], p->vec[V_P2], p->vec[V_Q2]}, p->sc, p->hist,
                p->L.hist_len, &o, true));
    TRY(rotate_out(p, Elt::F64, p->vec[V_XB], W));
  } else {
    OpFn A = [p](const double* x, double* y, double* red, int* nb, const int32_t* done) {
      return op_apply_paper(p, x, y, red, nb, done);
    };
    OpFn M = [p](const double* x, double* z, double* red, int* nb, const int32_t* done) {
      return op_precond_paper(p, x, z, red, nb, done);
    };
    // Small plans replay captured iterations: there the launches, not the
    // kernels, set the iteration time.
    const bool graph = p->n < kGraphMaxN && !p->timing && !(p->d.flags & CPHIFI_FLAG_NO_GRAPH);
    TRY(run_pcg(p, A, M, b, W, warm, p->d.tol, maxit,
                PcgVecs{p->vec[V_R], p->vec[V_Z], p->vec[V_P], p->vec[V_Q]}, p->sc, p->hist,
                p->L.hist_len, &o, false, graph));
  }
  info->iters = o.iters;
  info->refine_steps = 0;
  info->relres_recursive = o.relres;
  if (info->history != nullptr) {
    const int cnt = std::min(o.iters + 1, p->L.hist_len);
    CPHIFI_HIP(hipMemcpyAsync(info->history, p->hist, sizeof(double) * cnt,
                              hipMemcpyDeviceToHost, p->st));
  }
  // Timing covers the solve only: the certificate below is not part of it.
  TRY(timing_collect(p, &info->gemm_ms, &info->gemm_launches));
  const bool t = p->timing;
  p->timing = false;
  double rel = 0.0;
  const int rs = true_relres(p, b, W, &rel);
  p->timing = t;
  TRY(rs);
  info->relres_true = rel;
  int status = o.status;
  if (status == CPHIFI_OK && !(rel <= 10.0 * p->d.tol)) status = CPHIFI_NOT_CONVERGED;
  if (!std::isfinite(rel)) status = CPHIFI_NUMERIC;
  info->status = status;
  return status;
}

// FP64 iterative refinement around inner PCG solves in the eigenbasis of K at
// the plan's low precision.  The refinement itself lives in the eigenbasis:
// with bbar = U^T b and the accumulated correction xbar, each step takes the
// FP64 residual rbar = bbar - Abar xbar of the rotated system (two FP64 passes
// over U_K; U_K is orthogonal, so ||rbar|| = ||b - A U xbar||), solves
// Abar_lp dbar = rbar at low precision and adds dbar to xbar.  W = U xbar is
// formed once at the end and certified by the FP64 residual of the original
// system (two passes over K); should that certificate miss the target while
// the rotated one met it, refinement continues.  When the last step's
// contraction predicts that the next residual meets tol with a margin
// (kCertifyFirst), the rotated residual is skipped and W is certified at once
// (three passes instead of five); on a miss the certificate's residual,
// rotated into the eigenbasis (one pass), continues the refinement.
//
// The right-hand side comes either as b = K Bm or, from the whole-subproblem
// entry, as Bm itself (the observed MTTKRP, eq. for B in Section 4.4): then
// bbar = U^T K Bm = D_K U^T Bm takes one pass over U_K instead of a pass over
// K followed by one over U_K, and the certificate forms b - A W without b.
int solve_mixed(cphifi_plan* p, const double* b, const double* Bm, double* W,
                cphifi_solve_info* info) {
  const bool warm = (p->d.flags & CPHIFI_FLAG_WARM_START) != 0;
  const int64_t len = p->n * p->r;
  const int maxit = eff_maxit(p->d);
  const int max_refine = p->d.max_refine > 0 ? p->d.max_refine : 30;
  const double inner_tol = p->d.inner_tol > 0.0 ? p->d.inner_tol : kInnerTol;
  const Elt elt = p->lp;
  double* bbar = p->vec[V_T2];
  double* xbar = p->vec[V_TMP];
  double* rbar = p->vec[V_RB];
  int nb = 0;
  // The rotations into and out of the eigenbasis use the FP64 eigenvectors:
  // a rounded U_K is not orthogonal, and its error, mapped through the
  // ill-conditioned system, makes the refinement diverge.  Only the inner
  // operator runs at low precision; the FP64 residual corrects its error.
  if (Bm != nullptr) {
    TRY(prod_Ut(p, Elt::F64, Bm, nullptr));
    TRY(launch_reduce_partials(p->part, false, p->last_ksplit, p->ldp, p->n, (int)p->r, bbar,
                               nullptr, nullptr, nullptr, nullptr, p->st, p->dKc));
  } else {
    TRY(rotate_in(p, Elt::F64, b, bbar));
  }
  TRY(launch_dot(bbar, bbar, len, p->red[1], &nb, nullptr, p->st));
  TRY(launch_store_sum(p->red[1], nb, p->sc2, 1, p->st));
  if (warm)
    TRY(rotate_in(p, Elt::F64, W, xbar));
  else
    TRY(launch_fill(xbar, 0.0, len, p->st));
  OpFn A = [p, elt](const double* x, double* y, double* red, int* nbk, const int32_t* done) {
    return op_apply_eig(p, elt, x, y, red, nbk, done);
  };
  OpFn M = [p](const double* x, double* z, double* red, int* nbk, const int32_t* done) {
    return op_precond_eig(p, x, z, red, nbk, done);
  };
  int total_inner = 0, k = 0, status = CPHIFI_NOT_CONVERGED;
  double rel = INFINITY, rel_prev = INFINITY, cert = INFINITY, bb_bar = 0.0;
  bool fresh = !warm;  // xbar = 0: its residual is bbar
  // W = U xbar and its certificate.  It leaves b - A W in vec[V_RF].
  // ||b|| = ||U^T b|| (U_K orthogonal) when b is not formed.  The
  // certificate's products are timed only when the FP64 product is the timed
  // kernel (CPHIFI_FLAG_TIME_FP64: every FP64 product of the solve).
  auto certify = [&](double* c) -> int {
    TRY(rotate_out(p, Elt::F64, xbar, W));
    const bool t = p->timing;
    p->timing = t && (p->d.flags & CPHIFI_FLAG_TIME_FP64);
    const int rs = Bm != nullptr ? true_relres_from_B(p, Bm, W, bb_bar, c)
                                 : true_relres(p, b, W, c);
    p->timing = t;
    return rs;
  };
  // ||rbar|| / ||bbar|| (||bbar||^2 sits in scratch[1] of sc2).
  auto rbar_rel = [&](double* out) -> int {
    TRY(launch_dot(rbar, rbar, len, p->red[0], &nb, nullptr, p->st));
    TRY(launch_store_sum(p->red[0], nb, p->sc2, 0, p->st));
    TRY(poll(p, p->sc2));
    const double rr = p->h_sc->scratch[0], bb = p->h_sc->scratch[1];
    bb_bar = bb;
    *out = bb > 0.0 ? std::sqrt(rr / bb) : (rr > 0.0 ? INFINITY : 0.0);
    return CPHIFI_OK;
  };
  // Set once a certificate has missed: the eigenbasis residual then disagrees
  // with the residual of the original system (e.g. eigenpairs that are not
  // those of K to working accuracy), and every later step starts from the
  // certificate's own residual b - A W, rotated by U^T.
  bool true_res = false;
  double last_step_tol = 0.0;  // none yet: a warm start's first residual is FP64
  TRY(join_setup(p));  // the inner PCG applies the eq. fx preconditioner
  for (;;) {
    // The residual of xbar in the eigenbasis.
    bool certified = false;
    if (fresh) {
      TRY(launch_copy(rbar, bbar, len, p->st));
    } else if (true_res || (std::isfinite(rel_prev) && rel_prev > 0.0 &&
                            rel * (rel / rel_prev) <= kCertifyFirst * p->d.tol)) {
      // The contraction of the last step predicts convergence: certify
      // W = U xbar at once (one pass over U_K, two over K) rather than first
      // forming the rotated residual (two passes over U_K).  Should the
      // certificate miss, its residual b - A W rotated by U^T (one pass) is
      // the next step's right-hand side.
      TRY(certify(&cert));
      certified = true;
      if (!std::isfinite(cert)) {
        status = CPHIFI_NUMERIC;
        break;
      }
      if (cert <= p->d.tol || k >= max_refine) {
        status = cert <= p->d.tol ? CPHIFI_OK : CPHIFI_NOT_CONVERGED;
        rel = cert;  // = ||U^T (b - A W)|| / ||b|| up to rounding
        break;
      }
      true_res = true;
      TRY(rotate_in(p, Elt::F64, p->vec[V_RF], rbar));
    } else {
      // FP32 when the residual is predicted large enough (kF32Residual)
      const Elt re = p->ut32 != nullptr && last_step_tol > 0.0 &&
                             rel * last_step_tol >= kF32Residual
                         ? Elt::F32
                         : Elt::F64;
      TRY(op_apply_eig(p, re, xbar, p->vec[V_Q], nullptr, nullptr, nullptr));
      TRY(launch_copy(rbar, bbar, len, p->st));
      TRY(launch_axpby(rbar, -1.0, p->vec[V_Q], 1.0, len, nullptr, p->st));
    }
    rel_prev = rel;
    TRY(rbar_rel(&rel));
    if (!std::isfinite(rel)) {
      status = CPHIFI_NUMERIC;
      break;
    }
    if (!certified && (rel <= p->d.tol || k >= max_refine)) {
      TRY(certify(&cert));
      if (!std::isfinite(cert)) {
        status = CPHIFI_NUMERIC;
        break;
      }
      if (cert <= p->d.tol || k >= max_refine) {
        status = cert <= p->d.tol ? CPHIFI_OK : CPHIFI_NOT_CONVERGED;
        break;
      }
      // the rotated residual met tol, the certificate did not: refine on
      // from the certificate's residual
      true_res = true;
      TRY(rotate_in(p, Elt::F64, p->vec[V_RF], rbar));
      TRY(rbar_rel(&rel));
      if (!std::isfinite(rel)) {
        status = CPHIFI_NUMERIC;
        break;
      }
    }
    // the default inner tolerance is loosened for the steps that cannot reach
    // tol anyway (kInnerLoose); an explicit one holds for every step
    const double step_tol = (p->d.inner_tol <= 0.0 && rel * kInnerLoose > p->d.tol)
                                ? std::max(inner_tol, kInnerLoose)
                                : inner_tol;
    PcgOut o;
    TRY(run_pcg(p, A, M, rbar, p->vec[V_XB], false, step_tol, maxit,
                PcgVecs{p->vec[V_R2], p->vec[V_Z2], p->vec[V_P2], p->vec[V_Q2]}, p->sc, nullptr,
                0, &o, true));
    last_step_tol = step_tol;
    total_inner += o.iters;
    if (o.status == CPHIFI_NUMERIC) {
      status = CPHIFI_NUMERIC;
      break;
    }
    TRY(launch_axpby(xbar, 1.0, p->vec[V_XB], 1.0, len, nullptr, p->st));
    ++k;
    fresh = false;
  }
  info->iters = total_inner;
  info->refine_steps = k;
  info->relres_true = cert;
  info->relres_recursive = rel;
  TRY(timing_collect(p, &info->gemm_ms, &info->gemm_launches));
  info->status = status;
  return status;
}

int validate_desc(const cphifi_ui_desc* d) {
  if (d == nullptr) {
    set_error("desc is NULL");
    return CPHIFI_INVALID_ARG;
  }
  if (d->n < 1 || d->r < 1 || d->r > kMaxRank || d->q < 0 || d->q > INT32_MAX ||
      d->n > INT32_MAX) {
    set_error("bad sizes n=%lld r=%lld q=%lld (need n >= 1, 1 <= r <= 64, 0 <= q < 2^31)",
              (long long)d->n, (long long)d->r, (long long)d->q);
    return CPHIFI_INVALID_ARG;
  }
  if (d->ldk != 0 && d->ldk < d->n) {
    set_error("ldk=%lld < n=%lld", (long long)d->ldk, (long long)d->n);
    return CPHIFI_INVALID_ARG;
  }
  // Section 4.1 adds the shift rho > 0 so that the system matrix is
  // definite for any observation set (K may be singular); the preconditioner's
  // diagonal 1 / (gamma dV dK^2 + lambda dK + rho) needs it too.
  if (!(d->lambda > 0.0) || !(d->rho > 0.0) || !std::isfinite(d->lambda) ||
      !std::isfinite(d->rho)) {
    set_error("need lambda > 0 and rho > 0 (lambda=%g rho=%g)", d->lambda, d->rho);
    return CPHIFI_INVALID_ARG;
  }
  if (!(d->tol > 0.0)) {
    set_error("need tol > 0");
    return CPHIFI_INVALID_ARG;
  }
  if (d->precision != CPHIFI_FP64 && d->precision != CPHIFI_MIXED_FP32 &&
      d->precision != CPHIFI_MIXED_BF16) {
    set_error("unknown precision %d", d->precision);
    return CPHIFI_INVALID_ARG;
  }
  if (d->precision != CPHIFI_FP64 && (d->flags & CPHIFI_FLAG_NO_PRECOND)) {
    set_error("FLAG_NO_PRECOND is only available with CPHIFI_FP64");
    return CPHIFI_INVALID_ARG;
  }
  if ((d->flags & CPHIFI_FLAG_FIBER_COLLAPSE) && (d->I < 1 || d->J < 1)) {
    set_error("FLAG_FIBER_COLLAPSE needs the implicit factor form (I, J >= 1)");
    return CPHIFI_INVALID_ARG;
  }
  return CPHIFI_OK;
}

// Optional tile override "mw,s,ksplit" from the environment (tuning sweeps).
GemmPlan plan_from_env(const char* var, Elt elt, bool trans, int64_t n, int r,
                       const GemmPlan& dflt, int num_cu) {
  const char* s = std::getenv(var);
  if (s == nullptr) return dflt;
  int mw = 0, ss = 0, ks = 0;
  if (std::sscanf(s, "%d,%d,%d", &mw, &ss, &ks) < 2 || !gemm_cfg_valid(elt, mw, ss)) return dflt;
  return make_gemm_plan(elt, trans, n, r, mw, ss, ks, num_cu);
}

// out <- B(s,:) = sum_{l in seg(s)} y_l Zhat(l,:), the observed MTTKRP.
int mttkrp(cphifi_plan* p, const double* y, double* out) {
  ObsArgs a{};
  a.n = p->n;
  a.r = (int)p->r;
  a.obs_i = p->in.obs_i;
  a.obs_j = p->in.obs_j;
  a.A = p->in.A;
  a.B = p->in.B;
  a.Zhat = p->in.Zhat;
  a.y = y;
  a.out = out;
  a.tpart = p->tpart;
  a.done = nullptr;
  return launch_obs(ObsMode::Mttkrp, false, p->tasks, a, p->I, p->J, p->st);
}

// Pinned host memory, events and side stream of a plan.
void release_host(cphifi_plan* p) {
  if (p->side != nullptr) {
    (void)hipStreamSynchronize(p->side);
    (void)hipStreamDestroy(p->side);
    p->side = nullptr;
  }
  for (hipEvent_t* e : {&p->fork_ev, &p->join_ev})
    if (*e != nullptr) (void)hipEventDestroy(*e), *e = nullptr;
  for (hipEvent_t& e : p->pev)
    if (e != nullptr) (void)hipEventDestroy(e), e = nullptr;
  if (p->h_flag) (void)hipHostFree(p->h_flag);
  if (p->h_sc) (void)hipHostFree(p->h_sc);
  p->h_flag = p->d_flag = nullptr;
  p->h_sc = p->d_sc = nullptr;
}

// The side stream and its two events, made on first use (plans that serve
// only the batched solver never need them).  False if they cannot be made:
// the setup then runs in order on the plan's stream.
bool make_side(cphifi_plan* p) {
  if (p->side != nullptr) return true;
  // on the plan's device, whichever is current
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess ||
      (cur != p->device && hipSetDevice(p->device) != hipSuccess)) {
    (void)hipGetLastError();
    return false;
  }
  bool ok = hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&p->join_ev, hipEventDisableTiming) == hipSuccess &&
            // default priority, like every stream of the library
            hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) == hipSuccess;
  if (cur != p->device) (void)hipSetDevice(cur);
  if (!ok) {
    (void)hipGetLastError();  // leave no error for the next launch check
    for (hipEvent_t* e : {&p->fork_ev, &p->join_ev})
      if (*e != nullptr) (void)hipEventDestroy(*e), *e = nullptr;
    p->side = nullptr;
  }
  return ok;
}

// Per-solve setup: V = (A^T A) had (B^T B) (or the given V), its eigenpairs,
// the eq. fx diagonal D, and the copies and clamps the operators read.  With
// overlap, the V chain (one workgroup for the Jacobi sweeps: ~0.4 ms at
// r = 40) runs on the side stream, forked from the plan's stream, and the
// caller must call join_setup before the first preconditioner application;
// the rest of the setup and the right-hand side go on meanwhile.
int setup_plan(cphifi_plan* p, bool overlap) {
  const int r = (int)p->r;
  TRY(join_setup(p));  // a chain still in flight writes what this one writes
  hipStream_t vs = p->st;
  if (overlap && make_side(p)) {
    CPHIFI_HIP(hipEventRecord(p->fork_ev, p->st));
    CPHIFI_HIP(hipStreamWaitEvent(p->side, p->fork_ev, 0));
    vs = p->side;
  }
  int rc = p->in.V != nullptr ? launch_copy(p->V, p->in.V, (int64_t)r * r, vs)
                              : launch_gram(p->in.A, p->I, p->in.B, p->J, r, p->V, vs);
  if (rc == CPHIFI_OK) rc = launch_jacobi_eig(p->V, r, p->UV, p->dV, vs);
  if (rc == CPHIFI_OK)
    rc = launch_precond_diag(p->in.dK, p->dV, p->n, r, p->gamma, p->d.lambda, p->d.rho, p->D,
                             vs);
  if (vs != p->st) {
    // join whatever was enqueued, also after a failed launch
    CPHIFI_HIP(hipEventRecord(p->join_ev, vs));
    p->join_pending = true;
  }
  TRY(rc);
  // The FP32 factor copies of the low-precision gather follow A and B, which
  // may have changed since the plan was made (alternating optimisation).
  if (p->fgram != nullptr) TRY(launch_fiber_gram(p->in.B, p->J, r, p->fgram, p->st));
  if (p->a32 != nullptr) {
    TRY(launch_to_f32(p->a32, p->in.A, p->I * r, p->st));
    TRY(launch_to_f32(p->b32, p->in.B, p->J * r, p->st));
  }
  TRY(launch_clamp_nonneg(p->in.dK, p->dKc, p->n, p->st));
  p->setup_done = true;
  return CPHIFI_OK;
}

}  // namespace

// ======================================================================= C ABI
extern "C" {

const char* cphifi_status_string(int status) {
  switch (status) {
    case CPHIFI_OK: return "CPHIFI_OK";
    case CPHIFI_INVALID_ARG: return "CPHIFI_INVALID_ARG";
    case CPHIFI_HIP_ERROR: return "CPHIFI_HIP_ERROR";
    case CPHIFI_UNSUPPORTED: return "CPHIFI_UNSUPPORTED";
    case CPHIFI_BREAKDOWN: return "CPHIFI_BREAKDOWN";
    case CPHIFI_NUMERIC: return "CPHIFI_NUMERIC";
    case CPHIFI_NOT_CONVERGED: return "CPHIFI_NOT_CONVERGED";
  }
  return "CPHIFI_UNKNOWN";
}

const char* cphifi_last_error(void) { return g_last_error.c_str(); }

const char* cphifi_version(void) { return "cphifi 0.1.0 gfx950"; }

int cphifi_ui_workspace_bytes(const cphifi_ui_desc* d, size_t* bytes) {
  clear_error();
  if (bytes == nullptr) {
    set_error("bytes is NULL");
    return CPHIFI_INVALID_ARG;
  }
  TRY(validate_desc(d));
  *bytes = make_layout(*d).total;
  return CPHIFI_OK;
}

int cphifi_ui_plan_create(cphifi_plan** out, const cphifi_ui_desc* d, const cphifi_ui_inputs* in,
                          void* workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  if (out == nullptr || in == nullptr) {
    set_error("out / inputs is NULL");
    return CPHIFI_INVALID_ARG;
  }
  *out = nullptr;
  TRY(validate_desc(d));
  const bool expl = in->Zhat != nullptr;
  if (in->K == nullptr || in->UK == nullptr || in->dK == nullptr || in->obs_ptr == nullptr) {
    set_error("K, UK, dK and obs_ptr are required");
    return CPHIFI_INVALID_ARG;
  }
  if (expl) {
    if (in->A != nullptr || in->B != nullptr) {
      set_error("give either Zhat or (A, B), not both");
      return CPHIFI_INVALID_ARG;
    }
    if (in->V == nullptr) {
      set_error("the explicit Zhat form needs V (the full Khatri-Rao Gram)");
      return CPHIFI_INVALID_ARG;
    }
  } else {
    if (in->A == nullptr || in->B == nullptr || d->I < 1 || d->J < 1) {
      set_error("the implicit form needs A (I x r), B (J x r) with I, J >= 1");
      return CPHIFI_INVALID_ARG;
    }
    if (d->q > 0 && (in->obs_i == nullptr || in->obs_j == nullptr)) {
      set_error("obs_i / obs_j are required");
      return CPHIFI_INVALID_ARG;
    }
  }
  const Layout L = make_layout(*d);
  if (workspace == nullptr || workspace_bytes < L.total ||
      (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) {
    set_error("workspace must be >= %zu bytes and 256-byte aligned (got %zu)", L.total,
              workspace_bytes);
    return CPHIFI_INVALID_ARG;
  }
  const int64_t n = d->n, q = d->q;
  hipStream_t st = (hipStream_t)stream;

  // Observation CSR: check it on the host and build the task list.
  std::vector<int32_t> ptr(n + 1);
  CPHIFI_HIP(hipMemcpyAsync(ptr.data(), in->obs_ptr, sizeof(int32_t) * (n + 1),
                            hipMemcpyDeviceToHost, st));
  CPHIFI_HIP(hipStreamSynchronize(st));
  if (ptr[0] != 0 || ptr[n] != q) {
    set_error("obs_ptr must start at 0 and end at q=%lld (got %d .. %d)", (long long)q, ptr[0],
              ptr[n]);
    return CPHIFI_INVALID_ARG;
  }
  for (int64_t s = 0; s < n; ++s)
    if (ptr[s + 1] < ptr[s]) {
      set_error("obs_ptr decreases at %lld", (long long)s);
      return CPHIFI_INVALID_ARG;
    }
  bool owner = false;
  std::vector<int32_t> oi, oj;
  if (!expl && q > 0) {
    // Both index arrays are always range-checked here (the gather clamps an
    // index to stay in bounds, which would otherwise turn a bad index into a
    // wrong answer with status OK).
    oi.resize(q);
    oj.resize(q);
    CPHIFI_HIP(hipMemcpyAsync(oi.data(), in->obs_i, sizeof(int32_t) * q, hipMemcpyDeviceToHost,
                              st));
    CPHIFI_HIP(hipMemcpyAsync(oj.data(), in->obs_j, sizeof(int32_t) * q, hipMemcpyDeviceToHost,
                              st));
    CPHIFI_HIP(hipStreamSynchronize(st));
    for (int64_t l = 0; l < q; ++l)
      if (oi[l] < 0 || oi[l] >= d->I || oj[l] < 0 || oj[l] >= d->J) {
        set_error("observation %lld has index (%d, %d) outside I=%lld, J=%lld", (long long)l,
                  oi[l], oj[l], (long long)d->I, (long long)d->J);
        return CPHIFI_INVALID_ARG;
      }
    // one sample per time point (the unaligned setting)?
    owner = true;
    for (int64_t s = 0; s < n && owner; ++s)
      for (int32_t l = ptr[s] + 1; l < ptr[s + 1]; ++l)
        if (oi[l] != oi[ptr[s]]) {
          owner = false;
          break;
        }
  }
  std::vector<int32_t> tseg, tbeg, tend, tslot, tfirst, mseg, mptr, rowm(n, -1);
  int32_t nslot = 0;
  for (int64_t s = 0; s < n; ++s) {
    const int32_t b0 = ptr[s], e0 = ptr[s + 1];
    const int32_t cnt = e0 - b0;
    const int32_t nt = std::max<int32_t>(1, (cnt + kObsChunk - 1) / kObsChunk);
    if (nt > 1) rowm[s] = (int32_t)mseg.size();
    if (nt == 1) {
      tseg.push_back((int32_t)s);
      tbeg.push_back(b0);
      tend.push_back(e0);
      tslot.push_back(-1);
      tfirst.push_back(1);
    } else {
      mseg.push_back((int32_t)s);
      mptr.push_back(nslot);
      for (int32_t j = 0; j < nt; ++j) {
        tseg.push_back((int32_t)s);
        tbeg.push_back(b0 + j * kObsChunk);
        tend.push_back(std::min<int32_t>(e0, b0 + (j + 1) * kObsChunk));
        tslot.push_back(nslot++);
        tfirst.push_back(j == 0 ? 1 : 0);
      }
    }
  }
  mptr.push_back(nslot);
  // Fiber collapse: every (time, sample) pair observed at all must be observed
  // at each of the J features exactly once.  Fibers of a time point are listed
  // in ascending sample order (a fixed summation order).
  std::vector<int32_t> fptr, fidx;
  int32_t fmax = 0;
  if (d->flags & CPHIFI_FLAG_FIBER_COLLAPSE) {
    const int64_t J = d->J;
    fptr.assign(n + 1, 0);
    std::vector<int32_t> cnt(d->I, 0);
    std::vector<uint8_t> seen((size_t)d->I * J, 0);
    std::vector<int32_t> samples;
    for (int64_t s = 0; s < n; ++s) {
      samples.clear();
      for (int32_t l = ptr[s]; l < ptr[s + 1]; ++l) {
        const size_t key = (size_t)oi[l] * J + oj[l];
        if (seen[key]) {
          set_error("FLAG_FIBER_COLLAPSE: (time %lld, sample %d, feature %d) observed twice",
                    (long long)s, oi[l], oj[l]);
          return CPHIFI_INVALID_ARG;
        }
        seen[key] = 1;
        if (cnt[oi[l]]++ == 0) samples.push_back(oi[l]);
      }
      std::sort(samples.begin(), samples.end());
      for (int32_t i : samples) {
        if (cnt[i] != J) {
          set_error("FLAG_FIBER_COLLAPSE: (time %lld, sample %d) has %d of the %lld features",
                    (long long)s, i, cnt[i], (long long)J);
          return CPHIFI_INVALID_ARG;
        }
        fidx.push_back(i);
        cnt[i] = 0;
      }
      for (int32_t l = ptr[s]; l < ptr[s + 1]; ++l) seen[(size_t)oi[l] * J + oj[l]] = 0;
      fptr[s + 1] = (int32_t)fidx.size();
      fmax = std::max<int32_t>(fmax, fptr[s + 1] - fptr[s]);
    }
    if ((int64_t)fidx.size() > q / J + 1) {
      set_error("internal: fiber list exceeds its bound");
      return CPHIFI_INVALID_ARG;
    }
  }
  const int64_t ntask = (int64_t)tseg.size();
  if (ntask > L.ntask_max || nslot > L.nslot_max || (int64_t)mseg.size() > L.nmulti_max) {
    set_error("internal: observation task list exceeds its bound");
    return CPHIFI_INVALID_ARG;
  }

  cphifi_plan* p = new cphifi_plan();
  p->d = *d;
  p->in = *in;
  p->st = st;
  p->n = n;
  p->r = d->r;
  p->q = q;
  p->ldk = eff_ldk(*d);
  p->I = expl ? 0 : d->I;
  p->J = expl ? 0 : d->J;
  p->ldp = (int)round_up(d->r, 16);
  p->L = L;
  p->ws = (char*)workspace;
  p->timing = (d->flags & CPHIFI_FLAG_TIME_KERNELS) != 0;
  if (d->gamma > 0.0) {
    p->gamma = d->gamma;
  } else if (!expl) {
    p->gamma = (double)q / ((double)n * (double)d->I * (double)d->J);
  } else {
    delete p;
    set_error("gamma must be given (> 0) with the explicit Zhat form");
    return CPHIFI_INVALID_ARG;
  }
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    p->device = dev;
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cu > 0)
      p->num_cu = cu;
  }
  char* ws = p->ws;
  for (int i = 0; i < NVEC; ++i) p->vec[i] = (double*)(ws + L.vec[i]);
  p->part = ws + L.part;
  p->tpart = (double*)(ws + L.tpart);
  for (int i = 0; i < 3; ++i) p->red[i] = (double*)(ws + L.red[i]);
  p->sc = (DevScalars*)(ws + L.sc);
  p->sc2 = (DevScalars*)(ws + L.sc2);
  p->hist = (double*)(ws + L.hist);
  p->V = (double*)(ws + L.V);
  p->UV = (double*)(ws + L.UV);
  p->dV = (double*)(ws + L.dV);
  p->D = (double*)(ws + L.D);
  p->dKc = (double*)(ws + L.dKc);
  p->tasks.ntask = (int32_t)ntask;
  p->tasks.nmulti = (int32_t)mseg.size();
  p->tasks.seg = (int32_t*)(ws + L.tseg);
  p->tasks.beg = (int32_t*)(ws + L.tbeg);
  p->tasks.end = (int32_t*)(ws + L.tend);
  p->tasks.slot = (int32_t*)(ws + L.tslot);
  p->tasks.first = (int32_t*)(ws + L.tfirst);
  p->tasks.mseg = (int32_t*)(ws + L.mseg);
  p->tasks.mptr = (int32_t*)(ws + L.mptr);
  // One lane row per segment instead of one wave per segment when no segment
  // is split and the segments are short (at most kShortSegment observations
  // on average) or of nearly equal length (the longest at most 5/4 of the
  // mean), so the rows of a wave finish together: each segment's setup (its
  // indices, A row and Xhat row) then overlaps with 64/L - 1 others.
  int64_t maxlen = 0;
  for (int64_t s = 0; s < n; ++s) maxlen = std::max<int64_t>(maxlen, ptr[s + 1] - ptr[s]);
  p->tasks.rows = mseg.empty() && (q <= kShortSegment * n || 4 * maxlen * n <= 5 * q);
  p->tasks.obs_ptr = in->obs_ptr;
  p->tasks.nseg = n;
  p->tasks.owner = owner;
  p->rowm = (int32_t*)(ws + L.rowm);

  auto fail = [&](int code) {
    release_host(p);
    delete p;
    return code;
  };
  auto up = [&](int32_t* dst, const std::vector<int32_t>& v) -> int {
    if (v.empty()) return CPHIFI_OK;
    CPHIFI_HIP(hipMemcpyAsync(dst, v.data(), sizeof(int32_t) * v.size(), hipMemcpyHostToDevice,
                              st));
    return CPHIFI_OK;
  };
  if (hipHostMalloc((void**)&p->h_sc, sizeof(DevScalars),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    p->h_sc = nullptr;
    set_error("hipHostMalloc of the scalar mirror failed");
    return fail(CPHIFI_HIP_ERROR);
  }
  if (hipHostGetDevicePointer((void**)&p->d_sc, p->h_sc, 0) != hipSuccess) {
    set_error("hipHostGetDevicePointer of the scalar mirror failed");
    return fail(CPHIFI_HIP_ERROR);
  }
  if (hipHostMalloc((void**)&p->h_flag, 64, hipHostMallocMapped | hipHostMallocCoherent) !=
      hipSuccess) {
    p->h_flag = nullptr;
    set_error("hipHostMalloc of the convergence flag failed");
    return fail(CPHIFI_HIP_ERROR);
  }
  if (hipHostGetDevicePointer((void**)&p->d_flag, p->h_flag, 0) != hipSuccess) {
    set_error("hipHostGetDevicePointer of the convergence flag failed");
    return fail(CPHIFI_HIP_ERROR);
  }
  *(volatile int32_t*)p->h_flag = 0;
  for (int i = 0; i < kPollRing; ++i)
    if (hipEventCreateWithFlags(&p->pev[i], hipEventDisableTiming) != hipSuccess) {
      p->pev[i] = nullptr;
      set_error("hipEventCreateWithFlags failed");
      return fail(CPHIFI_HIP_ERROR);
    }
  int rc = CPHIFI_OK;
  if ((rc = up(p->tasks.seg, tseg)) || (rc = up(p->tasks.beg, tbeg)) ||
      (rc = up(p->tasks.end, tend)) || (rc = up(p->tasks.slot, tslot)) ||
      (rc = up(p->tasks.first, tfirst)) || (rc = up(p->tasks.mseg, mseg)) ||
      (rc = up(p->tasks.mptr, mptr)) || (rc = up(p->rowm, rowm)))
    return fail(rc);

  const int rr = (int)d->r;
  p->gp64n = plan_from_env("CPHIFI_TILE_F64", Elt::F64, false, n, rr,
                           choose_gemm(Elt::F64, false, n, rr, p->num_cu), p->num_cu);
  p->gp64t = plan_from_env("CPHIFI_TILE_F64T", Elt::F64, true, n, rr,
                           choose_gemm(Elt::F64, true, n, rr, p->num_cu), p->num_cu);
  p->small = small_plan(*d);
  if (d->flags & CPHIFI_FLAG_FIBER_COLLAPSE) {
    p->fptr = (int32_t*)(ws + L.fptr);
    p->fidx = (int32_t*)(ws + L.fidx);
    p->fgram = (double*)(ws + L.fgram);
    p->fmax = fmax;
    if ((rc = up(p->fptr, fptr)) || (rc = up(p->fidx, fidx))) return fail(rc);
    // G = B^T B now (the operator may be applied before any setup), and again
    // at every setup (B may change between solves)
    if ((rc = launch_fiber_gram(in->B, d->J, (int)d->r, p->fgram, st))) return fail(rc);
  }
  if (d->flags & CPHIFI_FLAG_TOEPLITZ_K) {
    // c = the first row of K; the plan is refused unless every entry of K is
    // c(|s - k|) to within 1e-12 max|c| (a kernel evaluated on a rounded
    // uniform grid matches along its diagonals only to rounding).
    p->toep = (double*)(ws + L.toep);
    std::vector<double> c(n);
    if (hipMemcpyAsync(p->toep, in->K, sizeof(double) * n, hipMemcpyDeviceToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(c.data(), in->K, sizeof(double) * n, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("plan_create: copy of the first row of K failed");
      return fail(CPHIFI_HIP_ERROR);
    }
    double cmax = 0.0;
    for (double v : c) cmax = std::max(cmax, std::fabs(v));
    *(volatile int32_t*)p->h_flag = 0;
    if ((rc = launch_toeplitz_check(in->K, p->ldk, n, p->toep, 1e-12 * cmax, p->d_flag, st)))
      return fail(rc);
    if (hipStreamSynchronize(st) != hipSuccess) {
      set_error("plan_create: Toeplitz check failed to run");
      return fail(CPHIFI_HIP_ERROR);
    }
    if (*(volatile int32_t*)p->h_flag != 0) {
      *(volatile int32_t*)p->h_flag = 0;
      set_error("FLAG_TOEPLITZ_K: K is not symmetric Toeplitz to within 1e-12 max|K(0,:)|");
      return fail(CPHIFI_INVALID_ARG);
    }
  }
  if (keeps_ukt(*d)) {
    p->ukt = (double*)(ws + L.ukt);
    if ((rc = launch_convert_lowp(Elt::F64, true, in->UK, p->ldk, n, p->ukt, p->ldk, st)))
      return fail(rc);
  }
  // timed kernel (CPHIFI_FLAG_TIME_KERNELS): FP64 plans time the transposed FP64
  // products (K X and U_K X, three of the four per iteration), mixed plans the
  // low-precision ones
  p->timed_trans = d->precision == CPHIFI_FP64;
  if (d->precision != CPHIFI_FP64 && in->A != nullptr && L.a32 != 0) {
    p->a32 = (float*)(ws + L.a32);
    p->b32 = (float*)(ws + L.b32);
    if ((rc = launch_to_f32(p->a32, in->A, d->I * d->r, st)) ||
        (rc = launch_to_f32(p->b32, in->B, d->J * d->r, st)))
      return fail(rc);
  }
  if (d->precision == CPHIFI_MIXED_BF16) {
    p->lp = Elt::BF16;
    p->timed_elt = Elt::BF16;
    p->ulp = ws + L.ulp;
    p->utlp = ws + L.utlp;
    p->xthi = (__bf16*)(ws + L.xthi);
    p->xtlo = (__bf16*)(ws + L.xtlo);
    p->gplpn = bf16_stream_k(plan_from_env("CPHIFI_TILE_BF16", Elt::BF16, false, n, rr,
                                           choose_gemm(Elt::BF16, false, n, rr, p->num_cu),
                                           p->num_cu),
                             n, p->num_cu);
    if ((rc = launch_convert_lowp(Elt::BF16, false, in->UK, p->ldk, n, p->utlp, L.ldl, st,
                                  true)) ||
        (rc = launch_convert_lowp(Elt::BF16, true, in->UK, p->ldk, n, p->ulp, L.ldl, st, true)))
      return fail(rc);
    if (keeps_ut32(*d)) {
      p->ut32 = (float*)(ws + L.ut32);
      p->gp32n = choose_gemm(Elt::F32, false, n, rr, p->num_cu);
      p->gp32t = choose_gemm(Elt::F32, true, n, rr, p->num_cu);
      if ((rc = launch_convert_lowp(Elt::F32, false, in->UK, p->ldk, n, p->ut32, L.ldl, st)))
        return fail(rc);
    }
  } else if (d->precision == CPHIFI_MIXED_FP32) {
    p->lp = Elt::F32;
    p->timed_elt = Elt::F32;
    p->utlp = ws + L.utlp;
    p->gplpn = plan_from_env("CPHIFI_TILE_F32", Elt::F32, false, n, rr,
                             choose_gemm(Elt::F32, false, n, rr, p->num_cu), p->num_cu);
    p->gplpt = plan_from_env("CPHIFI_TILE_F32T", Elt::F32, true, n, rr,
                             choose_gemm(Elt::F32, true, n, rr, p->num_cu), p->num_cu);
    if ((rc = launch_convert_lowp(Elt::F32, false, in->UK, p->ldk, n, p->utlp, L.ldl, st)))
      return fail(rc);
  }
  if (d->flags & CPHIFI_FLAG_TIME_FP64) {
    p->timed_elt = Elt::F64;
    p->timed_trans = true;
  }
  // scalars start in a defined state
  if ((rc = launch_fill((double*)p->sc, 0.0, sizeof(DevScalars) / sizeof(double), st)) ||
      (rc = launch_fill((double*)p->sc2, 0.0, sizeof(DevScalars) / sizeof(double), st)))
    return fail(rc);
  if (hipStreamSynchronize(st) != hipSuccess) {
    set_error("plan_create: stream synchronisation failed");
    return fail(CPHIFI_HIP_ERROR);
  }
  *out = p;
  return CPHIFI_OK;
}

int cphifi_ui_setup(cphifi_plan* p) {
  clear_error();
  if (p == nullptr) {
    set_error("plan is NULL");
    return CPHIFI_INVALID_ARG;
  }
  return setup_plan(p, false);
}

int cphifi_ui_rhs(cphifi_plan* p, const double* y, double* b) {
  clear_error();
  if (p == nullptr || b == nullptr || (y == nullptr && p->q > 0)) {
    set_error("rhs: NULL argument");
    return CPHIFI_INVALID_ARG;
  }
  TRY(mttkrp(p, y, p->vec[V_Y1]));
  const bool t = p->timing;
  p->timing = false;
  const int rc = prod_K(p, p->vec[V_Y1], nullptr);
  p->timing = t;
  TRY(rc);
  return launch_reduce_partials(p->part, false, p->last_ksplit, p->ldp, p->n, (int)p->r, b,
                                nullptr, nullptr, nullptr, nullptr, p->st);
}

int cphifi_ui_mttkrp(cphifi_plan* p, const double* y, double* Bm) {
  clear_error();
  if (p == nullptr || Bm == nullptr || (y == nullptr && p->q > 0)) {
    set_error("mttkrp: NULL argument");
    return CPHIFI_INVALID_ARG;
  }
  return mttkrp(p, y, Bm);
}

int cphifi_ui_apply(cphifi_plan* p, const double* x, double* y) {
  clear_error();
  if (p == nullptr || x == nullptr || y == nullptr || x == y) {
    set_error("apply: bad arguments");
    return CPHIFI_INVALID_ARG;
  }
  return op_apply_paper(p, x, y, nullptr, nullptr, nullptr);
}

int cphifi_ui_precond(cphifi_plan* p, const double* x, double* z) {
  clear_error();
  if (p == nullptr || x == nullptr || z == nullptr || x == z) {
    set_error("precond: bad arguments");
    return CPHIFI_INVALID_ARG;
  }
  if (!p->setup_done) {
    set_error("precond: call cphifi_ui_setup first");
    return CPHIFI_INVALID_ARG;
  }
  return op_precond_paper(p, x, z, nullptr, nullptr, nullptr);
}

int cphifi_ui_apply_lowp(cphifi_plan* p, const double* xbar, double* ybar) {
  clear_error();
  if (p == nullptr || xbar == nullptr || ybar == nullptr || xbar == ybar) {
    set_error("apply_lowp: bad arguments");
    return CPHIFI_INVALID_ARG;
  }
  TRY(launch_clamp_nonneg(p->in.dK, p->dKc, p->n, p->st));
  return op_apply_eig(p, p->lp, xbar, ybar, nullptr, nullptr, nullptr);
}

int cphifi_ui_solve(cphifi_plan* p, const double* b, double* W, cphifi_solve_info* info) {
  clear_error();
  if (p == nullptr || b == nullptr || W == nullptr || info == nullptr || b == W) {
    set_error("solve: bad arguments");
    return CPHIFI_INVALID_ARG;
  }
  if (!p->setup_done) {
    set_error("solve: call cphifi_ui_setup first");
    return CPHIFI_INVALID_ARG;
  }
  double* hist = info->history;
  std::memset(info, 0, sizeof(*info));
  info->history = hist;
  p->ev_used = 0;
  if (p->d.precision == CPHIFI_FP64) {
    TRY(join_setup(p));
    return solve_fp64(p, b, W, info);
  }
  return solve_mixed(p, b, nullptr, W, info);
}

int cphifi_ui_solve_subproblem(cphifi_plan* p, const double* y, double* W,
                               cphifi_solve_info* info) {
  clear_error();
  if (p == nullptr || W == nullptr || info == nullptr) {
    set_error("solve_subproblem: bad arguments");
    return CPHIFI_INVALID_ARG;
  }
  if (p->d.precision != CPHIFI_FP64 && y == nullptr && p->q > 0) {
    set_error("solve_subproblem: y is NULL");
    return CPHIFI_INVALID_ARG;
  }
  // The setup's eig(V) chain overlaps the right-hand side (the gather and
  // one n x n pass); the solves join it before their first preconditioner
  // application, and every return joins it, so nothing of this call is left
  // outside the plan's stream.
  int rc = setup_plan(p, true);
  if (rc == CPHIFI_OK) {
    if (p->d.precision == CPHIFI_FP64) {
      rc = cphifi_ui_rhs(p, y, p->vec[V_B]);
      if (rc == CPHIFI_OK) rc = cphifi_ui_solve(p, p->vec[V_B], W, info);
    } else {
      // Mixed forms: the refinement starts from Bm (no pass over K for b).
      rc = mttkrp(p, y, p->vec[V_B]);
      if (rc == CPHIFI_OK) {
        double* hist = info->history;
        std::memset(info, 0, sizeof(*info));
        info->history = hist;
        p->ev_used = 0;
        rc = solve_mixed(p, nullptr, p->vec[V_B], W, info);
      }
    }
  }
  const int rj = join_setup(p);
  return rc != CPHIFI_OK ? rc : rj;
}

int cphifi_ui_plan_destroy(cphifi_plan* p) {
  clear_error();
  if (p == nullptr) return CPHIFI_OK;
  if (p->pcg_graph != nullptr) (void)hipGraphExecDestroy(p->pcg_graph);
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  release_host(p);
  delete p;
  return CPHIFI_OK;
}

}  // extern "C"
