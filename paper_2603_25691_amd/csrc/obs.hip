// Per-observation gather-dot-scatter of the two-step product (Section 4.4.1):
//   xbar_l   = Xhat(t_l, :) . Zhat(l, :)                       (eq. vl)
//   Yhat1(s,:) = sum_{l: t_l = s} xbar_l Zhat(l, :)              (eq. yhat1)
// and the observed MTTKRP B(s,:) = sum_{l: t_l = s} y_l Zhat(l,:) that feeds the
// right-hand side.  Zhat(l,:) is either read (explicit rows, any tensor order)
// or formed on the fly as A(i_l,:) * B(j_l,:) (3-way Khatri-Rao rows, eq. zhat).
//
// Work unit: one wave per task = (segment s, contiguous observation range).
// Lanes form 64/G groups of G >= r lanes; a group handles one observation per
// step, lane c of the group holding column c.  The dot product of eq. vl is
// a butterfly over the G lanes of the group; the scatter of eq. yhat1 keeps a
// per-lane running sum that is folded across groups once at the end.  Segments
// longer than one task write partial rows that a second kernel adds in order,
// so results are deterministic (no atomics).  xbar never leaves registers.
#include "cphifi_internal.h"

namespace cphifi {
namespace {

struct TaskView {
  const int32_t* seg;
  const int32_t* beg;
  const int32_t* end;
  const int32_t* slot;
  const int32_t* first;
  int32_t ntask;
};

struct ObsDev {
  ObsArgs a;
  int64_t I, J;
};

template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int G, bool EXPL, int MODE, typename PT>
__global__ __launch_bounds__(256) void obs_kernel(TaskView t, ObsDev d) {
  const ObsArgs& a = d.a;
  if (a.done != nullptr && *a.done) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t task = (int64_t)blockIdx.x * 4 + wave;
  if (task >= t.ntask) return;
  constexpr int P = 64 / G;
  const int g = lane / G, c = lane % G;
  const int r = a.r;
  const bool col = c < r;
  const int64_t s = t.seg[task];
  const int64_t beg = t.beg[task], end = t.end[task];
  const int32_t slot = t.slot[task];

  double xh = 0.0;
  if (MODE == 0) {
    if (col) {
      const PT* part = (const PT*)a.part;
      for (int sp = 0; sp < a.ksplit; ++sp)
        xh += (double)part[((int64_t)sp * a.n + s) * a.ldp + c];
    }
    if (a.Xhat != nullptr && t.first[task] && g == 0 && col) a.Xhat[s * r + c] = xh;
  }

  double acc = 0.0;
  for (int64_t base = beg; base < end; base += P) {
    const int64_t l = base + g;
    const bool act = l < end;
    double z = 0.0;
    if (act && col) {
      if (EXPL) {
        z = a.Zhat[l * r + c];
      } else {
        const int64_t ii = min<int64_t>(max(a.obs_i[l], 0), d.I - 1);
        const int64_t jj = min<int64_t>(max(a.obs_j[l], 0), d.J - 1);
        z = a.A[ii * r + c] * a.B[jj * r + c];
      }
    }
    double w;
    if (MODE == 0) {
      w = group_sum<G>(z * xh);  // xbar_l, eq. vl
    } else {
      w = act ? a.y[l] : 0.0;
    }
    acc += w * z;  // eq. yhat1 (or the MTTKRP)
  }
#pragma unroll
  for (int off = G; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
  if (g == 0 && col) {
    double* dst = slot < 0 ? a.out + s * r : a.tpart + (int64_t)slot * r;
    dst[c] = acc;
  }
}

// Adds the partial rows of segments that were split over several tasks.
__global__ void segment_reduce_kernel(const int32_t* __restrict__ mseg,
                                      const int32_t* __restrict__ mptr, int32_t nmulti,
                                      const double* __restrict__ tpart, int r,
                                      double* __restrict__ out, const int32_t* done) {
  if (done != nullptr && *done) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t m = (int64_t)blockIdx.x * 4 + wave;
  if (m >= nmulti || lane >= r) return;
  double acc = 0.0;
  for (int32_t k = mptr[m]; k < mptr[m + 1]; ++k) acc += tpart[(int64_t)k * r + lane];
  out[(int64_t)mseg[m] * r + lane] = acc;
}

template <int G, bool EXPL, int MODE>
int launch_g(bool pf, const TaskView& tv, const ObsDev& d, hipStream_t st) {
  const int blocks = (tv.ntask + 3) / 4;
  if (blocks == 0) return CPHIFI_OK;
  if (pf)
    hipLaunchKernelGGL((obs_kernel<G, EXPL, MODE, float>), dim3(blocks), dim3(256), 0, st, tv, d);
  else
    hipLaunchKernelGGL((obs_kernel<G, EXPL, MODE, double>), dim3(blocks), dim3(256), 0, st, tv,
                       d);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

template <bool EXPL, int MODE>
int launch_m(int r, bool pf, const TaskView& tv, const ObsDev& d, hipStream_t st) {
  if (r <= 4) return launch_g<4, EXPL, MODE>(pf, tv, d, st);
  if (r <= 8) return launch_g<8, EXPL, MODE>(pf, tv, d, st);
  if (r <= 16) return launch_g<16, EXPL, MODE>(pf, tv, d, st);
  if (r <= 32) return launch_g<32, EXPL, MODE>(pf, tv, d, st);
  return launch_g<64, EXPL, MODE>(pf, tv, d, st);
}

}  // namespace

int launch_obs(ObsMode mode, bool part_is_float, const ObsTasks& t, const ObsArgs& a,
               int64_t I, int64_t J, hipStream_t st) {
  if (a.r < 1 || a.r > kMaxRank) {
    set_error("launch_obs: bad rank %d", a.r);
    return CPHIFI_INVALID_ARG;
  }
  const bool expl = a.Zhat != nullptr;
  if (!expl && (a.A == nullptr || a.B == nullptr || I < 1 || J < 1)) {
    set_error("launch_obs: implicit factor form needs A, B, I, J");
    return CPHIFI_INVALID_ARG;
  }
  TaskView tv{t.seg, t.beg, t.end, t.slot, t.first, t.ntask};
  ObsDev d{a, I, J};
  int st_ = CPHIFI_OK;
  if (mode == ObsMode::Gather)
    st_ = expl ? launch_m<true, 0>(a.r, part_is_float, tv, d, st)
               : launch_m<false, 0>(a.r, part_is_float, tv, d, st);
  else
    st_ = expl ? launch_m<true, 1>(a.r, part_is_float, tv, d, st)
               : launch_m<false, 1>(a.r, part_is_float, tv, d, st);
  if (st_ != CPHIFI_OK) return st_;
  if (t.nmulti > 0) {
    hipLaunchKernelGGL(segment_reduce_kernel, dim3((t.nmulti + 3) / 4), dim3(256), 0, st, t.mseg,
                       t.mptr, t.nmulti, a.tpart, a.r, a.out, a.done);
    CPHIFI_CHECK_LAUNCH();
  }
  return CPHIFI_OK;
}

}  // namespace cphifi
