// Grid launches of the per-observation gather-dot-scatter (eqs. vl, yhat1) and
// of the observed MTTKRP; the wave tile and its design are in obs_tile.h.
#include "cphifi_internal.h"
#include "obs_tile.h"

#include <cstdlib>

namespace cphifi {
namespace {

using tiles::ObsDev;
using tiles::TaskView;
using tiles::obs_task;

template <int L, int CPL, int FORM, int MODE, typename PT>
__global__ __launch_bounds__(256) void obs_kernel(TaskView t, ObsDev d) {
  if (d.a.done != nullptr && *d.a.done) return;
  const int64_t task = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (task >= t.ntask) return;
  obs_task<L, CPL, FORM, MODE, PT, false, PT>(t, d, task, threadIdx.x & 63);
}

// Lane-row form: wave w takes segments [w spw, (w + 1) spw), 64/L at a time
// (spw a multiple of 64/L, at most kSegPerWave).  In every form the arithmetic
// type is that of the partials: FP64 after an FP64 product, FP32 (with the
// plan's FP32 copies of A and B) after a low-precision one.
template <int L, int CPL, int FORM, int MODE, typename PT>
__global__ __launch_bounds__(256) void obs_rows_kernel(ObsDev d, const int32_t* obs_ptr,
                                                       int64_t n, int spw) {
  if (d.a.done != nullptr && *d.a.done) return;
  constexpr int ROWS = 64 / L;
  const int64_t sb = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * spw;
  for (int k = 0; k < spw; k += ROWS) {
    const int64_t s0 = sb + k;
    if (s0 >= n) break;
    tiles::obs_rows<L, CPL, FORM, MODE, PT, false, PT>(
        d, obs_ptr, s0, (int)min((int64_t)ROWS, n - s0), threadIdx.x & 63);
  }
}

// B (J x r, FP64 or the FP32 copy) staged in LDS once per workgroup, then read
// from there by every observation; the workgroups stride over the tasks (or
// short-segment wave units) so the staging is amortised.  Used in the implicit
// and owner forms when the copy fits the element type's limit: a larger copy
// limits the workgroups per CU.  Measured at J r = 8000 (n = 30658, 200
// observations per time point, lane-row form): FP64, 64000 bytes, two
// workgroups per CU, 116 us against 150 us reading B through L2 (MTTKRP 124
// against 188 us); FP32, 32000 bytes, 66 against 63 us, so FP32 (and the task
// form, not measured at this size) keeps the L2 form above 16 KB.
// CPHIFI_OBS_LDS_BYTES overrides the limits (at most 64 KB).
constexpr int kObsLdsBytesF64 = 65536;
constexpr int kObsLdsBytesF32 = 16384;
constexpr int kObsLdsGrid = 1024;  // workgroups of the staged form (grid-stride)


template <typename T>
__device__ __forceinline__ void stage_rows(T* dst, const T* src, int64_t len) {
  for (int64_t e = threadIdx.x; e < len; e += blockDim.x) dst[e] = src[e];
  __syncthreads();
}

__device__ __forceinline__ const double* factor_b(const ObsDev& d, double) { return d.a.B; }
__device__ __forceinline__ const float* factor_b(const ObsDev& d, float) { return d.a.B32; }

template <int L, int CPL, int FORM, int MODE, typename PT>
__global__ __launch_bounds__(256) void obs_lds_kernel(TaskView t, ObsDev d) {
  if (d.a.done != nullptr && *d.a.done) return;
  extern __shared__ __attribute__((aligned(16))) double lds_raw[];
  PT* sB = reinterpret_cast<PT*>(lds_raw);
  stage_rows(sB, factor_b(d, PT(0)), d.J * d.a.r);
  for (int64_t task = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); task < t.ntask;
       task += (int64_t)gridDim.x * 4)
    obs_task<L, CPL, FORM, MODE, PT, true, PT>(t, d, task, threadIdx.x & 63, sB);
}

// G: observations per lane row in flight per step.
template <int L, int CPL, int FORM, int MODE, typename PT, int G = tiles::kGroups>
__global__ __launch_bounds__(256) void obs_rows_lds_kernel(ObsDev d, const int32_t* obs_ptr,
                                                           int64_t n, int spw) {
  if (d.a.done != nullptr && *d.a.done) return;
  extern __shared__ __attribute__((aligned(16))) double lds_raw[];
  PT* sB = reinterpret_cast<PT*>(lds_raw);
  stage_rows(sB, factor_b(d, PT(0)), d.J * d.a.r);
  constexpr int ROWS = 64 / L;
  for (int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); w * spw < n;
       w += (int64_t)gridDim.x * 4) {
    const int64_t sb = w * spw;
    for (int k = 0; k < spw; k += ROWS) {
      const int64_t s0 = sb + k;
      if (s0 >= n) break;
      tiles::obs_rows<L, CPL, FORM, MODE, PT, true, PT, G>(
          d, obs_ptr, s0, (int)min((int64_t)ROWS, n - s0), threadIdx.x & 63, sB);
    }
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

// Segments per wave of the lane-row form: enough waves for about 16 per CU
// (latency-bound work), at least one segment per lane row.
template <int L>
int rows_per_wave(int64_t nseg) {
  constexpr int ROWS = 64 / L;
  constexpr int64_t kTargetWaves = 256 * 16;
  int64_t spw = (nseg + kTargetWaves - 1) / kTargetWaves;
  spw = (spw + ROWS - 1) / ROWS * ROWS;
  return (int)std::max<int64_t>(ROWS, std::min<int64_t>(kSegPerWave, spw));
}

// LDS limit of the staged form for FP32 (pf) or FP64 factor rows, in the
// lane-row form (rows) or the task form; the override is read once.
size_t obs_lds_limit(bool pf, bool rows) {
  static const long env = [] {
    const char* v = std::getenv("CPHIFI_OBS_LDS_BYTES");
    return v != nullptr ? std::atol(v) : -1L;
  }();
  if (env >= 0) return (size_t)std::min<long>(env, 65536L);
  return (pf || !rows) ? (size_t)kObsLdsBytesF32 : (size_t)kObsLdsBytesF64;
}

template <int L, int CPL, int FORM, int MODE>
int launch_c(bool pf, const TaskView& tv, const ObsDev& d, const ObsTasks& t, hipStream_t st) {
  const size_t lds = (pf ? sizeof(float) : sizeof(double)) * (size_t)d.J * d.a.r;
  const int spw = rows_per_wave<L>(t.nseg);
  if (FORM != tiles::kExplicit && lds <= obs_lds_limit(pf, t.rows)) {
    if (t.rows) {
      const int64_t units = (t.nseg + spw - 1) / spw;
      const int64_t blocks = std::min<int64_t>(kObsLdsGrid, (units + 3) / 4);
      if (blocks == 0) return CPHIFI_OK;
      if (pf)
        hipLaunchKernelGGL((obs_rows_lds_kernel<L, CPL, FORM, MODE, float>),
                           dim3((unsigned)blocks), dim3(256), lds, st, d, t.obs_ptr, t.nseg,
                           spw);
      else if (lds > (size_t)kObsLdsBytesF32)
        // a copy of B above 16 KB holds the kernel at two workgroups per CU,
        // so the registers allow eight observations per lane row in flight
        hipLaunchKernelGGL((obs_rows_lds_kernel<L, CPL, FORM, MODE, double, 8>),
                           dim3((unsigned)blocks), dim3(256), lds, st, d, t.obs_ptr, t.nseg,
                           spw);
      else
        hipLaunchKernelGGL((obs_rows_lds_kernel<L, CPL, FORM, MODE, double>),
                           dim3((unsigned)blocks), dim3(256), lds, st, d, t.obs_ptr, t.nseg,
                           spw);
    } else {
      const int64_t blocks = std::min<int64_t>(kObsLdsGrid, (tv.ntask + 3) / 4);
      if (blocks == 0) return CPHIFI_OK;
      if (pf)
        hipLaunchKernelGGL((obs_lds_kernel<L, CPL, FORM, MODE, float>), dim3((unsigned)blocks),
                           dim3(256), lds, st, tv, d);
      else
        hipLaunchKernelGGL((obs_lds_kernel<L, CPL, FORM, MODE, double>), dim3((unsigned)blocks),
                           dim3(256), lds, st, tv, d);
    }
    CPHIFI_CHECK_LAUNCH();
    return CPHIFI_OK;
  }
  if (t.rows) {
    const int64_t blocks = (t.nseg + 4 * (int64_t)spw - 1) / (4 * (int64_t)spw);
    if (blocks == 0) return CPHIFI_OK;
    if (pf)
      hipLaunchKernelGGL((obs_rows_kernel<L, CPL, FORM, MODE, float>), dim3((unsigned)blocks),
                         dim3(256), 0, st, d, t.obs_ptr, t.nseg, spw);
    else
      hipLaunchKernelGGL((obs_rows_kernel<L, CPL, FORM, MODE, double>), dim3((unsigned)blocks),
                         dim3(256), 0, st, d, t.obs_ptr, t.nseg, spw);
    CPHIFI_CHECK_LAUNCH();
    return CPHIFI_OK;
  }
  const int blocks = (tv.ntask + 3) / 4;
  if (blocks == 0) return CPHIFI_OK;
  if (pf)
    hipLaunchKernelGGL((obs_kernel<L, CPL, FORM, MODE, float>), dim3(blocks), dim3(256), 0, st, tv,
                       d);
  else
    hipLaunchKernelGGL((obs_kernel<L, CPL, FORM, MODE, double>), dim3(blocks), dim3(256), 0, st,
                       tv, d);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}

// Lanes per observation: L = 4 up to r = 20, 8 up to r = 40, 16 beyond; each
// lane then holds ceil(r / L) <= 5 columns.
template <int FORM, int MODE>
int launch_m(int r, bool pf, const TaskView& tv, const ObsDev& d, const ObsTasks& t,
             hipStream_t st) {
  if (r <= 4) return launch_c<4, 1, FORM, MODE>(pf, tv, d, t, st);
  if (r <= 8) return launch_c<4, 2, FORM, MODE>(pf, tv, d, t, st);
  if (r <= 12) return launch_c<4, 3, FORM, MODE>(pf, tv, d, t, st);
  if (r <= 16) return launch_c<4, 4, FORM, MODE>(pf, tv, d, t, st);
  if (r <= 20) return launch_c<4, 5, FORM, MODE>(pf, tv, d, t, st);
  if (r <= 24) return launch_c<8, 3, FORM, MODE>(pf, tv, d, t, st);
  if (r <= 32) return launch_c<8, 4, FORM, MODE>(pf, tv, d, t, st);
  if (r <= 40) return launch_c<8, 5, FORM, MODE>(pf, tv, d, t, st);
  if (r <= 48) return launch_c<16, 3, FORM, MODE>(pf, tv, d, t, st);
  return launch_c<16, 4, FORM, MODE>(pf, tv, d, t, st);
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
  if (!expl && (I * a.r * 8 > (int64_t)UINT32_MAX || J * a.r * 8 > (int64_t)UINT32_MAX)) {
    set_error("launch_obs: factor matrices beyond 4 GiB need the explicit Zhat form");
    return CPHIFI_UNSUPPORTED;
  }
  if (!expl && part_is_float && mode == ObsMode::Gather &&
      (a.A32 == nullptr || a.B32 == nullptr)) {
    set_error("launch_obs: the FP32 gather needs FP32 copies of A and B");
    return CPHIFI_INVALID_ARG;
  }
  TaskView tv{t.seg, t.beg, t.end, t.slot, t.first, t.ntask};
  ObsDev d{a, I, J};
  int st_ = CPHIFI_OK;
  if (t.rows && (t.nmulti > 0 || t.obs_ptr == nullptr)) {
    set_error("launch_obs: the short-segment form needs the CSR and no split segments");
    return CPHIFI_INVALID_ARG;
  }
  using tiles::kExplicit;
  using tiles::kImplicit;
  using tiles::kOwner;
  const bool own = !expl && t.owner;
  if (mode == ObsMode::Gather)
    st_ = expl  ? launch_m<kExplicit, 0>(a.r, part_is_float, tv, d, t, st)
          : own ? launch_m<kOwner, 0>(a.r, part_is_float, tv, d, t, st)
                : launch_m<kImplicit, 0>(a.r, part_is_float, tv, d, t, st);
  else
    st_ = expl  ? launch_m<kExplicit, 1>(a.r, part_is_float, tv, d, t, st)
          : own ? launch_m<kOwner, 1>(a.r, part_is_float, tv, d, t, st)
                : launch_m<kImplicit, 1>(a.r, part_is_float, tv, d, t, st);
  if (st_ != CPHIFI_OK) return st_;
  if (!t.rows && t.nmulti > 0) {
    hipLaunchKernelGGL(segment_reduce_kernel, dim3((t.nmulti + 3) / 4), dim3(256), 0, st, t.mseg,
                       t.mptr, t.nmulti, a.tpart, a.r, a.out, a.done);
    CPHIFI_CHECK_LAUNCH();
  }
  return CPHIFI_OK;
}

}  // namespace cphifi
