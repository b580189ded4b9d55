#pragma once

// Wave tile of the per-observation gather-dot-scatter of the two-step product
// (Section 4.4.1):
//   xbar_l   = Xhat(t_l, :) . Zhat(l, :)                       (eq. vl)
//   Yhat1(s,:) = sum_{l: t_l = s} xbar_l Zhat(l, :)              (eq. yhat1)
// and the observed MTTKRP B(s,:) = sum_{l: t_l = s} y_l Zhat(l,:) that feeds the
// right-hand side.  Zhat(l,:) is either read (explicit rows, any tensor order)
// or formed on the fly as A(i_l,:) * B(j_l,:) (3-way Khatri-Rao rows, eq. zhat).
//
// Work unit: one wave per task = (segment s, contiguous observation range).
// Lane layout: the wave is 64/L rows of L lanes (L in {4, 8, 16}, chosen from
// r so that each lane holds CPL = ceil(r/L) <= 5 columns c0, c0+L, ...).  Row
// g takes one observation of a group of 64/L.  For each observation:
//  * Zhat(l, :) is formed from coalesced row reads of A and B (or of Zhat);
//  * xbar_l (eq. vl) is an L-lane row sum done with log2(L) DPP steps (no LDS,
//    no barrier), every lane of the row receiving the total;
//  * the scatter of eq. (yhat1) is a per-lane multiply-add into CPL running sums.
// Four groups are unrolled so their index and row loads are in flight together;
// the rows' running sums are folded once per task.  Segments longer than one
// task write partial rows that a second kernel adds in a fixed order, so
// results are deterministic (no atomics); xbar never leaves registers.  The
// tile is one wave's work, so it runs both as a plain grid (obs.hip) and as
// work items of the persistent batched solver (batch.hip).
#include "cphifi_internal.h"

namespace cphifi {
namespace tiles {

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

// v from lane (dpp permutation of) within each 16-lane row.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over aligned groups of L lanes (L = 4, 8, 16), result in every lane of the
// group: xor 1 and xor 2 (quad permutations), then the half-row mirror (pairs
// the two quads of an 8-lane half) and the row mirror (pairs the two halves).
template <int L>
__device__ __forceinline__ double group_sum(double v) {
  v += dpp_d<0xB1>(v);                      // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);                      // quad_perm [2,3,0,1]
  if (L >= 8) v += dpp_d<0x141>(v);         // row_half_mirror
  if (L >= 16) v += dpp_d<0x140>(v);        // row_mirror
  return v;
}

constexpr int kGroups = 4;  // observation groups unrolled per step

template <int L, int CPL, bool EXPL, int MODE, typename PT>
__device__ __forceinline__ void obs_task(const TaskView& t, const ObsDev& d, int64_t task) {
  constexpr int ROWS = 64 / L;  // observations per group
  const ObsArgs& a = d.a;
  const int lane = item_tid() & 63;
  const int r = a.r;
  const int g = lane / L, cl = lane % L;
  const int64_t s = t.seg[task];
  const int64_t beg = t.beg[task], end = t.end[task];
  const int32_t slot = t.slot[task];

  uint32_t cidx[CPL];  // in-bounds column index used for loads
  bool con[CPL];       // real column
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int c = cl + L * j;
    con[j] = c < r;
    cidx[j] = (uint32_t)min(c, r - 1);
  }

  const uint32_t Imax = (uint32_t)(d.I - 1), Jmax = (uint32_t)(d.J - 1), ur = (uint32_t)r;
  const char* __restrict__ Abytes = (const char*)a.A;
  const char* __restrict__ Bbytes = (const char*)a.B;
  uint32_t cbyte[CPL];
#pragma unroll
  for (int j = 0; j < CPL; ++j) cbyte[j] = cidx[j] * 8u;
  constexpr int STEP = ROWS * kGroups;

  // Observation indices are software-pipelined one step ahead: the next step's
  // (HBM) index loads are in flight while this step's rows are read and used.
  auto fetch_idx = [&](int64_t base_, int32_t (&ii_)[kGroups], int32_t (&jj_)[kGroups]) {
#pragma unroll
    for (int u = 0; u < kGroups; ++u) {
      const int64_t l = base_ + ROWS * u + g;
      const int64_t o = l < end ? l : end - 1;
      if (!EXPL) {
        ii_[u] = a.obs_i[o];
        jj_[u] = a.obs_j[o];
      }
    }
  };
  int32_t ii_cur[kGroups] = {}, jj_cur[kGroups] = {};
  if (beg < end) fetch_idx(beg, ii_cur, jj_cur);

  // Xhat(s, :); zero in padding columns, so they drop out of the dot products.
  double xh[CPL];
#pragma unroll
  for (int j = 0; j < CPL; ++j) xh[j] = 0.0;
  if (MODE == 0) {
    const PT* part = (const PT*)a.part;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      double v = 0.0;
      for (int sp = 0; sp < a.ksplit; ++sp)
        v += (double)part[((int64_t)sp * a.n + s) * a.ldp + cidx[j]];
      xh[j] = con[j] ? v : 0.0;
      if (a.Xhat != nullptr && t.first[task] && g == 0 && con[j]) a.Xhat[s * r + cidx[j]] = v;
    }
  }

  double acc[CPL];
#pragma unroll
  for (int j = 0; j < CPL; ++j) acc[j] = 0.0;
  for (int64_t base = beg; base < end; base += STEP) {
    int32_t ii_nxt[kGroups] = {}, jj_nxt[kGroups] = {};
    if (base + STEP < end) fetch_idx(base + STEP, ii_nxt, jj_nxt);
    double z[kGroups][CPL];
    double w[kGroups];
    bool on[kGroups];
    // Branch-free loads: clamp to an in-bounds observation, mask the result.
#pragma unroll
    for (int u = 0; u < kGroups; ++u) {
      const int64_t l = base + ROWS * u + g;
      on[u] = l < end;
      const int64_t o = on[u] ? l : end - 1;
      if (EXPL) {
#pragma unroll
        for (int j = 0; j < CPL; ++j) z[u][j] = a.Zhat[o * r + cidx[j]];
      } else {
        // byte offsets in 32 bits (I r and J r doubles fit, checked on the host)
        const uint32_t ib = min((uint32_t)max(ii_cur[u], 0), Imax) * ur * 8u;
        const uint32_t jb = min((uint32_t)max(jj_cur[u], 0), Jmax) * ur * 8u;
#pragma unroll
        for (int j = 0; j < CPL; ++j)
          z[u][j] = *(const double*)(Abytes + (ib + cbyte[j])) *
                    *(const double*)(Bbytes + (jb + cbyte[j]));
      }
      if (MODE == 1) w[u] = on[u] ? a.y[o] : 0.0;
    }
    if (MODE == 0) {
#pragma unroll
      for (int u = 0; u < kGroups; ++u) {
        double part = 0.0;
#pragma unroll
        for (int j = 0; j < CPL; ++j) part += z[u][j] * xh[j];
        const double xb = group_sum<L>(part);  // xbar_l, eq. vl
        w[u] = on[u] ? xb : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < kGroups; ++u)
#pragma unroll
      for (int j = 0; j < CPL; ++j) acc[j] += w[u] * z[u][j];  // eq. yhat1 / MTTKRP
#pragma unroll
    for (int u = 0; u < kGroups; ++u) {
      ii_cur[u] = ii_nxt[u];
      jj_cur[u] = jj_nxt[u];
    }
  }
  // fold the observation rows of the wave
#pragma unroll
  for (int j = 0; j < CPL; ++j)
#pragma unroll
    for (int off = L; off < 64; off <<= 1) acc[j] += __shfl_xor(acc[j], off, 64);
  if (g == 0) {
    double* dst = slot < 0 ? a.out + s * r : a.tpart + (int64_t)slot * r;
#pragma unroll
    for (int j = 0; j < CPL; ++j)
      if (con[j]) dst[cidx[j]] = acc[j];
  }
}

// Short segments: each L-lane row of the wave takes one whole segment, so a
// wave works on 64/L segments at once, each row accumulating its segment's
// observations kGroups at a time and writing its own output row (no fold
// across rows).  Segments [s0, s0 + nseg), nseg <= 64/L, read from the CSR
// obs_ptr; for segments without a split over several tasks (the caller
// checks), this gives the same Yhat1 / MTTKRP rows as obs_task.
template <int L, int CPL, bool EXPL, int MODE, typename PT>
__device__ __forceinline__ void obs_rows(const ObsDev& d, const int32_t* obs_ptr, int64_t s0,
                                         int nseg) {
  const ObsArgs& a = d.a;
  const int lane = item_tid() & 63;
  const int r = a.r;
  const int g = lane / L, cl = lane % L;
  const bool row_on = g < nseg;
  const int64_t s = s0 + (row_on ? g : 0);
  const int64_t beg = obs_ptr[s];
  const int64_t end = row_on ? (int64_t)obs_ptr[s + 1] : beg;
  const int64_t last = end > beg ? end - 1 : -1;  // clamp target of masked loads

  uint32_t cidx[CPL];
  bool con[CPL];
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int c = cl + L * j;
    con[j] = c < r;
    cidx[j] = (uint32_t)min(c, r - 1);
  }
  const uint32_t Imax = (uint32_t)(d.I - 1), Jmax = (uint32_t)(d.J - 1), ur = (uint32_t)r;
  const char* __restrict__ Abytes = (const char*)a.A;
  const char* __restrict__ Bbytes = (const char*)a.B;
  uint32_t cbyte[CPL];
#pragma unroll
  for (int j = 0; j < CPL; ++j) cbyte[j] = cidx[j] * 8u;

  // wave-uniform step count: the longest segment of the wave
  int maxlen = (int)(end - beg);
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) maxlen = max(maxlen, __shfl_xor(maxlen, off, 64));
  const int nstep = (maxlen + kGroups - 1) / kGroups;

  auto obs_at = [&](int step, int u) -> int64_t {
    const int64_t l = beg + (int64_t)step * kGroups + u;
    return l < end ? l : last;
  };
  auto fetch_idx = [&](int step, int32_t (&ii_)[kGroups], int32_t (&jj_)[kGroups]) {
#pragma unroll
    for (int u = 0; u < kGroups; ++u) {
      const int64_t o = obs_at(step, u);
      ii_[u] = 0;
      jj_[u] = 0;
      if (!EXPL && o >= 0) {
        ii_[u] = a.obs_i[o];
        jj_[u] = a.obs_j[o];
      }
    }
  };
  int32_t ii_cur[kGroups] = {}, jj_cur[kGroups] = {};
  if (nstep > 0) fetch_idx(0, ii_cur, jj_cur);

  double xh[CPL];
#pragma unroll
  for (int j = 0; j < CPL; ++j) xh[j] = 0.0;
  if (MODE == 0) {
    const PT* part = (const PT*)a.part;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      double v = 0.0;
      for (int sp = 0; sp < a.ksplit; ++sp)
        v += (double)part[((int64_t)sp * a.n + s) * a.ldp + cidx[j]];
      xh[j] = con[j] ? v : 0.0;
      if (a.Xhat != nullptr && row_on && con[j]) a.Xhat[s * r + cidx[j]] = v;
    }
  }

  double acc[CPL];
#pragma unroll
  for (int j = 0; j < CPL; ++j) acc[j] = 0.0;
  for (int step = 0; step < nstep; ++step) {
    int32_t ii_nxt[kGroups] = {}, jj_nxt[kGroups] = {};
    if (step + 1 < nstep) fetch_idx(step + 1, ii_nxt, jj_nxt);
    double z[kGroups][CPL];
    double w[kGroups];
    bool on[kGroups];
#pragma unroll
    for (int u = 0; u < kGroups; ++u) {
      const int64_t l = beg + (int64_t)step * kGroups + u;
      on[u] = l < end;
      const int64_t o = on[u] ? l : last;
      if (EXPL) {
#pragma unroll
        for (int j = 0; j < CPL; ++j) z[u][j] = o >= 0 ? a.Zhat[o * r + cidx[j]] : 0.0;
      } else {
        const uint32_t ib = min((uint32_t)max(ii_cur[u], 0), Imax) * ur * 8u;
        const uint32_t jb = min((uint32_t)max(jj_cur[u], 0), Jmax) * ur * 8u;
#pragma unroll
        for (int j = 0; j < CPL; ++j)
          z[u][j] = *(const double*)(Abytes + (ib + cbyte[j])) *
                    *(const double*)(Bbytes + (jb + cbyte[j]));
      }
      if (MODE == 1) w[u] = on[u] ? a.y[o] : 0.0;
    }
    if (MODE == 0) {
#pragma unroll
      for (int u = 0; u < kGroups; ++u) {
        double part = 0.0;
#pragma unroll
        for (int j = 0; j < CPL; ++j) part += z[u][j] * xh[j];
        const double xb = group_sum<L>(part);  // xbar_l, eq. vl
        w[u] = on[u] ? xb : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < kGroups; ++u)
#pragma unroll
      for (int j = 0; j < CPL; ++j) acc[j] += w[u] * z[u][j];  // eq. yhat1 / MTTKRP
#pragma unroll
    for (int u = 0; u < kGroups; ++u) {
      ii_cur[u] = ii_nxt[u];
      jj_cur[u] = jj_nxt[u];
    }
  }
  if (row_on) {
#pragma unroll
    for (int j = 0; j < CPL; ++j)
      if (con[j]) a.out[s * r + cidx[j]] = acc[j];
  }
}

}  // namespace tiles
}  // namespace cphifi
