#pragma once

// Wave tiles of the per-observation gather-dot-scatter of the two-step product
// (Section 4.4.1):
//   xbar_l   = Xhat(t_l, :) . Zhat(l, :)                       (eq. vl)
//   Yhat1(s,:) = sum_{l: t_l = s} xbar_l Zhat(l, :)              (eq. yhat1)
// and the observed MTTKRP B(s,:) = sum_{l: t_l = s} y_l Zhat(l,:) that feeds the
// right-hand side.  Zhat(l,:) comes in three forms (FORM):
//   kImplicit  A(i_l,:) * B(j_l,:) formed on the fly (3-way Khatri-Rao rows);
//   kExplicit  read from the caller's Zhat rows (any tensor order);
//   kOwner     A(i,:) * B(j_l,:) where every observation of a segment has the
//              same i -- the unaligned setting of Section 4, where each pooled
//              time point belongs to one sample.  Then Xhat(s,:) * A(i,:) and
//              the final scaling by A(i,:) are done once per segment, and an
//              observation reads only its row of B.
//
// Lane layout: a wave is 64/L rows of L lanes (L in {4, 8, 16}, chosen from r
// so that each lane holds CPL = ceil(r/L) <= 5 columns c0, c0+L, ...).
//  * obs_task: one wave per task = (segment s, contiguous observation range);
//    row g takes one observation of a group of 64/L, and the rows' running
//    sums are folded once per task.  Segments longer than one task write
//    partial rows that a second pass adds in a fixed order.
//  * obs_rows: for short segments, each row takes one whole segment, so a
//    wave works on 64/L segments at once and each row writes its own output.
// For each observation, xbar_l (eq. vl) is an L-lane row sum done with log2(L)
// DPP steps (no LDS, no barrier), every lane of the row receiving the total,
// and the scatter of eq. (yhat1) is a per-lane multiply-add into CPL running
// sums.  Four observations per row are unrolled so their index and row loads
// are in flight together; the next step's index loads are issued one step
// ahead.  No atomics: results are deterministic; xbar never leaves registers.
// The tiles are one wave's work, so they run both as plain grids (obs.hip)
// and as work items of the persistent batched solver (batch.hip); `lane` is
// the lane in the wave (threadIdx.x & 63, or item_tid() & 63 inside a
// persistent kernel).
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

enum : int { kImplicit = 0, kExplicit = 1, kOwner = 2 };

// v from lane (dpp permutation of) within each 16-lane row.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_d(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over aligned groups of L lanes (L = 4, 8, 16), result in every lane of the
// group: xor 1 and xor 2 (quad permutations), then the half-row mirror (pairs
// the two quads of an 8-lane half) and the row mirror (pairs the two halves).
template <int L, typename VT>
__device__ __forceinline__ VT group_sum(VT v) {
  v += dpp_d<0xB1>(v);                      // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);                      // quad_perm [2,3,0,1]
  if (L >= 8) v += dpp_d<0x141>(v);         // row_half_mirror
  if (L >= 16) v += dpp_d<0x140>(v);        // row_mirror
  return v;
}

constexpr int kGroups = 4;  // observations per row unrolled per step

// The factor rows in the element type VT of the arithmetic: FP64, or the
// FP32 copies.
__device__ __forceinline__ const char* factor_bytes(const double* f64, const float* f32, double) {
  return (const char*)f64;
}
__device__ __forceinline__ const char* factor_bytes(const double* f64, const float* f32, float) {
  return (const char*)f32;
}

// Per-lane state of one row of the wave for one segment, and the step that
// consumes kGroups of its observations.  BL: the factor rows B(j,:) are read
// from a copy in LDS (`Bsrc`, same row-major layout) instead of from HBM/L2.
// VT: element type of the factor rows and of the arithmetic (double, or float
// for the low-precision inner operator: half the bytes per factor row, one
// DPP step per lane-row reduction step instead of two).
template <int L, int CPL, int FORM, int MODE, bool BL = false, typename VT = double,
          int G = kGroups>
struct ObsRow {
  uint32_t cidx[CPL];  // in-bounds column index used for loads
  bool con[CPL];       // real column
  uint32_t cbyte[CPL];
  uint32_t Imax, Jmax, ur;
  const char* Abytes;
  const char* Bbytes;
  VT arow[CPL];  // kOwner: A(i, :) of the segment's sample
  VT xv[CPL];    // Xhat(s,:), times A(i,:) for kOwner (zero in padding)
  VT acc[CPL];
  int32_t ii[G], jj[G];  // indices of the current step

  __device__ __forceinline__ void init(const ObsDev& d, int cl, const VT* Bsrc) {
    const int r = d.a.r;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const int c = cl + L * j;
      con[j] = c < r;
      cidx[j] = (uint32_t)min(c, r - 1);
      cbyte[j] = cidx[j] * (uint32_t)sizeof(VT);
      arow[j] = VT(1);
      xv[j] = VT(0);
      acc[j] = VT(0);
    }
    Imax = (uint32_t)(d.I - 1);
    Jmax = (uint32_t)(d.J - 1);
    ur = (uint32_t)r;
    Abytes = factor_bytes(d.a.A, d.a.A32, VT(0));
    Bbytes = BL ? (const char*)Bsrc : factor_bytes(d.a.B, d.a.B32, VT(0));
#pragma unroll
    for (int u = 0; u < G; ++u) ii[u] = jj[u] = 0;
  }

  // kOwner: the segment's sample row, from its first observation `o` (< 0:
  // empty segment, row 0 stands in).
  __device__ __forceinline__ void owner(const ObsDev& d, int64_t o) {
    if (FORM != kOwner) return;
    const int32_t i = o >= 0 ? d.a.obs_i[o] : 0;
    const uint32_t ib = min((uint32_t)max(i, 0), Imax) * ur * (uint32_t)sizeof(VT);
#pragma unroll
    for (int j = 0; j < CPL; ++j) arow[j] = *(const VT*)(Abytes + (ib + cbyte[j]));
  }

  // Xhat(s,:) summed over the split-K slabs of the product that made it.
  template <typename PT>
  __device__ __forceinline__ void xhat(const ObsDev& d, int64_t s, bool store) {
    const ObsArgs& a = d.a;
    const PT* part = (const PT*)a.part;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      double v = 0.0;
      for (int sp = 0; sp < a.ksplit; ++sp)
        v += (double)part[((int64_t)sp * a.n + s) * a.ldp + cidx[j]];
      if (store && a.Xhat != nullptr && con[j]) a.Xhat[s * a.r + cidx[j]] = v;
      xv[j] = con[j] ? (VT)(v * (double)arow[j]) : VT(0);
    }
  }

  // Index loads of observations o_u (< 0: none).
  __device__ __forceinline__ void fetch(const ObsDev& d, const int64_t (&o)[G],
                                        int32_t (&ii_)[G], int32_t (&jj_)[G]) {
#pragma unroll
    for (int u = 0; u < G; ++u) {
      ii_[u] = 0;
      jj_[u] = 0;
      if (FORM != kExplicit && o[u] >= 0) {
        if (FORM == kImplicit) ii_[u] = d.a.obs_i[o[u]];
        jj_[u] = d.a.obs_j[o[u]];
      }
    }
  }

  // One step: observations o_u (masked by on_u; o_u in bounds or < 0).
  __device__ __forceinline__ void step(const ObsDev& d, const int64_t (&o)[G],
                                       const bool (&on)[G]) {
    const ObsArgs& a = d.a;
    VT z[G][CPL];
    VT w[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      if (FORM == kExplicit) {
#pragma unroll
        for (int j = 0; j < CPL; ++j)
          z[u][j] = o[u] >= 0 ? (VT)a.Zhat[o[u] * a.r + cidx[j]] : VT(0);
      } else {
        // byte offsets in 32 bits (I r and J r doubles fit, checked on the host)
        const uint32_t jb = min((uint32_t)max(jj[u], 0), Jmax) * ur * (uint32_t)sizeof(VT);
        if (FORM == kOwner) {
#pragma unroll
          for (int j = 0; j < CPL; ++j) z[u][j] = *(const VT*)(Bbytes + (jb + cbyte[j]));
        } else {
          const uint32_t ib = min((uint32_t)max(ii[u], 0), Imax) * ur * (uint32_t)sizeof(VT);
#pragma unroll
          for (int j = 0; j < CPL; ++j)
            z[u][j] = *(const VT*)(Abytes + (ib + cbyte[j])) *
                      *(const VT*)(Bbytes + (jb + cbyte[j]));
        }
      }
      if (MODE == 1) w[u] = on[u] ? (VT)a.y[o[u]] : VT(0);
    }
    if (MODE == 0) {
#pragma unroll
      for (int u = 0; u < G; ++u) {
        VT part = VT(0);
#pragma unroll
        for (int j = 0; j < CPL; ++j) part += z[u][j] * xv[j];
        const VT xb = group_sum<L>(part);  // xbar_l, eq. vl
        w[u] = on[u] ? xb : VT(0);
      }
    }
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
      for (int j = 0; j < CPL; ++j) acc[j] += w[u] * z[u][j];  // eq. yhat1 / MTTKRP
  }
};

// One wave per task (see the file comment).  BL / Bsrc / VT: see ObsRow.
template <int L, int CPL, int FORM, int MODE, typename PT, bool BL = false, typename VT = double>
__device__ __forceinline__ void obs_task(const TaskView& t, const ObsDev& d, int64_t task,
                                         int lane, const VT* Bsrc = nullptr) {
  constexpr int ROWS = 64 / L;  // observations per group
  constexpr int STEP = ROWS * kGroups;
  const ObsArgs& a = d.a;
  const int g = lane / L, cl = lane % L;
  const int64_t s = t.seg[task];
  const int64_t beg = t.beg[task], end = t.end[task];
  const int32_t slot = t.slot[task];

  ObsRow<L, CPL, FORM, MODE, BL, VT> R;
  R.init(d, cl, Bsrc);
  auto obs_of = [&](int64_t base, int64_t (&o)[kGroups], bool (&on)[kGroups]) {
#pragma unroll
    for (int u = 0; u < kGroups; ++u) {
      const int64_t l = base + ROWS * u + g;
      on[u] = l < end;
      o[u] = on[u] ? l : end - 1;  // branch-free: clamp to an in-bounds observation
    }
  };
  if (beg < end) {
    int64_t o[kGroups];
    bool on[kGroups];
    obs_of(beg, o, on);
    R.fetch(d, o, R.ii, R.jj);
  }
  R.owner(d, beg < end ? beg : -1);
  if (MODE == 0) R.template xhat<PT>(d, s, t.first[task] && g == 0);

  for (int64_t base = beg; base < end; base += STEP) {
    int32_t ii_nxt[kGroups] = {}, jj_nxt[kGroups] = {};
    if (base + STEP < end) {
      int64_t on_[kGroups];
      bool onn[kGroups];
      obs_of(base + STEP, on_, onn);
      R.fetch(d, on_, ii_nxt, jj_nxt);
    }
    int64_t o[kGroups];
    bool on[kGroups];
    obs_of(base, o, on);
    R.step(d, o, on);
#pragma unroll
    for (int u = 0; u < kGroups; ++u) {
      R.ii[u] = ii_nxt[u];
      R.jj[u] = jj_nxt[u];
    }
  }
  // fold the observation rows of the wave
#pragma unroll
  for (int j = 0; j < CPL; ++j)
#pragma unroll
    for (int off = L; off < 64; off <<= 1) R.acc[j] += __shfl_xor(R.acc[j], off, 64);
  if (g == 0) {
    double* dst = slot < 0 ? a.out + s * a.r : a.tpart + (int64_t)slot * a.r;
#pragma unroll
    for (int j = 0; j < CPL; ++j)
      if (R.con[j]) dst[R.cidx[j]] = (double)(R.acc[j] * R.arow[j]);
  }
}

// Short segments: each L-lane row of the wave takes one whole segment of
// [s0, s0 + nseg), nseg <= 64/L, read from the CSR obs_ptr; for segments that
// are not split over several tasks (the caller checks) this gives the same
// rows as obs_task.
template <int L, int CPL, int FORM, int MODE, typename PT, bool BL = false, typename VT = double,
          int G = kGroups>
__device__ __forceinline__ void obs_rows(const ObsDev& d, const int32_t* obs_ptr, int64_t s0,
                                         int nseg, int lane, const VT* Bsrc = nullptr) {
  const ObsArgs& a = d.a;
  const int g = lane / L, cl = lane % L;
  const bool row_on = g < nseg;
  const int64_t s = s0 + (row_on ? g : 0);
  const int64_t beg = obs_ptr[s];
  const int64_t end = row_on ? (int64_t)obs_ptr[s + 1] : beg;
  const int64_t last = end > beg ? end - 1 : -1;  // clamp target of masked loads

  ObsRow<L, CPL, FORM, MODE, BL, VT, G> R;
  R.init(d, cl, Bsrc);
  // wave-uniform step count: the longest segment of the wave
  int maxlen = (int)(end - beg);
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) maxlen = max(maxlen, __shfl_xor(maxlen, off, 64));
  const int nstep = (maxlen + G - 1) / G;
  auto obs_of = [&](int st, int64_t (&o)[G], bool (&on)[G]) {
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int64_t l = beg + (int64_t)st * G + u;
      on[u] = l < end;
      o[u] = on[u] ? l : last;
    }
  };
  if (nstep > 0) {
    int64_t o[G];
    bool on[G];
    obs_of(0, o, on);
    R.fetch(d, o, R.ii, R.jj);
  }
  R.owner(d, last >= 0 ? beg : -1);
  if (MODE == 0) R.template xhat<PT>(d, s, row_on);

  for (int st = 0; st < nstep; ++st) {
    int32_t ii_nxt[G] = {}, jj_nxt[G] = {};
    if (st + 1 < nstep) {
      int64_t on_[G];
      bool onn[G];
      obs_of(st + 1, on_, onn);
      R.fetch(d, on_, ii_nxt, jj_nxt);
    }
    int64_t o[G];
    bool on[G];
    obs_of(st, o, on);
    R.step(d, o, on);
#pragma unroll
    for (int u = 0; u < G; ++u) {
      R.ii[u] = ii_nxt[u];
      R.jj[u] = jj_nxt[u];
    }
  }
  if (row_on) {
#pragma unroll
    for (int j = 0; j < CPL; ++j)
      if (R.con[j]) {
        const double v = (double)(R.acc[j] * R.arow[j]);
        if (a.xt_hi != nullptr) {
          const int64_t o = (int64_t)R.cidx[j] * a.ldxt + s;
          split_pair(v, &a.xt_hi[o], &a.xt_lo[o]);
        } else {
          a.out[s * a.r + R.cidx[j]] = v;
        }
      }
  }
}

}  // namespace tiles
}  // namespace cphifi
