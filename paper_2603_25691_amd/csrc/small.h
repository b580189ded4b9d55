// Persistent single-workgroup FP64 PCG for small subproblems (small.hip).
#pragma once

#include "cphifi_internal.h"

namespace cphifi {

constexpr int kSmallThreads = 1024;  // one workgroup
constexpr int kSmallCols = 4;        // columns per product work item
constexpr int kSmallMaxRank = 64;
constexpr int64_t kSmallMaxN = 2048;
// X of a product is staged in LDS: n r doubles at most.
constexpr int64_t kSmallMaxNR = 4096;
// Work bounds of the persistent path: one n x n by n x r product (n^2 r
// multiply-adds) and one gather-scatter (q r) per step on one CU stay within
// a few microseconds at these bounds, against ~70 microseconds of launches
// and host polls per iteration of the multi-kernel loop.
constexpr double kSmallMaxProductWork = 2.0e6;
constexpr double kSmallMaxObsWork = 5.0e5;

struct SmallOut {
  int32_t iters, status;
  double rr, bb;  // final ||r||^2 (recursive) and ||b||^2
};

struct SmallArgs {
  int64_t n, ldk;
  int r, warm, precond, maxit, hist_len;
  double lam, rho, tol;
  const double *K;                  // K (symmetric)
  const double *UK, *UKT;           // U^T row-major (eigenvector k = row k) and U row-major
  const double *UV, *D;             // eigenvectors of V (row-major r x r), eq. fx diagonal
  const int32_t *obs_ptr, *obs_i, *obs_j;
  const double *A, *B, *Zhat;       // implicit (A, B) or explicit Zhat rows
  const double* b;                  // right-hand side (n x r)
  double *X, *R, *Z, *P, *Q, *Xh, *Y1, *T1, *T2;  // n x r each (X: the solution)
  double* Wq;                       // q x r scratch (per-observation terms of the gather)
  double* hist;                     // or NULL: recursive relative residual per iteration
  SmallOut* out;
};

// Whether a subproblem of this size takes the persistent path (wq_cap: the
// doubles available for the q x r scratch).
bool small_path_fits(int64_t n, int r, int64_t q, int64_t wq_cap);
// obs_t: the time index of each of the q observations (device).
int launch_small_pcg(const SmallArgs& a, const int32_t* obs_t, int64_t q, hipStream_t st);

}  // namespace cphifi
