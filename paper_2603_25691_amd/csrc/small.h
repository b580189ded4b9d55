// Persistent multi-workgroup FP64 PCG for small subproblems (small.hip).
#pragma once

#include "cphifi_internal.h"

namespace cphifi {

constexpr int kSmallThreads = 256;   // threads per workgroup (4 waves)
constexpr int kSmallMaxWG = 128;     // workgroups of one launch (all co-resident)
constexpr int kSmallMaxRank = 32;
constexpr int64_t kSmallMaxN = 2048;

// Control block and partial sums of one launch, at the start of a scratch
// buffer of at least small_scratch_bytes() (the plan's product partials).
struct SmallCtl {
  int32_t err;   // a barrier wait timed out: every workgroup leaves
  int32_t pad[15];
  // Arrival flags of the grid barrier, one 64-byte line per workgroup: the
  // number of barriers the workgroup has reached.
  uint32_t flag[kSmallMaxWG * 16];
};
constexpr size_t small_scratch_bytes() {
  return sizeof(SmallCtl) + 4 * sizeof(double) * kSmallMaxWG;
}

struct SmallOut {
  int32_t iters, status;
  double rr, bb;  // final ||r||^2 (recursive) and ||b||^2
};

struct SmallArgs {
  int64_t n, ldk;
  int r, warm, precond, maxit, hist_len;
  double lam, rho, tol;
  int64_t spin_limit;               // bound of every barrier wait
  const double *K;                  // K (symmetric)
  const double *UK, *UKT;           // U^T row-major (eigenvector k = row k) and U row-major
  const double *UV, *D;             // eigenvectors of V (row-major r x r), eq. fx diagonal
  const int32_t *obs_ptr, *obs_i, *obs_j;
  const double *A, *B, *Zhat;       // implicit (A, B) or explicit Zhat rows
  const double* b;                  // right-hand side (n x r)
  double* X;                        // the solution (n x r)
  double *R0, *R1, *P0, *P1;        // residual and search direction, two buffers each
  double *Z, *Q, *Xh, *Y1, *T2;     // n x r each
  void* scratch;                    // SmallCtl + partial sums
  double* hist;                     // or NULL: recursive relative residual per iteration
  SmallOut* out;
};

// Bound of a barrier wait (spins of ~64 cycles: about 0.1 s).
constexpr int64_t kSmallSpinLimit = int64_t(1) << 22;
// Status written to SmallOut when a barrier wait timed out.
constexpr int32_t kSmallTimeout = -1000;

// Whether a subproblem of this size takes the persistent path.
bool small_path_fits(int64_t n, int r);
int launch_small_pcg(const SmallArgs& a, hipStream_t st);

}  // namespace cphifi
