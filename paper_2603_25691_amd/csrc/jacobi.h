// Cyclic Jacobi eigensolver for the small symmetric Gram matrix V = Z^T Z
// (r x r, eq. eigV), run by one 256-thread workgroup.  Shared by the stand-alone
// setup kernel and the per-solve setup phase of the persistent batched kernel,
// so both produce the same eigenpairs bit for bit.
//
// Disjoint rotation pairs of a round-robin (circle method) schedule are
// applied in parallel: rows first (J^T A), then columns (A J) and the
// eigenvector accumulator (V J).  For odd r the fixed player of the schedule is
// the dummy (player x is index x - 1), which keeps the convergence quadratic:
// with a real index fixed and the dummy rotating, the couplings of the fixed
// index to near-null directions decayed only linearly in a CPU model of the
// same schedule.  Stops when the off-diagonal mass is below (1e-15)^2 of the
// Frobenius mass, or after 60 sweeps.
#pragma once

#include <hip/hip_runtime.h>

namespace cphifi {

// Workspace of jacobi_sym for ranks up to MAXR (LDS).
template <int MAXR>
struct JacobiLds {
  double a[MAXR * (MAXR + 1)];
  double v[MAXR * (MAXR + 1)];
  double cs[MAXR / 2][2];
  int pr[MAXR / 2][2];
  double red[8];
};

// Deterministic sum over the 256 threads (4 waves), valid in every thread.
__device__ __forceinline__ double jacobi_block_sum(double x, double* red, int tid) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = x;
  __syncthreads();
  if (tid == 0) red[4] = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  return red[4];
}

// Eigenpairs of Vin (r x r row-major, r <= MAXR): UV (r x r row-major, column
// k = eigenvector k) and dV (r).  tid: the thread index in 0..255.
template <int MAXR>
__device__ __forceinline__ void jacobi_sym(const double* Vin, int r, double* UV, double* dV,
                                           JacobiLds<MAXR>& w, int tid) {
  constexpr int L = MAXR + 1;
  constexpr int NT = 256;
  double* a = w.a;
  double* v = w.v;
  const int m = r + (r & 1);  // even player count; player 0 is a dummy when r is odd
  const int shift = m - r;
  for (int e = tid; e < m * m; e += NT) {
    const int i = e / m, j = e % m;
    a[i * L + j] = (i < r && j < r) ? Vin[i * r + j] : 0.0;
    v[i * L + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  double fro = 0.0;
  for (int e = tid; e < r * r; e += NT) {
    const double x = a[(e / r) * L + (e % r)];
    fro += x * x;
  }
  fro = jacobi_block_sum(fro, w.red, tid);
  for (int sweep = 0; sweep < 60 && m > 1; ++sweep) {
    double off = 0.0;
    for (int e = tid; e < r * r; e += NT) {
      const int i = e / r, j = e % r;
      if (i != j) off += a[i * L + j] * a[i * L + j];
    }
    off = jacobi_block_sum(off, w.red, tid);
    if (!(off > 1e-30 * fro)) break;
    for (int round = 0; round < m - 1; ++round) {
      if (tid < m / 2) {
        // circle method: player 0 fixed, others rotate
        int p, q;
        if (tid == 0) {
          p = 0;
          q = 1 + (round % (m - 1));
        } else {
          p = 1 + ((round + tid) % (m - 1));
          q = 1 + ((round + (m - 1) - tid) % (m - 1));
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        // player -> index; the dummy's partner gets the identity rotation,
        // paired with index r (the zero padding row and column of a)
        p -= shift;
        q -= shift;
        const bool dummy = p < 0;
        if (dummy) p = r;
        double c = 1.0, s = 0.0;
        if (!dummy) {
          const double apq = a[p * L + q];
          if (apq != 0.0) {
            const double tau = (a[q * L + q] - a[p * L + p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        w.pr[tid][0] = p;
        w.pr[tid][1] = q;
        w.cs[tid][0] = c;
        w.cs[tid][1] = s;
      }
      __syncthreads();
      for (int e = tid; e < (m / 2) * m; e += NT) {  // rows
        const int k = e / m, j = e % m;
        const int p = w.pr[k][0], q = w.pr[k][1];
        const double c = w.cs[k][0], s = w.cs[k][1];
        const double ap = a[p * L + j], aq = a[q * L + j];
        a[p * L + j] = c * ap - s * aq;
        a[q * L + j] = s * ap + c * aq;
      }
      __syncthreads();
      for (int e = tid; e < (m / 2) * m; e += NT) {  // columns and vectors
        const int k = e / m, i = e % m;
        const int p = w.pr[k][0], q = w.pr[k][1];
        const double c = w.cs[k][0], s = w.cs[k][1];
        const double ap = a[i * L + p], aq = a[i * L + q];
        a[i * L + p] = c * ap - s * aq;
        a[i * L + q] = s * ap + c * aq;
        const double vp = v[i * L + p], vq = v[i * L + q];
        v[i * L + p] = c * vp - s * vq;
        v[i * L + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < r * r; e += NT) UV[e] = v[(e / r) * L + (e % r)];
  for (int i = tid; i < r; i += NT) dV[i] = a[i * L + i];
}

// Entry (a, b) of V = (A^T A) had (B^T B), summed in a fixed order (I rows of
// A, then J rows of B).  A: I x r, B: J x r, row-major.
__device__ __forceinline__ double gram_entry(const double* A, int64_t I, const double* B,
                                             int64_t J, int r, int a, int b) {
  double ga = 0.0, gb = 0.0;
  for (int64_t i = 0; i < I; ++i) ga += A[i * r + a] * A[i * r + b];
  for (int64_t j = 0; j < J; ++j) gb += B[j * r + a] * B[j * r + b];
  return ga * gb;
}

// D(s, c) = 1 / (gamma dV_c dK_s^2 + lambda dK_s + rho), dK clamped at 0
// (the inverse diagonal of eq. precon in the two eigenbases, Section 4.4.2).
__device__ __forceinline__ double precond_entry(double dk, double dv, double gamma, double lam,
                                                double rho) {
  const double d = fmax(dk, 0.0);
  return 1.0 / (gamma * dv * d * d + lam * d + rho);
}

}  // namespace cphifi
