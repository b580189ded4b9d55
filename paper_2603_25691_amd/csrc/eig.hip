// One-time eigendecomposition K = U_K D_K U_K^T of the kernel matrix (eq. eigK),
// a setup step outside the solve: rocSOLVER's divide-and-conquer symmetric
// eigensolver on the device.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "cphifi_internal.h"

using namespace cphifi;

extern "C" int cphifi_kernel_eig(int64_t n, const double* K, int64_t ldk, double* UK,
                                 double* dK, void* stream) {
  clear_error();
  if (ldk == 0) ldk = n;
  if (n < 1 || ldk < n || K == nullptr || UK == nullptr || dK == nullptr) {
    set_error("cphifi_kernel_eig: bad arguments (n=%lld ldk=%lld)", (long long)n,
              (long long)ldk);
    return CPHIFI_INVALID_ARG;
  }
  if (n > INT32_MAX || ldk > INT32_MAX) {
    set_error("cphifi_kernel_eig: n=%lld exceeds the 32-bit solver interface", (long long)n);
    return CPHIFI_UNSUPPORTED;
  }
  hipStream_t st = (hipStream_t)stream;
  if (UK != K)
    CPHIFI_HIP(hipMemcpy2DAsync(UK, (size_t)ldk * sizeof(double), K, (size_t)ldk * sizeof(double),
                                (size_t)n * sizeof(double), (size_t)n, hipMemcpyDeviceToDevice,
                                st));
  double* E = nullptr;
  rocblas_int* info = nullptr;
  CPHIFI_HIP(hipMalloc(&E, (size_t)n * sizeof(double)));
  if (hipMalloc(&info, sizeof(rocblas_int)) != hipSuccess) {
    (void)hipFree(E);
    set_error("cphifi_kernel_eig: hipMalloc failed");
    return CPHIFI_HIP_ERROR;
  }
  rocblas_handle h = nullptr;
  int status = CPHIFI_OK;
  if (rocblas_create_handle(&h) != rocblas_status_success) {
    set_error("cphifi_kernel_eig: rocblas_create_handle failed");
    status = CPHIFI_HIP_ERROR;
  } else {
    rocblas_set_stream(h, st);
    // Column-major view of the symmetric matrix; eigenvectors overwrite it as
    // columns, i.e. eigenvector k at UK + k*ldk.
    const rocblas_status rs = rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper,
                                               (rocblas_int)n, UK, (rocblas_int)ldk, dK, E, info);
    rocblas_int hinfo = 0;
    if (rs != rocblas_status_success) {
      set_error("cphifi_kernel_eig: rocsolver_dsyevd returned %d", (int)rs);
      status = CPHIFI_HIP_ERROR;
    } else if (hipMemcpyAsync(&hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, st) !=
                   hipSuccess ||
               hipStreamSynchronize(st) != hipSuccess) {
      set_error("cphifi_kernel_eig: synchronisation failed");
      status = CPHIFI_HIP_ERROR;
    } else if (hinfo != 0) {
      set_error("cphifi_kernel_eig: eigensolver did not converge (info=%d)", (int)hinfo);
      status = CPHIFI_NUMERIC;
    }
    rocblas_destroy_handle(h);
  }
  (void)hipFree(E);
  (void)hipFree(info);
  return status;
}
