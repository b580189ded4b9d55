// Stand-alone n x n by n x r product (tile tuning and per-variant tests), and
// its variant that takes no workspace (scratch in a static device array).
#include "cphifi_internal.h"

#include <mutex>

using namespace cphifi;

namespace {

constexpr size_t kAlign = 256;
constexpr int kEltBf16Tiled = 3;  // BF16 U in the 16 x 64 tile layout

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct ProductLayout {
  size_t part, xthi, xtlo, total;
  int64_t ldxt;
};

// Workspace of a product with `slabs` split-K partial slabs (FP64 for every
// element type: the FP32 / BF16 products write float partials, which fit).
ProductLayout product_layout(int64_t n, int64_t r, int elt, int slabs = kMaxSplit) {
  ProductLayout L{};
  const int64_t ldp = (r + 15) / 16 * 16;
  L.ldxt = (n + kLowpAlign - 1) / kLowpAlign * kLowpAlign;
  size_t off = 0;
  L.part = off;
  off = align_up(off + sizeof(double) * (size_t)slabs * n * ldp, kAlign);
  if (elt == (int)Elt::BF16 || elt == kEltBf16Tiled) {
    L.xthi = off;
    off = align_up(off + sizeof(__bf16) * (size_t)ldp * L.ldxt, kAlign);
    L.xtlo = off;
    off = align_up(off + sizeof(__bf16) * (size_t)ldp * L.ldxt, kAlign);
  }
  L.total = off;
  return L;
}

// Scratch of cphifi_product_static: one array per GPU (each device holds its
// own copy of this module's globals), never allocated or freed by the library.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
__device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current).  In host code the array's name is only a
// stand-in for the symbol, never a device address.
int scratch_on_current_device(void** out) {
  int dev = 0;
  CPHIFI_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("cphifi_product_static: device %d beyond the supported %d", dev, kMaxDevices);
    return CPHIFI_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    CPHIFI_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (ptr == nullptr || reinterpret_cast<uintptr_t>(ptr) % kAlign != 0) {
      set_error("cphifi_product_static: scratch symbol has no aligned device address");
      return CPHIFI_HIP_ERROR;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CPHIFI_OK;
}

int num_cus() {
  int num_cu = 256, dev = 0;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  return num_cu > 0 ? num_cu : 256;
}

// Y = op(U) diag(xscale) X with the split-K partials (and the BF16 split of X)
// in `ws` laid out by L for gp.ksplit slabs.
int run_product(Elt e, bool tiled, int trans, const GemmPlan& gp, int64_t n, const void* U,
                int64_t ldu, const double* X, int64_t r, const double* xscale, double* Y,
                char* ws, const ProductLayout& L, hipStream_t st) {
  const int ldp = (int)((r + 15) / 16 * 16);
  int rc;
  if (e == Elt::BF16) {
    __bf16* hi = (__bf16*)(ws + L.xthi);
    __bf16* lo = (__bf16*)(ws + L.xtlo);
    if ((rc = launch_split_bf16(X, r, (int)r, xscale, n, hi, lo, L.ldxt, nullptr, st))) return rc;
    if ((rc = launch_gemm_bf16(gp, (const __bf16*)U, ldu, n, X, r, (int)r, xscale, ws + L.part,
                               hi, lo, L.ldxt, nullptr, st, tiled)))
      return rc;
  } else {
    if ((rc = launch_gemm(e, trans != 0, gp, U, ldu, n, X, r, (int)r, xscale, ws + L.part,
                          nullptr, st)))
      return rc;
  }
  return launch_reduce_partials(ws + L.part, e != Elt::F64, gp.ksplit, ldp, n, (int)r, Y,
                                nullptr, nullptr, nullptr, nullptr, st);
}

int check_product_args(int elt, int trans, int mw, int s, int64_t n, const void* U, int64_t ldu,
                       const double* X, int64_t r, double* Y, const char* where) {
  if (elt < 0 || elt > kEltBf16Tiled || n < 1 || n > INT32_MAX || r < 1 || r > kMaxRank ||
      U == nullptr || X == nullptr || Y == nullptr || ldu < n) {
    set_error("%s: bad arguments", where);
    return CPHIFI_INVALID_ARG;
  }
  const Elt e = elt == kEltBf16Tiled ? Elt::BF16 : (Elt)elt;
  if (!gemm_cfg_valid(e, mw, s)) {
    set_error("%s: unsupported tile (mw=%d, s=%d) for element type %d", where, mw, s, elt);
    return CPHIFI_INVALID_ARG;
  }
  if (e == Elt::BF16 && trans) {
    set_error("%s: the BF16 product has no transposed form", where);
    return CPHIFI_INVALID_ARG;
  }
  return CPHIFI_OK;
}

// Streaming read of a device buffer (the achievable HBM read rate against
// which the products are compared): 16-byte non-temporal loads, four in flight
// per thread, grid-stride; each workgroup sums what it read and writes one
// partial, so no load can be dropped.
typedef double dvec2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void stream_read_kernel(const dvec2* __restrict__ p,
                                                          int64_t n2, double* partial) {
  __shared__ double red[256];
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (; i + 3 * stride < n2; i += 4 * stride) {
    const dvec2 a = __builtin_nontemporal_load(p + i);
    const dvec2 b = __builtin_nontemporal_load(p + i + stride);
    const dvec2 c = __builtin_nontemporal_load(p + i + 2 * stride);
    const dvec2 d = __builtin_nontemporal_load(p + i + 3 * stride);
    s0 += (a.x + b.x) + (c.x + d.x);
    s1 += (a.y + b.y) + (c.y + d.y);
  }
  for (; i < n2; i += stride) {
    const dvec2 a = __builtin_nontemporal_load(p + i);
    s0 += a.x;
    s1 += a.y;
  }
  red[threadIdx.x] = s0 + s1;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

}  // namespace

extern "C" {

int cphifi_stream_read(const void* buf, int64_t bytes, int32_t blocks, double* partial,
                       void* stream) {
  if (buf == nullptr || partial == nullptr || bytes <= 0 || bytes % 16 != 0 ||
      ((uintptr_t)buf % 16) != 0 || blocks < 1 || blocks > 65536) {
    set_error("cphifi_stream_read: need a 16-byte aligned buffer, bytes > 0 a multiple of 16, "
              "1 <= blocks <= 65536 (bytes=%lld blocks=%d)", (long long)bytes, blocks);
    return CPHIFI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(stream_read_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                     (const dvec2*)buf, bytes / 16, partial);
  CPHIFI_CHECK_LAUNCH();
  return CPHIFI_OK;
}


int cphifi_product_workspace_bytes(int64_t n, int64_t r, int elt, size_t* bytes) {
  clear_error();
  if (bytes == nullptr || n < 1 || r < 1 || r > kMaxRank || elt < 0 || elt > kEltBf16Tiled) {
    set_error("product_workspace_bytes: bad arguments");
    return CPHIFI_INVALID_ARG;
  }
  *bytes = product_layout(n, r, elt).total;
  return CPHIFI_OK;
}

int cphifi_product_tile_ok(int elt, int mw, int s) {
  if (elt < 0 || elt > kEltBf16Tiled) return 0;
  return gemm_cfg_valid(elt == kEltBf16Tiled ? Elt::BF16 : (Elt)elt, mw, s) ? 1 : 0;
}

int cphifi_product(int elt, int trans, int mw, int s, int ksplit, int64_t n, const void* U,
                   int64_t ldu, const double* X, int64_t r, const double* xscale, double* Y,
                   void* workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  int rc = check_product_args(elt, trans, mw, s, n, U, ldu, X, r, Y, "cphifi_product");
  if (rc != CPHIFI_OK) return rc;
  if (workspace == nullptr) {
    set_error("cphifi_product: workspace is NULL");
    return CPHIFI_INVALID_ARG;
  }
  const bool tiled = elt == kEltBf16Tiled;
  const Elt e = tiled ? Elt::BF16 : (Elt)elt;
  const ProductLayout L = product_layout(n, r, elt);
  if (workspace_bytes < L.total || reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) {
    set_error("cphifi_product: workspace must be >= %zu bytes, 256-byte aligned", L.total);
    return CPHIFI_INVALID_ARG;
  }
  GemmPlan gp = make_gemm_plan(e, trans != 0, n, (int)r, mw, s, ksplit, num_cus());
  if (tiled && ksplit <= 0) gp = bf16_stream_k(gp, n, num_cus());
  return run_product(e, tiled, trans, gp, n, U, ldu, X, r, xscale, Y, (char*)workspace, L,
                     (hipStream_t)stream);
}

size_t cphifi_product_static_max_bytes(void) { return kStaticScratchBytes; }

int cphifi_product_static(int elt, int trans, int mw, int s, int ksplit, int64_t n,
                          const void* U, int64_t ldu, const double* X, int64_t r,
                          const double* xscale, double* Y, void* stream) {
  clear_error();
  int rc = check_product_args(elt, trans, mw, s, n, U, ldu, X, r, Y, "cphifi_product_static");
  if (rc != CPHIFI_OK) return rc;
  const bool tiled = elt == kEltBf16Tiled;
  const Elt e = tiled ? Elt::BF16 : (Elt)elt;
  const int num_cu = num_cus();
  GemmPlan gp = make_gemm_plan(e, trans != 0, n, (int)r, mw, s, ksplit, num_cu);
  // An automatic split takes as many slabs as fit the static scratch (the
  // same split as cphifi_product whenever that fits); an explicit one must fit.
  while (ksplit <= 0 && gp.ksplit > 1 && product_layout(n, r, elt, gp.ksplit).total > kStaticScratchBytes)
    gp = make_gemm_plan(e, trans != 0, n, (int)r, mw, s, gp.ksplit - 1, num_cu);
  const ProductLayout L = product_layout(n, r, elt, gp.ksplit);
  if (L.total > kStaticScratchBytes) {
    set_error("cphifi_product_static: n=%lld r=%lld with split %d needs %zu bytes of scratch; "
              "the static scratch holds %zu (use cphifi_product with a workspace)",
              (long long)n, (long long)r, gp.ksplit, L.total, kStaticScratchBytes);
    return CPHIFI_INVALID_ARG;
  }
  void* ptr = nullptr;
  if ((rc = scratch_on_current_device(&ptr)) != CPHIFI_OK) return rc;
  return run_product(e, tiled, trans, gp, n, U, ldu, X, r, xscale, Y, (char*)ptr, L,
                     (hipStream_t)stream);
}

}  // extern "C"
