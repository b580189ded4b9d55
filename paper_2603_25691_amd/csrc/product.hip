// Stand-alone n x n by n x r product (tile tuning and per-variant tests).
#include "cphifi_internal.h"

using namespace cphifi;

namespace {

constexpr size_t kAlign = 256;
constexpr int kEltBf16Tiled = 3;  // BF16 U in the 16 x 64 tile layout

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct ProductLayout {
  size_t part, xthi, xtlo, total;
  int64_t ldxt;
};

ProductLayout product_layout(int64_t n, int64_t r, int elt) {
  ProductLayout L{};
  const int64_t ldp = (r + 15) / 16 * 16;
  L.ldxt = (n + kLowpAlign - 1) / kLowpAlign * kLowpAlign;
  size_t off = 0;
  L.part = off;
  off = align_up(off + sizeof(double) * (size_t)kMaxSplit * n * ldp, kAlign);
  if (elt == (int)Elt::BF16 || elt == kEltBf16Tiled) {
    L.xthi = off;
    off = align_up(off + sizeof(__bf16) * (size_t)ldp * L.ldxt, kAlign);
    L.xtlo = off;
    off = align_up(off + sizeof(__bf16) * (size_t)ldp * L.ldxt, kAlign);
  }
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

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
  if (elt < 0 || elt > kEltBf16Tiled || n < 1 || n > INT32_MAX || r < 1 || r > kMaxRank ||
      U == nullptr || X == nullptr || Y == nullptr || ldu < n || workspace == nullptr) {
    set_error("cphifi_product: bad arguments");
    return CPHIFI_INVALID_ARG;
  }
  const bool tiled = elt == kEltBf16Tiled;
  const Elt e = tiled ? Elt::BF16 : (Elt)elt;
  if (!gemm_cfg_valid(e, mw, s)) {
    set_error("cphifi_product: unsupported tile (mw=%d, s=%d) for element type %d", mw, s, elt);
    return CPHIFI_INVALID_ARG;
  }
  if (e == Elt::BF16 && trans) {
    set_error("cphifi_product: the BF16 product has no transposed form");
    return CPHIFI_INVALID_ARG;
  }
  const ProductLayout L = product_layout(n, r, elt);
  if (workspace_bytes < L.total || reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) {
    set_error("cphifi_product: workspace must be >= %zu bytes, 256-byte aligned", L.total);
    return CPHIFI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  int num_cu = 256, dev = 0;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  const GemmPlan gp = make_gemm_plan(e, trans != 0, n, (int)r, mw, s, ksplit, num_cu);
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

}  // extern "C"
