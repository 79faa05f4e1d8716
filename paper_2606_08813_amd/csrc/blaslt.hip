// Plain library GEMMs (hipBLASLt) for the dot products of centroid routing
// (§2.1 step 1, §2.3) and the learned router's layers: D = alpha A . B^T
// with A (rows x k) and B (cols x k) both row-major, BF16 or
// FP32 operands, FP32 accumulation and FP32 output (HIPBLAS_COMPUTE_32F: no
// reduced-precision FP32 path), D row-major (rows x cols).  In the library's column-major terms D^T (cols x rows) =
// B (k x cols, transposed) . A (k x rows): the TN layout.
//
// Descriptors are made once per (device, type, shape) by lt_gemm_prepare,
// which must run outside graph capture; lt_gemm_abt then only enqueues the
// library kernel (capturable).  No workspace is given to the library.  The
// algorithm is the heuristic's pick for a fixed reference row count, used for
// every row count it supports: one kernel, and so one summation order per
// output element, whatever the batch size, so that a row's result does not
// depend on the rows searched with it.
#include <hipblaslt/hipblaslt-ext.hpp>
#include <hipblaslt/hipblaslt.h>

#include <map>
#include <mutex>
#include <tuple>

#include "hntl_internal.h"

namespace hntl {
namespace {

struct LtShape {
  hipblasLtMatmulDesc_t desc = nullptr;
  hipblasLtMatrixLayout_t la = nullptr, lb = nullptr, ld = nullptr;
  hipblasLtMatmulAlgo_t algo{};
  bool ok = false;
};

struct LtDevice {
  hipblasLtHandle_t h = nullptr;
  std::map<std::tuple<int, int64_t, int64_t, int64_t>, LtShape> shapes;
};

std::mutex g_lt_mu;
LtDevice g_lt[64];
constexpr int64_t LT_REF_ROWS = 16384;

void lt_check(hipblasStatus_t st, const char* what) {
  if (st != HIPBLAS_STATUS_SUCCESS) throw HipError(hipErrorUnknown, std::string("hipBLASLt ") + what + " failed");
}

// The shape's descriptors (made on first use); null when the library has no
// algorithm for it.  Caller holds g_lt_mu.
LtShape* shape_locked(int dev, int dt, int64_t rows, int64_t cols, int64_t k) {
  LtDevice& D = g_lt[dev];
  auto key = std::make_tuple(dt, rows, cols, k);
  auto it = D.shapes.find(key);
  if (it != D.shapes.end()) return it->second.ok ? &it->second : nullptr;
  if (!D.h) lt_check(hipblasLtCreate(&D.h), "create");
  LtShape sh;
  const hipDataType in = dt == LT_BF16 ? HIP_R_16BF : HIP_R_32F;
  lt_check(hipblasLtMatmulDescCreate(&sh.desc, HIPBLAS_COMPUTE_32F, HIP_R_32F), "desc");
  const hipblasOperation_t ta = HIPBLAS_OP_T, tb = HIPBLAS_OP_N;
  lt_check(hipblasLtMatmulDescSetAttribute(sh.desc, HIPBLASLT_MATMUL_DESC_TRANSA, &ta, sizeof(ta)), "transa");
  lt_check(hipblasLtMatmulDescSetAttribute(sh.desc, HIPBLASLT_MATMUL_DESC_TRANSB, &tb, sizeof(tb)), "transb");
  // library A = our B (k x cols, ld k), library B = our A (k x rows, ld k), D (cols x rows, ld cols)
  lt_check(hipblasLtMatrixLayoutCreate(&sh.la, in, (uint64_t)k, (uint64_t)cols, k), "layout a");
  lt_check(hipblasLtMatrixLayoutCreate(&sh.lb, in, (uint64_t)k, (uint64_t)rows, k), "layout b");
  lt_check(hipblasLtMatrixLayoutCreate(&sh.ld, HIP_R_32F, (uint64_t)cols, (uint64_t)rows, cols), "layout d");
  hipblasLtMatmulPreference_t pref = nullptr;
  lt_check(hipblasLtMatmulPreferenceCreate(&pref), "preference");
  const uint64_t ws = 0;
  lt_check(hipblasLtMatmulPreferenceSetAttribute(pref, HIPBLASLT_MATMUL_PREF_MAX_WORKSPACE_BYTES, &ws, sizeof(ws)),
           "workspace");
  // the heuristic's algorithm for the reference row count, checked for this shape
  hipblasLtMatrixLayout_t lb_ref = nullptr, ld_ref = nullptr;
  lt_check(hipblasLtMatrixLayoutCreate(&lb_ref, in, (uint64_t)k, (uint64_t)LT_REF_ROWS, k), "layout b");
  lt_check(hipblasLtMatrixLayoutCreate(&ld_ref, HIP_R_32F, (uint64_t)cols, (uint64_t)LT_REF_ROWS, cols), "layout d");
  hipblasLtMatmulHeuristicResult_t res[1];
  int got = 0;
  const hipblasStatus_t st =
      hipblasLtMatmulAlgoGetHeuristic(D.h, sh.desc, sh.la, lb_ref, ld_ref, ld_ref, pref, 1, res, &got);
  (void)hipblasLtMatmulPreferenceDestroy(pref);
  (void)hipblasLtMatrixLayoutDestroy(lb_ref);
  (void)hipblasLtMatrixLayoutDestroy(ld_ref);
  if (st == HIPBLAS_STATUS_SUCCESS && got > 0 && res[0].state == HIPBLAS_STATUS_SUCCESS && res[0].workspaceSize == 0) {
    const float one = 1.f, zero = 0.f;
    size_t need = 0;
    if (hipblaslt_ext::matmulIsAlgoSupported(D.h, sh.desc, &one, sh.la, sh.lb, &zero, sh.ld, sh.ld, res[0].algo,
                                             need) == HIPBLAS_STATUS_SUCCESS &&
        need == 0) {
      sh.algo = res[0].algo;
      sh.ok = true;
    }
  }
  auto& slot = D.shapes[key];
  slot = sh;
  return slot.ok ? &slot : nullptr;
}

}  // namespace

bool lt_gemm_prepare(int dt, int64_t rows, int64_t cols, int64_t k) {
  if (rows <= 0 || cols <= 0 || k <= 0) return false;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return false;
  std::lock_guard<std::mutex> lk(g_lt_mu);
  return shape_locked(dev, dt, rows, cols, k) != nullptr;
}

bool lt_gemm_abt(int dt, const void* A, const void* B, float* D, int64_t rows, int64_t cols, int64_t k,
                 hipStream_t s, float alpha) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return false;
  std::lock_guard<std::mutex> lk(g_lt_mu);
  LtShape* sh = shape_locked(dev, dt, rows, cols, k);
  if (!sh) return false;
  const float zero = 0.f;
  lt_check(hipblasLtMatmul(g_lt[dev].h, sh->desc, &alpha, B, sh->la, A, sh->lb, &zero, D, sh->ld, D, sh->ld,
                           &sh->algo, nullptr, 0, s),
           "matmul");
  return true;
}

}  // namespace hntl
