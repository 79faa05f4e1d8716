// Host-side internals of the HNTL library: the index object, error plumbing and
// the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/hntl.h"

namespace hntl {

// Block-SoA layout (Section 2.4 of the paper, re-laid for wave64): the members
// of each grain occupy ceil(n_g / B) consecutive blocks of B = 64 vectors.  A
// block stores its tangent coordinates dimension-major, code[j][b] for
// j < rp and lane b < 64, followed nowhere by ids: a member's position
// (block-local lane + the grain's first position) maps to its original id
// through perm, read only for the candidates that survive the scan.  The rank
// is padded to rp = 8 * ceil(r / 8) with zero coordinates, and padding lanes
// of a grain's last block hold eps = +inf.
constexpr int B = HNTL_BLOCK;

// Learned router: MLP d -> h1 -> h2 -> G (FP32 masters, BF16 copies for the
// MFMA GEMMs) and the input standardisation.  Layer l: W[l] is out x in,
// row-major.
struct Router {
  int d = 0, h1 = 0, h2 = 0, G = 0;
  float* W[3] = {};
  float* b[3] = {};
  uint16_t* Wb[3] = {};
  float* mean = nullptr;
  float* stdv = nullptr;
  bool trained = false;
  void alloc(int d, int h1, int h2, int G);
  int64_t wsize(int l) const;
  int64_t bsize(int l) const;
  void refresh_bf16(hipStream_t s);
  ~Router();
};

struct Index;
// Buffers of one learned routing of up to nq queries.
struct RouterScratch {
  uint16_t *xh = nullptr, *h1 = nullptr, *h2 = nullptr;
  float* negS = nullptr;
  int32_t *fb_rows = nullptr, *fb_count = nullptr, *fb_probes = nullptr;
  float *fb_Q = nullptr, *fb_qn = nullptr, *fb_pdist = nullptr;
  float2* znorm = nullptr;  // per row: the smallest negated score and the softmax normaliser
  size_t layout(char* base, const Index& ix, int64_t nq, int P);
};

struct Index {
  int device = 0;
  uint64_t N = 0;
  uint32_t d = 0, G = 0, r = 0, rp = 0;
  uint64_t nblocks = 0;
  uint32_t codes_mask = 1u;
  uint32_t max_grain = 0;
  uint32_t kmeans_iters_run = 0;

  float* centroids = nullptr;  // G x d
  float* cnorm = nullptr;      // G, ||mu_g||^2
  float* basis = nullptr;      // G x r x d
  int32_t* goff = nullptr;     // G + 1 grain-order offsets
  int32_t* boff = nullptr;     // G + 1 block offsets
  int32_t* perm = nullptr;     // N
  float* codes = nullptr;      // nblocks x rp x B
  float* eps = nullptr;        // nblocks x B
  uint32_t* codes_bf16 = nullptr;  // nblocks x (rp / 2) x B words, 2 bf16 per word
  uint32_t* codes_fp8 = nullptr;   // nblocks x (rp / 4) x B words, 4 e4m3fn per word
  float* scales = nullptr;         // G fp8 scales
  uint32_t* codes_i16 = nullptr;   // nblocks x (rp / 2) x B words, 2 int16 per word (eq. 5 codes)
  float* i16_steps = nullptr;      // G x 4: inv_g, rinv_g, (1 / inv_g)^2, 1 / rinv_g
  float* eps_i16 = nullptr;        // nblocks x B: r_hat_i / rinv_g (0 past a grain's members)
  uint16_t* basis_bf16 = nullptr;  // G x r x d (bf16 bits)
  float* X = nullptr;          // N x d, original row order
  float* blo = nullptr;        // G x rp: per-grain minimum of each code coordinate
  float* bhi = nullptr;        // G x rp: per-grain maximum
  float* emin = nullptr;       // G: per-grain minimum eps_i
  int32_t* gorder = nullptr;   // G: grains by size, largest first (made by the first search plan)
  uint16_t* cent_split = nullptr;  // G x 3d bf16: [hi | lo | hi] of the centroids (split-BF16 routing, on first use)
  float* eps_id = nullptr;         // N: eps_i by original row id (Mode A answers, on first use)
  std::unique_ptr<Router> router;  // learned router (trained or imported), else null

  std::vector<int64_t> offsets_h;
  std::vector<int32_t> boff_h;
  std::vector<double> captured;  // per grain (build only)
  uint64_t device_bytes = 0;

  ~Index();
};

// ----------------------------------------------------------------- errors
void set_error(const std::string& msg);
hntl_status fail(hntl_status s, const std::string& msg);

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t _e = (expr);                                                                    \
    if (_e != hipSuccess)                                                                      \
      throw ::hntl::HipError(_e, std::string(#expr) + ": " + hipGetErrorString(_e));           \
  } while (0)

struct HipError {
  hipError_t code;
  std::string msg;
  HipError(hipError_t c, std::string m) : code(c), msg(std::move(m)) {}
};
struct ArgError {
  hntl_status code;
  std::string msg;
};

template <class T>
T* dev_alloc(Index* ix, size_t n) {
  void* p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) throw HipError(e, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  if (ix) ix->device_bytes += n * sizeof(T);
  return (T*)p;
}

// Stream-ordered scratch of one call: allocations are released on the stream
// when the object goes out of scope.
struct Scratch {
  hipStream_t s;
  std::vector<void*> ptrs;
  explicit Scratch(hipStream_t st) : s(st) {}
  template <class T>
  T* get(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMallocAsync(&p, n * sizeof(T), s);
    if (e != hipSuccess) throw HipError(e, "hipMallocAsync of " + std::to_string(n * sizeof(T)) + " bytes failed");
    ptrs.push_back(p);
    return (T*)p;
  }
  ~Scratch() {
    for (void* p : ptrs) (void)hipFreeAsync(p, s);
  }
};

// ----------------------------------------------------------- launchers
// routing / k-means distances: D[i][j] = ||a_i||^2 + ||b_j||^2 - 2 a_i . b_j
void launch_row_norms(const float* A, int64_t rows, int d, float* out, hipStream_t s);
// With nlim (device), rows from *nlim - row_base on are skipped (batches whose
// size lives in device memory).
// Split-BF16 routing distances: D (rows x G) = max(an + ||mu||^2 - 2 <a, mu>, 0) with
// <a, mu> from BF16 MFMA over [a_hi | a_hi | a_lo] . [mu_hi | mu_lo | mu_hi]; As is
// scratch of rows x 3d bf16.  ensure_centroid_split makes the index's centroid split once.
// launch_dist_bf16: the same with <a, mu> = bf16(a) . bf16(mu) (As: rows x d bf16).
void ensure_centroid_split(Index& ix, hipStream_t s);
void launch_dist_bf16x3(const Index& ix, const float* A, const float* an, int64_t rows, uint16_t* As, float* D,
                        hipStream_t s, const int32_t* nlim = nullptr, int64_t row_base = 0);
void launch_dist_bf16(const Index& ix, const float* A, const float* an, int64_t rows, uint16_t* As, float* D,
                      hipStream_t s, const int32_t* nlim = nullptr, int64_t row_base = 0);
void launch_dist_matrix(const float* A, const float* an, int64_t rows, const float* Bm, const float* bn,
                        int cols, int d, float* D, hipStream_t s, const int32_t* nlim = nullptr,
                        int64_t row_base = 0);
void launch_argmin_rows(const float* A, const float* an, int64_t rows, const float* Bm, const float* bn,
                        int cols, int d, int32_t* label, float* dmin, hipStream_t s);
// top-P per row of D; with A and Bm given, D holds expansion distances whose
// error is at most err (an[row] + bn[col]) and the winners are re-scored by
// exact direct differences (routing).  Rows beyond *nlim - row_base get probes
// -1.  overflow (optional, device) counts rows whose error window reached the
// end of the shortlist and were re-read whole.
void launch_topk_rows(const float* D, int64_t rows, int cols, int P, int32_t* idx, float* val, hipStream_t s,
                      const float* A = nullptr, const float* an = nullptr, const float* Bm = nullptr,
                      const float* bn = nullptr, int d = 0, float err = 0.f, const int32_t* nlim = nullptr,
                      int64_t row_base = 0, unsigned int* overflow = nullptr, float2* znorm = nullptr);

// Centroid routing (Section 2.1 step 1): the P nearest centroids of every row
// of Q by FP32 direct differences, from a shortlist of expansion distances
// whose products run on MFMA in one of three forms.
enum { ROUTE_F32 = 0, ROUTE_BF16 = 1, ROUTE_BF16X3 = 2 };
struct RouteScratch {
  int form = ROUTE_F32;
  int64_t chunk = 0;        // rows per distance block
  float* qn = nullptr;      // nq query norms
  float* D = nullptr;       // chunk x G expansion distances
  uint16_t* As = nullptr;   // chunk x d (BF16) or chunk x 3d (split BF16) query operands
  size_t layout(char* base, const Index& ix, int64_t nq, int form);
};
float route_err(int form);
inline int route_form(uint32_t flags) {
  return (flags & HNTL_FLAG_ROUTE_BF16X3) ? ROUTE_BF16X3 : (flags & HNTL_FLAG_ROUTE_BF16) ? ROUTE_BF16 : ROUTE_F32;
}
void launch_route_centroid(const Index& ix, const float* Q, int64_t nq, int P, const RouteScratch& w,
                           int32_t* probes, float* pdist, hipStream_t s, const int32_t* nlim = nullptr,
                           unsigned int* overflow = nullptr);

// exact k nearest rows of B (cols x d) for every row of A (rows x d), k <= 16:
// MFMA expansion shortlist of 32 per row, re-scored by direct differences
void launch_knn(const float* A, int64_t rows, const float* Bm, int64_t cols, int d, int k, int32_t* ids, float* dist,
                hipStream_t s);

// grain bucketing of (query, probe) pairs; work-item lists cut from it
enum { LIST_SLOT0 = 0, LIST_REST = 1, LIST_ALL = 2 };
struct ItemLists {
  int32_t* ioff[3];    // G + 1 each: exclusive prefix of items per grain
  int32_t* lstart[3];  // G each: first position of the list's pairs of grain g in `order`
  int32_t* lcount[3];  // G each: number of the list's pairs of grain g
  int tile[3];         // pairs per work item
};
struct Buckets {
  int32_t* gcount;   // G: pairs per grain
  int32_t* gcount0;  // G: probe-slot-0 pairs per grain
  int32_t* gstart;   // G
  int32_t* cur0;     // G
  int32_t* cur1;     // G
  int32_t* order;    // npairs: pair ids grouped by grain, slot-0 pairs first
  ItemLists lists;
  int max_items[3];  // upper bounds of the item counts (grid sizes)
  int G;
};
void launch_bucket(const int32_t* probes, int64_t nq, int P, int G, Buckets& b, hipStream_t s,
                   const int32_t* gorder = nullptr, const int32_t* nsplit = nullptr, bool counts_zeroed = false);
// up to 8 fills in one launch (graph-friendly resets)
struct FillSeg {
  int32_t* p;
  int64_t n;
  int32_t v;
};
struct FillList {
  FillSeg seg[8];
  int n;
};
void launch_fill_multi(const FillList& L, hipStream_t s);
// One work item of the fused kernel, decoded once per run: a projection item
// (16 pairs of grain g from order[off]) or a scan item (cnt pairs of grain g
// from order[off] against block range `range`; its pairs' tangents come from
// projection items c0 .. c1).
struct ItemDesc {
  int32_t g, range, off, cnt, c0, c1, pad0, pad1;
};
// Items 0 .. nP-1 are the projection items (LIST_ALL, 16 pairs), then the
// scan items of LIST_SLOT0 and LIST_REST (qt pairs x block ranges), in the
// lists' item order; threads past the device item count write nothing.
void launch_item_table(const ItemLists& lists, const int32_t* gorder, int G, int qt, int64_t max_items,
                       ItemDesc* out, hipStream_t s);
void launch_pair_lists(const int32_t* probes, int64_t nq, int P, int G, const int32_t* nsplit, int32_t* lbase,
                       int32_t* qoff, hipStream_t s);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);

constexpr int PROJECT_TILE = 64;  // pairs per workgroup of the shared-basis projection kernel
// Projection item size (LIST_ALL tile) for queries Q: PROJECT_TILE where the
// shared-basis kernel applies (vector loads: d % 4 == 0 FP32, d % 8 == 0 BF16,
// 16-byte aligned Q), else 16.
int project_tile(const Index& ix, const float* Q, bool bf16);
// gorder: the rank -> grain map when the buckets were built in that order (ioff by rank), else null
void launch_project(const Index& ix, const float* Q, int P, const Buckets& b, float* T, float* epsq, bool bf16,
                    const int32_t* gorder, hipStream_t s);  // over LIST_ALL
// Scan of the bucketed pairs.  With `bound_lists` (the lists of probe slot 0,
// already written into part), each pair starts from its query's C-th key of
// slot 0 as threshold and, when `prune`, is skipped outright if an exact
// lower bound of eq. 6 over its grain exceeds that threshold.
void launch_scan(const Index& ix, int codes, const float* T, const float* epsq, int P, int C,
                 const Buckets& b, int list, uint64_t* part, const uint64_t* bound_lists, bool prune,
                 unsigned long long* scored, hipStream_t s);
void launch_grain_bounds(Index& ix, hipStream_t s);
// Before the slot-0 pass of the staged scan: entry C - 1 of each query's
// slot-0 list := KEY_NONE (part is nq x P x C keys).
void launch_reset_slot0_tail(uint64_t* part, int64_t nq, int P, int C, hipStream_t s);
// Build-side steps shared by the build and the append (build.hip).
void pca_encode_grains(Index* ix, const int64_t* d_off, const std::vector<int32_t>& glist, uint32_t eig_iters,
                       uint64_t seed, uint64_t stream_base, hipStream_t s);
// Exact member means (FP64 sums in member order) of grains gmap[0 .. ng-1]
// (gmap null: grains 0 .. ng-1).
void launch_segmented_mean(const float* X, int d, const int32_t* order, const int64_t* off, const int* gmap, int ng,
                           float* cent, hipStream_t s);
// eps_i by original id, made once (Mode A).
void ensure_eps_by_id(Index& ix, hipStream_t s);
// eps_id != null: Mode A (reconstruction distances of the pool, no raw vectors).
void launch_merge_rerank(const Index& ix, const float* Q, int64_t nq, int P, int C, int k,
                         const int32_t* probes, const uint64_t* part, const int32_t* pool_in, int32_t* pool_out,
                         float* pool_D_out, int32_t* ids, float* dist, hipStream_t s,
                         const int32_t* qoff = nullptr, const float* eps_id = nullptr,
                         const int32_t* nlim = nullptr);  // rows from *nlim on: -1 / +inf only

// Persistent fused project-scan-select kernel (the batching form).  Its
// waves take work items from one device ticket counter, in three runs:
// projection items (LIST_ALL, 16 pairs), then scan items of probe slot 0,
// then scan items of the other slots (QT pairs, one item per block range of
// R blocks; R = 0 scans whole grains).  Inside each run items follow the
// grain order `gorder` (largest grain first).
struct FusedArgs {
  // index
  const void* codes;
  const float* scales;
  const float* eps;
  const int32_t* goff;
  const int32_t* boff;
  const int32_t* perm;
  const float* blo;
  const float* bhi;
  const float* emin;
  const float* centroids;
  const float* basis;
  const uint16_t* basis16;
  int d, r, G, P, C;
  // batch
  const float* Q;
  // work items
  const int32_t* ioff[3];  // indexed by grain rank
  const int32_t* lstart[3];
  const int32_t* lcount[3];
  const int32_t* gorder;
  const int32_t* order;
  const int32_t* lbase;  // per pair: first list slot (null: the pair id)
  int R;
  int phase;  // 0: every item; 1: projection + slot-0 items; 2: the other slots
  // shared state (reset before every launch)
  int32_t* ticket;     // 1
  int32_t* proj_done;  // one flag per projection item: 1 once its tangents are written
  uint32_t* qbound;    // per query: order image of the smallest known C-th distance
  int32_t* err;        // 1: set if a wait gave up
  float* T;            // npairs x r tangents
  float* epsq;         // npairs
  uint64_t* part;      // lists x C keys
  unsigned long long* scored;
  int proj_bf16;
  int proj_ext;  // 1: tangents come from a separate projection launch (no projection items, no waits)
  const ItemDesc* items;  // decoded work items, in ticket order
  int prune;
};

// learned routing: probes by descending router score (three BF16 MFMA layer
// products with fused bias / GELU epilogues, then a top-P over the scores);
// rows whose largest softmax probability is below tau fall back to centroid
// routing.  Rows from *nlim on are skipped.
// mass in (0, 1): each learned row keeps its probes up to the first slot at
// which the cumulative softmax probability reaches mass (later slots: -1).
void launch_route_learned(const Index& ix, const float* Q, int64_t nq, int P, float tau, int32_t* probes,
                          float* pdist, const RouterScratch& w, hipStream_t s, const int32_t* nlim = nullptr,
                          float mass = 0.f);

// build helpers
void launch_pack_codes(const Index& ix, const float* codes_go, const float* eps_go, hipStream_t s);
void launch_derive_lowp(Index& ix, hipStream_t s);

int pow2_at_least(int x);

}  // namespace hntl

// The opaque handle of the C ABI.
struct hntl_index {
  hntl::Index ix;
};
