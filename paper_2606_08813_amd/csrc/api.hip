// C ABI of the HNTL library: argument checking, index import/export and the
// search pipeline (route -> bucket -> project -> scan -> merge/rerank).
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>

#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

hntl_status fail(hntl_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

Index::~Index() {
  void* ptrs[] = {centroids, cnorm,    basis,   goff,      boff,     perm,       codes,  eps,
                  codes_bf16, codes_fp8, scales, basis_bf16, codes_i16, i16_steps, eps_i16, X,
                  blo,       bhi,       emin,   gorder,     cent_split, eps_id};
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(device);
  router.reset();
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  (void)hipSetDevice(prev);
}

namespace {

std::mutex g_pool_mu;
bool g_pool_done[64] = {};

void ensure_pool(int dev) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (dev < 0 || dev >= 64 || g_pool_done[dev]) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = std::numeric_limits<uint64_t>::max();
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  g_pool_done[dev] = true;
}

// Run f and turn exceptions into status codes.
template <class F>
hntl_status guarded(F&& f) {
  try {
    f();
    return HNTL_OK;
  } catch (const ArgError& e) {
    return fail(e.code, e.msg);
  } catch (const HipError& e) {
    return fail(e.code == hipErrorOutOfMemory || e.code == hipErrorMemoryAllocation ? HNTL_ENOMEM : HNTL_EDEVICE,
                e.msg);
  } catch (const std::bad_alloc&) {
    return fail(HNTL_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(HNTL_EDEVICE, e.what());
  }
}

void require(bool ok, const std::string& msg, hntl_status code = HNTL_EINVAL) {
  if (!ok) throw ArgError{code, msg};
}

template <class T>
std::vector<T> to_host(const T* p, size_t n) {
  std::vector<T> v(n);
  if (n) HIP_TRY(hipMemcpy(v.data(), p, n * sizeof(T), hipMemcpyDefault));
  return v;
}

template <class T>
T* upload(Index* ix, const T* src, size_t n) {
  T* d = dev_alloc<T>(ix, n);
  if (n) HIP_TRY(hipMemcpy(d, src, n * sizeof(T), hipMemcpyDefault));
  return d;
}

// Per-thread record of HIP events for HNTL_FLAG_PROFILE.
struct ProfRec {
  hipEvent_t ev[HNTL_NUM_STAGES + 1];
  bool used[HNTL_NUM_STAGES];
};
struct Profiler {
  std::vector<hipEvent_t> pool;
  std::vector<ProfRec> recs;
  unsigned long long* scored = nullptr;  // device counter of (pair, member) scores
  int scored_dev = -1;
  unsigned long long* counter(int dev) {
    if (!scored || scored_dev != dev) {
      HIP_TRY(hipMalloc((void**)&scored, sizeof(unsigned long long)));
      HIP_TRY(hipMemset(scored, 0, sizeof(unsigned long long)));
      scored_dev = dev;
    }
    return scored;
  }
  ~Profiler() {
    for (auto& r : recs)
      for (auto e : r.ev) pool.push_back(e);
    for (auto e : pool) (void)hipEventDestroy(e);
  }
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    return e;
  }
};
thread_local Profiler g_prof;

// Marks stage boundaries of one profiled call.
struct StageClock {
  bool on;
  hipStream_t s;
  ProfRec rec{};
  int cur = -1;
  StageClock(bool enable, hipStream_t st) : on(enable), s(st) {
    if (!on) return;
    for (int i = 0; i <= HNTL_NUM_STAGES; ++i) rec.ev[i] = g_prof.get();
    for (int i = 0; i < HNTL_NUM_STAGES; ++i) rec.used[i] = false;
  }
  // enter stage i (stages are entered in increasing order)
  void at(int i) {
    if (!on) return;
    HIP_TRY(hipEventRecord(rec.ev[i], s));
    for (int j = cur + 1; j < i; ++j) HIP_TRY(hipEventRecord(rec.ev[j], s));
    rec.used[i] = true;
    cur = i;
  }
  void done() {
    if (!on) return;
    for (int j = cur + 1; j <= HNTL_NUM_STAGES; ++j) HIP_TRY(hipEventRecord(rec.ev[j], s));
    g_prof.recs.push_back(rec);
    on = false;
  }
  ~StageClock() {
    if (on)
      for (auto e : rec.ev) g_prof.pool.push_back(e);
  }
};

__global__ void nonfinite_kernel(const float* __restrict__ A, int64_t n, int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(A[i])) atomicOr(flag, 1);
}

// Caller buffers of one staged search (any stage input may be injected, any
// stage output observed; see hntl_search_stages).
// Non-finite query values are rejected (EINVAL) by every call that returns
// after its work has finished: HNTL_FLAG_SYNC, or HNTL_FLAG_CHECK_Q (which
// implies the wait).  An asynchronous call cannot report them.
inline bool checks_queries(const hntl_search_params& sp) {
  return (sp.flags & (HNTL_FLAG_CHECK_Q | HNTL_FLAG_SYNC)) != 0;
}

struct StagedIO {
  const int32_t* probes_in;
  int32_t* probes_out;
  float* pdist_out;
  const float* tangent_in;
  const float* epsq_in;
  float* tangent_out;
  float* epsq_out;
  const int32_t* pool_in;
  int32_t* pool_out;
  float* pool_D_out;
  int32_t* ids;
  float* dist;
};

hntl_status check_search(const hntl_index* index, const float* Q, uint32_t nq, const hntl_search_params* sp,
                         const StagedIO& io) {
  if (!index || !sp) return fail(HNTL_EINVAL, "null index or params");
  const Index& ix = index->ix;
  const uint32_t P = sp->P, C = sp->C, k = sp->k;
  if (P < 1 || P > ix.G) return fail(HNTL_EINVAL, "need 1 <= P <= G");
  if (P > HNTL_MAX_P) return fail(HNTL_EUNSUPPORTED, "P exceeds HNTL_MAX_P");
  if (k < 1 || C < k) return fail(HNTL_EINVAL, "need 1 <= k <= C");
  if (C > HNTL_MAX_C) return fail(HNTL_EUNSUPPORTED, "C exceeds HNTL_MAX_C");
  if (sp->codes > HNTL_CODES_INT16) return fail(HNTL_EINVAL, "unknown codes form");
  if (sp->codes == HNTL_CODES_INT16 && (sp->flags & HNTL_FLAG_MODE_A))
    return fail(HNTL_EUNSUPPORTED, "Mode A answers use the FP32 / BF16 / FP8 code forms");
  if (!(ix.codes_mask & (1u << sp->codes))) return fail(HNTL_ESTATE, "codes form not built for this index");
  if ((io.tangent_in == nullptr) != (io.epsq_in == nullptr))
    return fail(HNTL_EINVAL, "tangent_in and epsq_in go together");
  if (sp->route > HNTL_ROUTE_LEARNED) return fail(HNTL_EINVAL, "unknown route");
  if ((sp->flags & HNTL_FLAG_ROUTE_BF16X3) && (sp->flags & HNTL_FLAG_ROUTE_BF16))
    return fail(HNTL_EINVAL, "choose one centroid routing form");
  if (!(sp->mass >= 0.f && sp->mass <= 1.f)) return fail(HNTL_EINVAL, "mass must lie in [0, 1]");
  const bool learned = sp->route == HNTL_ROUTE_LEARNED && !io.probes_in && !io.pool_in;
  if (learned && !(ix.router && ix.router->trained)) return fail(HNTL_ESTATE, "learned routing needs a trained router");
  const bool mode_a = (sp->flags & HNTL_FLAG_MODE_A) != 0;
  if (!mode_a && !ix.X) return fail(HNTL_ESTATE, "this index holds no raw vectors: only Mode A searches");
  if (mode_a && io.pool_in) return fail(HNTL_EUNSUPPORTED, "Mode A answers need the merged pool, not an injected one");
  if (nq == 0) return HNTL_OK;
  if (!Q || !io.ids || !io.dist) return fail(HNTL_EINVAL, "Q, ids and dist are required");
  return HNTL_OK;
}

bool routes_by_centroid(const hntl_search_params& sp, const StagedIO& io) {
  return !io.pool_in && !io.probes_in && sp.route != HNTL_ROUTE_LEARNED;
}

// Index data a search derives on first use: the split centroid operands of
// the BF16 routing forms and eps by row id for Mode A.
void derive_search_data(Index& ix, const hntl_search_params& sp, const StagedIO& io, hipStream_t s) {
  if (routes_by_centroid(sp, io) && route_form(sp.flags) != ROUTE_F32) ensure_centroid_split(ix, s);
  if (sp.flags & HNTL_FLAG_MODE_A) ensure_eps_by_id(ix, s);
}

bool search_data_ready(const Index& ix, const hntl_search_params& sp, const StagedIO& io) {
  if (routes_by_centroid(sp, io) && route_form(sp.flags) != ROUTE_F32 && !ix.cent_split) return false;
  if ((sp.flags & HNTL_FLAG_MODE_A) && !ix.eps_id) return false;
  return true;
}

// Scratch of one staged search, carved from one block (base == nullptr: the
// sizing pass, which returns the bytes needed).
struct StagedScratch {
  int* qflag = nullptr;      // non-finite query flag (HNTL_FLAG_CHECK_Q)
  int32_t* probes = nullptr;  // probes when the caller observes none
  RouterScratch rw;
  RouteScratch cw;
  Buckets b{};
  float* T = nullptr;
  float* eq = nullptr;
  uint64_t* part = nullptr;

  size_t layout(char* base, const Index& ix, const float* Q, uint32_t nq, const hntl_search_params& sp,
                const StagedIO& io) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
      off = (off + 255) / 256 * 256;
      char* p = base ? base + off : nullptr;
      off += std::max<size_t>(bytes, 1);
      return p;
    };
    const int64_t P = sp.P, npairs = (int64_t)nq * P;
    if (checks_queries(sp)) qflag = (int*)take(sizeof(int));
    if (io.pool_in) return off;
    if (!io.probes_in) {
      if (!io.probes_out) probes = (int32_t*)take(sizeof(int32_t) * npairs);
      if (sp.route == HNTL_ROUTE_LEARNED) {
        char* rb = take(rw.layout(nullptr, ix, nq, (int)P));
        rw.layout(rb, ix, nq, (int)P);
      } else {
        const int form = route_form(sp.flags);
        char* rb = take(cw.layout(nullptr, ix, nq, form));
        cw.layout(rb, ix, nq, form);
      }
    }
    b.G = (int)ix.G;
    b.gcount = (int32_t*)take(4 * (size_t)ix.G);
    b.gcount0 = (int32_t*)take(4 * (size_t)ix.G);
    b.gstart = (int32_t*)take(4 * (size_t)ix.G);
    b.cur0 = (int32_t*)take(4 * (size_t)ix.G);
    b.cur1 = (int32_t*)take(4 * (size_t)ix.G);
    b.order = (int32_t*)take(4 * (size_t)npairs);
    // the projection item size depends only on d, the code form and Q's alignment
    const int tiles[3] = {16, 16, project_tile(ix, Q, (sp.flags & HNTL_FLAG_PROJECT_BF16) != 0)};
    const int64_t np[3] = {(int64_t)nq, (int64_t)nq * (P - 1), npairs};
    for (int L = 0; L < 3; ++L) {
      b.lists.tile[L] = tiles[L];
      b.lists.ioff[L] = (int32_t*)take(4 * ((size_t)ix.G + 1));
      b.lists.lstart[L] = (int32_t*)take(4 * (size_t)ix.G);
      b.lists.lcount[L] = (int32_t*)take(4 * (size_t)ix.G);
      b.max_items[L] = (int)(np[L] / tiles[L] + std::min<int64_t>(ix.G, np[L]) + 1);
    }
    if (!io.tangent_in) {
      if (!io.tangent_out) T = (float*)take(4 * (size_t)npairs * ix.r);
      if (!io.epsq_out) eq = (float*)take(4 * (size_t)npairs);
    }
    part = (uint64_t*)take(8 * (size_t)npairs * sp.C);
    return off;
  }
};

// The staged search's launch sequence on scratch w (laid out for this call).
void run_staged(const Index& ix, const float* Q, uint32_t nq, const hntl_search_params& sp, const StagedIO& io,
                StagedScratch& w, hipStream_t s) {
  const uint32_t P = sp.P, C = sp.C, k = sp.k;
  if (checks_queries(sp)) {
    launch_fill_i32(w.qflag, 1, 0, s);
    const int64_t n = (int64_t)nq * ix.d;
    hipLaunchKernelGGL(nonfinite_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Q, n, w.qflag);
    HIP_TRY(hipGetLastError());
    int hflag = 0;
    HIP_TRY(hipMemcpyAsync(&hflag, w.qflag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    require(hflag == 0, "queries contain NaN or Inf");
  }
  const bool mode_a = (sp.flags & HNTL_FLAG_MODE_A) != 0;
  StageClock clk((sp.flags & HNTL_FLAG_PROFILE) != 0, s);
  const uint64_t* part = nullptr;
  const int32_t* probes = io.probes_in;
  if (!io.pool_in) {
    // 1. routing
    if (!probes) {
      clk.at(HNTL_STAGE_ROUTE);
      int32_t* pr = io.probes_out ? io.probes_out : w.probes;
      if (sp.route == HNTL_ROUTE_LEARNED)
        launch_route_learned(ix, Q, nq, (int)P, sp.tau, pr, io.pdist_out, w.rw, s, nullptr, sp.mass);
      else
        launch_route_centroid(ix, Q, nq, (int)P, w.cw, pr, io.pdist_out, s);
      probes = pr;
    }
    // 2. bucketing by grain (each grain's probe-slot-0 pairs first, so that
    //    slot 0 is scanned first and its C-th key bounds the other slots)
    clk.at(HNTL_STAGE_BUCKET);
    launch_bucket(probes, nq, (int)P, (int)ix.G, w.b, s);
    // 3. projection
    const float* T = io.tangent_in;
    const float* eq = io.epsq_in;
    if (!T) {
      clk.at(HNTL_STAGE_PROJECT);
      float* To = io.tangent_out ? io.tangent_out : w.T;
      float* eo = io.epsq_out ? io.epsq_out : w.eq;
      launch_project(ix, Q, (int)P, w.b, To, eo, (sp.flags & HNTL_FLAG_PROJECT_BF16) != 0, nullptr, s);
      T = To;
      eq = eo;
    }
    // 4. scan + per-pair top-C: slot 0 unbounded, then the other slots
    //    bounded by it (and pruned by the exact lower bound unless disabled)
    uint64_t* pt = w.part;
    clk.at(HNTL_STAGE_SCAN);
    unsigned long long* scored = (sp.flags & HNTL_FLAG_PROFILE) ? g_prof.counter(ix.device) : nullptr;
    if (P > 1) launch_reset_slot0_tail(pt, nq, (int)P, (int)C, s);
    launch_scan(ix, (int)sp.codes, T, eq, (int)P, (int)C, w.b, LIST_SLOT0, pt, nullptr, false, scored, s);
    if (P > 1) {
      const bool bounded = !(sp.flags & HNTL_FLAG_NO_PRUNE);
      launch_scan(ix, (int)sp.codes, T, eq, (int)P, (int)C, w.b, LIST_REST, pt, bounded ? pt : nullptr, bounded,
                  scored, s);
    }
    part = pt;
  }
  // 5. pool merge + exact rerank
  clk.at(HNTL_STAGE_RERANK);
  launch_merge_rerank(ix, Q, nq, (int)P, (int)C, (int)k, probes, part, io.pool_in, io.pool_out, io.pool_D_out, io.ids,
                      io.dist, s, nullptr, mode_a ? ix.eps_id : nullptr);
  clk.done();
  if (sp.flags & HNTL_FLAG_SYNC) {
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
  }
}

// Scratch of hntl_search_noalloc: one static device array per GPU, held until
// the process ends.  Its address on a device comes from hipGetSymbolAddress,
// taken once per device with that device current; host code never passes
// the array's own name to a kernel or a copy (on the host it is only a
// stand-in, not a device address).
__device__ __align__(256) unsigned char scratch[HNTL_NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

// Device address of this device's scratch array (the current device).
char* noalloc_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= 64) throw ArgError{HNTL_EUNSUPPORTED, "device ordinal above 63"};
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw ArgError{HNTL_EDEVICE, "no device address for the static scratch array"};
    g_scratch_ptr[dev] = p;
  }
  return static_cast<char*>(g_scratch_ptr[dev]);
}

}  // namespace

// Finish an index whose host-side grain offsets, codes and eps (grain order) are
// known: block offsets, Block-SoA packing, centroid norms.
void finish_index(Index* ix, const std::vector<int64_t>& off, const float* codes_go_host, const float* eps_go_host) {
  const uint32_t G = ix->G, r = ix->r, rp = ix->rp;
  ix->offsets_h = off;
  ix->boff_h.assign(G + 1, 0);
  uint32_t maxg = 0;
  for (uint32_t g = 0; g < G; ++g) {
    const int64_t n = off[g + 1] - off[g];
    maxg = std::max<uint32_t>(maxg, (uint32_t)n);
    ix->boff_h[g + 1] = ix->boff_h[g] + (int32_t)((n + B - 1) / B);
  }
  ix->max_grain = maxg;
  ix->nblocks = (uint64_t)ix->boff_h[G];
  std::vector<float> blk((size_t)ix->nblocks * rp * B, 0.f);
  std::vector<float> eb((size_t)ix->nblocks * B, std::numeric_limits<float>::infinity());
  for (uint32_t g = 0; g < G; ++g) {
    const int64_t a = off[g], n = off[g + 1] - off[g];
    for (int64_t i = 0; i < n; ++i) {
      const int64_t blkid = ix->boff_h[g] + i / B, lane = i % B;
      const float* z = codes_go_host + (size_t)(a + i) * r;
      float* dst = blk.data() + (size_t)blkid * rp * B + lane;
      for (uint32_t j = 0; j < r; ++j) dst[(size_t)j * B] = z[j];
      eb[(size_t)blkid * B + lane] = eps_go_host[a + i];
    }
  }
  std::vector<int32_t> goff32(G + 1);
  for (uint32_t g = 0; g <= G; ++g) goff32[g] = (int32_t)off[g];
  ix->goff = upload(ix, goff32.data(), G + 1);
  ix->boff = upload(ix, ix->boff_h.data(), G + 1);
  ix->codes = upload(ix, blk.data(), blk.size());
  ix->eps = upload(ix, eb.data(), eb.size());
  ix->cnorm = dev_alloc<float>(ix, G);
  launch_row_norms(ix->centroids, G, (int)ix->d, ix->cnorm, nullptr);
  launch_grain_bounds(*ix, nullptr);
  HIP_TRY(hipDeviceSynchronize());
}

}  // namespace hntl

using namespace hntl;

extern "C" {

const char* hntl_last_error(void) { return g_last_error.c_str(); }

const char* hntl_version(void) { return "hntl-mi355x 0.1 (gfx950)"; }

void hntl_index_free(hntl_index* index) { delete index; }

hntl_status hntl_index_create(uint64_t N, uint32_t d, uint32_t G, uint32_t r, const float* centroids,
                              const float* basis, const int64_t* offsets, const int32_t* perm, const float* codes,
                              const float* eps, const float* X, uint32_t codes_mask, hntl_index** out) {
  g_last_error.clear();
  if (!out) return fail(HNTL_EINVAL, "out is NULL");
  *out = nullptr;
  if (!centroids || !basis || !offsets || !perm || !codes || !eps)
    return fail(HNTL_EINVAL, "null array pointer");  // X may be null: an index for Mode A answers only
  if (N == 0 || d == 0 || G == 0 || r == 0) return fail(HNTL_EINVAL, "N, d, G and r must be positive");
  if (G > N) return fail(HNTL_EINVAL, "G > N");
  if (r > d) return fail(HNTL_EINVAL, "r > d");
  if (r > HNTL_MAX_R) return fail(HNTL_EUNSUPPORTED, "r exceeds HNTL_MAX_R");
  if (N >= (1ull << 31)) return fail(HNTL_EUNSUPPORTED, "N must be below 2^31");
  hntl_index* h = nullptr;
  hntl_status st = guarded([&] {
    int dev = 0;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) throw ArgError{HNTL_EDEVICE, "no GPU device"};
    HIP_TRY(hipGetDevice(&dev));
    auto off = to_host(offsets, (size_t)G + 1);
    require(off[0] == 0 && off[G] == (int64_t)N, "offsets must start at 0 and end at N");
    for (uint32_t g = 0; g < G; ++g) require(off[g + 1] >= off[g], "offsets must be non-decreasing");
    auto pm = to_host(perm, (size_t)N);
    std::vector<uint8_t> seen(N, 0);
    for (uint64_t i = 0; i < N; ++i) {
      require(pm[i] >= 0 && (uint64_t)pm[i] < N && !seen[pm[i]], "perm must be a permutation of 0..N-1");
      seen[pm[i]] = 1;
    }
    for (uint32_t g = 0; g < G; ++g)
      for (int64_t i = off[g] + 1; i < off[g + 1]; ++i)
        require(pm[i] > pm[i - 1], "ids inside a grain must ascend");
    auto cz = to_host(codes, (size_t)N * r);
    auto ce = to_host(eps, (size_t)N);
    for (uint64_t i = 0; i < N; ++i) require(ce[i] >= 0.f && std::isfinite(ce[i]), "eps must be finite and >= 0");
    h = new hntl_index();
    Index* ix = &h->ix;
    ix->device = dev;
    ix->N = N;
    ix->d = d;
    ix->G = G;
    ix->r = r;
    ix->rp = (r + 7) / 8 * 8;
    ix->centroids = upload(ix, centroids, (size_t)G * d);
    ix->basis = upload(ix, basis, (size_t)G * r * d);
    ix->perm = upload(ix, pm.data(), N);
    if (X) ix->X = upload(ix, X, (size_t)N * d);
    finish_index(ix, off, cz.data(), ce.data());
    ix->captured.assign(G, -1.0);
    ix->codes_mask = 1u;
    if (codes_mask & ~1u) {
      ix->codes_mask |= codes_mask & ((1u << HNTL_CODES_BF16) | (1u << HNTL_CODES_FP8_E4M3) | (1u << HNTL_CODES_INT16));
      launch_derive_lowp(*ix, nullptr);
      HIP_TRY(hipDeviceSynchronize());
    }
  });
  if (st != HNTL_OK) {
    delete h;
    return st;
  }
  *out = h;
  return HNTL_OK;
}

hntl_status hntl_index_export(const hntl_index* index, float* centroids, float* basis, int64_t* offsets,
                              int32_t* perm, float* codes, float* eps, float* scales) {
  g_last_error.clear();
  if (!index) return fail(HNTL_EINVAL, "index is NULL");
  const Index& ix = index->ix;
  if (scales && !ix.scales) return fail(HNTL_ESTATE, "FP8 codes were not built");
  return guarded([&] {
    const uint32_t G = ix.G, r = ix.r, rp = ix.rp, d = ix.d;
    if (centroids) HIP_TRY(hipMemcpy(centroids, ix.centroids, sizeof(float) * G * d, hipMemcpyDefault));
    if (basis) HIP_TRY(hipMemcpy(basis, ix.basis, sizeof(float) * (size_t)G * r * d, hipMemcpyDefault));
    if (offsets) HIP_TRY(hipMemcpy(offsets, ix.offsets_h.data(), sizeof(int64_t) * (G + 1), hipMemcpyDefault));
    if (perm) HIP_TRY(hipMemcpy(perm, ix.perm, sizeof(int32_t) * ix.N, hipMemcpyDefault));
    if (scales) HIP_TRY(hipMemcpy(scales, ix.scales, sizeof(float) * G, hipMemcpyDefault));
    if (codes || eps) {
      auto blk = to_host(ix.codes, (size_t)ix.nblocks * rp * B);
      auto eb = to_host(ix.eps, (size_t)ix.nblocks * B);
      std::vector<float> cz(codes ? (size_t)ix.N * r : 0), ce(eps ? ix.N : 0);
      for (uint32_t g = 0; g < G; ++g) {
        const int64_t a = ix.offsets_h[g], n = ix.offsets_h[g + 1] - a;
        for (int64_t i = 0; i < n; ++i) {
          const int64_t blkid = ix.boff_h[g] + i / B, lane = i % B;
          if (codes)
            for (uint32_t j = 0; j < r; ++j) cz[(size_t)(a + i) * r + j] = blk[((size_t)blkid * rp + j) * B + lane];
          if (eps) ce[a + i] = eb[(size_t)blkid * B + lane];
        }
      }
      if (codes) HIP_TRY(hipMemcpy(codes, cz.data(), sizeof(float) * cz.size(), hipMemcpyDefault));
      if (eps) HIP_TRY(hipMemcpy(eps, ce.data(), sizeof(float) * ce.size(), hipMemcpyDefault));
    }
  });
}

hntl_status hntl_index_export_codes(const hntl_index* index, uint32_t codes, void* out, float* scales) {
  g_last_error.clear();
  if (!index) return fail(HNTL_EINVAL, "index is NULL");
  const Index& ix = index->ix;
  const bool resid = (codes & HNTL_EXPORT_RESIDUALS) != 0;
  codes &= ~HNTL_EXPORT_RESIDUALS;
  if (codes != HNTL_CODES_BF16 && codes != HNTL_CODES_FP8_E4M3 && codes != HNTL_CODES_INT16)
    return fail(HNTL_EINVAL, "codes must be BF16, FP8 or INT16");
  if (resid && codes != HNTL_CODES_INT16) return fail(HNTL_EINVAL, "residual codes exist for INT16 only");
  if (!(ix.codes_mask & (1u << codes))) return fail(HNTL_ESTATE, "codes form not built for this index");
  if (resid)
    return guarded([&] {
      // r_hat_i from the stored decoded residual fl32(r_hat_i * fl32(1 / rinv_g)):
      // its relative error is below 2^-23, so r_hat_i <= 65535 is the nearest integer
      // of decoded * rinv_g
      const uint32_t G = ix.G;
      auto st = to_host(ix.i16_steps, (size_t)G * 4);
      auto dec = to_host(ix.eps_i16, (size_t)ix.nblocks * B);
      if (scales) {
        std::vector<float> rinv(G);
        for (uint32_t g = 0; g < G; ++g) rinv[g] = st[(size_t)g * 4 + 1];
        HIP_TRY(hipMemcpy(scales, rinv.data(), sizeof(float) * G, hipMemcpyDefault));
      }
      if (!out) return;
      std::vector<uint16_t> o(ix.N);
      for (uint32_t g = 0; g < G; ++g) {
        const int64_t a = ix.offsets_h[g], n = ix.offsets_h[g + 1] - a;
        for (int64_t i = 0; i < n; ++i) {
          const double v = (double)dec[((size_t)ix.boff_h[g] + i / B) * B + i % B] * (double)st[(size_t)g * 4 + 1];
          o[a + i] = (uint16_t)std::llround(v);
        }
      }
      HIP_TRY(hipMemcpy(out, o.data(), o.size() * sizeof(uint16_t), hipMemcpyDefault));
    });
  return guarded([&] {
    const uint32_t G = ix.G, r = ix.r, rp = ix.rp;
    if (scales && codes == HNTL_CODES_FP8_E4M3)
      HIP_TRY(hipMemcpy(scales, ix.scales, sizeof(float) * G, hipMemcpyDefault));
    if (scales && codes == HNTL_CODES_INT16) {  // inv_g
      auto st = to_host(ix.i16_steps, (size_t)G * 4);
      std::vector<float> inv(G);
      for (uint32_t g = 0; g < G; ++g) inv[g] = st[(size_t)g * 4];
      HIP_TRY(hipMemcpy(scales, inv.data(), sizeof(float) * G, hipMemcpyDefault));
    }
    if (!out) return;
    const int per = codes == HNTL_CODES_FP8_E4M3 ? 4 : 2;  // values per 32-bit word
    auto words = to_host(codes == HNTL_CODES_BF16 ? ix.codes_bf16 : codes == HNTL_CODES_INT16 ? ix.codes_i16 : ix.codes_fp8,
                         (size_t)ix.nblocks * (rp / per) * B);
    const size_t esz = per == 2 ? 2 : 1;
    std::vector<uint8_t> o((size_t)ix.N * r * esz);
    for (uint32_t g = 0; g < G; ++g) {
      const int64_t a = ix.offsets_h[g], n = ix.offsets_h[g + 1] - a;
      for (int64_t i = 0; i < n; ++i) {
        const int64_t blkid = ix.boff_h[g] + i / B, lane = i % B;
        for (uint32_t j = 0; j < r; ++j) {
          const uint32_t w = words[((size_t)blkid * (rp / per) + j / per) * B + lane];
          const uint32_t v = (w >> ((j % per) * (32 / per))) & (per == 2 ? 0xFFFFu : 0xFFu);
          const size_t at = ((size_t)(a + i) * r + j) * esz;
          o[at] = (uint8_t)v;
          if (esz == 2) o[at + 1] = (uint8_t)(v >> 8);
        }
      }
    }
    HIP_TRY(hipMemcpy(out, o.data(), o.size(), hipMemcpyDefault));
  });
}

hntl_status hntl_index_info_get(const hntl_index* index, hntl_index_info* out) {
  g_last_error.clear();
  if (!index || !out) return fail(HNTL_EINVAL, "null pointer");
  const Index& ix = index->ix;
  std::memset(out, 0, sizeof(*out));
  out->N = ix.N;
  out->d = ix.d;
  out->G = ix.G;
  out->r = ix.r;
  out->block = B;
  out->codes_mask = ix.codes_mask;
  out->n_blocks = ix.nblocks;
  out->device_bytes = ix.device_bytes;
  double s = 0;
  int n = 0;
  for (uint32_t g = 0; g < ix.G; ++g)
    if (ix.captured.size() == ix.G && ix.captured[g] >= 0 && ix.offsets_h[g + 1] > ix.offsets_h[g]) {
      s += ix.captured[g];
      ++n;
    }
  out->captured_variance = n ? s / n : -1.0;
  out->kmeans_iters_run = ix.kmeans_iters_run;
  out->max_grain = ix.max_grain;
  return HNTL_OK;
}

hntl_status hntl_index_captured(const hntl_index* index, double* out) {
  g_last_error.clear();
  if (!index || !out) return fail(HNTL_EINVAL, "null pointer");
  const Index& ix = index->ix;
  if (ix.captured.size() != ix.G) return fail(HNTL_ESTATE, "no captured-variance record");
  std::memcpy(out, ix.captured.data(), sizeof(double) * ix.G);
  return HNTL_OK;
}

hntl_status hntl_search_stages(const hntl_index* index, const float* Q, uint32_t nq, const hntl_search_params* sp,
                               const int32_t* probes_in, int32_t* probes_out, float* pdist_out,
                               const float* tangent_in, const float* epsq_in, float* tangent_out, float* epsq_out,
                               const int32_t* pool_in, int32_t* pool_out, float* pool_D_out, int32_t* ids,
                               float* dist, void* stream) {
  g_last_error.clear();
  const StagedIO io{probes_in, probes_out, pdist_out, tangent_in, epsq_in, tangent_out, epsq_out,
                    pool_in,   pool_out,   pool_D_out, ids,       dist};
  const hntl_status st = check_search(index, Q, nq, sp, io);
  if (st != HNTL_OK || nq == 0) return st;
  const Index& ix = index->ix;
  hipStream_t s = (hipStream_t)stream;
  return guarded([&] {
    HIP_TRY(hipSetDevice(ix.device));
    ensure_pool(ix.device);
    derive_search_data(const_cast<Index&>(ix), *sp, io, s);  // derived index data, made once under a lock
    Scratch sc(s);
    StagedScratch w;
    char* base = sc.get<char>(w.layout(nullptr, ix, Q, nq, *sp, io));
    w.layout(base, ix, Q, nq, *sp, io);
    run_staged(ix, Q, nq, *sp, io, w, s);
  });
}

hntl_status hntl_search_noalloc(const hntl_index* index, const float* Q, uint32_t nq,
                                const hntl_search_params* sp, int32_t* ids, float* dist, void* stream) {
  g_last_error.clear();
  const StagedIO io{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                    nullptr, nullptr, nullptr, ids,     dist};
  const hntl_status st = check_search(index, Q, nq, sp, io);
  if (st != HNTL_OK || nq == 0) return st;
  if (sp->flags & HNTL_FLAG_PROFILE)
    return fail(HNTL_EINVAL, "hntl_search_noalloc records no stage events (HNTL_FLAG_PROFILE)");
  const Index& ix = index->ix;
  if (!search_data_ready(ix, *sp, io))
    return fail(HNTL_ESTATE, "derived index data missing (split centroids of a BF16 routing form, or eps by id of "
                             "Mode A): run one hntl_search with the same flags first");
  StagedScratch w;
  const size_t need = w.layout(nullptr, ix, Q, nq, *sp, io);
  if (need > (size_t)HNTL_NOALLOC_SCRATCH_BYTES)
    return fail(HNTL_EINVAL, "hntl_search_noalloc needs " + std::to_string(need) + " bytes of scratch for this call, "
                             "more than HNTL_NOALLOC_SCRATCH_BYTES (" + std::to_string(HNTL_NOALLOC_SCRATCH_BYTES) +
                             "): use a smaller batch or hntl_search");
  hipStream_t s = (hipStream_t)stream;
  return guarded([&] {
    HIP_TRY(hipSetDevice(ix.device));
    char* base = noalloc_scratch(ix.device);
    w.layout(base, ix, Q, nq, *sp, io);
    run_staged(ix, Q, nq, *sp, io, w, s);
  });
}

hntl_status hntl_profile_read(double* ms, uint32_t n, uint32_t* calls, uint64_t* scored) {
  g_last_error.clear();
  return guarded([&] {
    if (scored) *scored = 0;
    if (g_prof.scored) {
      unsigned long long v = 0;
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipMemcpy(&v, g_prof.scored, sizeof(v), hipMemcpyDeviceToHost));
      HIP_TRY(hipMemset(g_prof.scored, 0, sizeof(v)));
      if (scored) *scored = v;
    }
    std::vector<double> acc(HNTL_NUM_STAGES, 0.0);
    for (auto& r : g_prof.recs) {
      HIP_TRY(hipEventSynchronize(r.ev[HNTL_NUM_STAGES]));
      for (int i = 0; i < HNTL_NUM_STAGES; ++i) {
        if (!r.used[i]) continue;
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, r.ev[i], r.ev[i + 1]));
        acc[i] += t;
      }
    }
    if (calls) *calls = (uint32_t)g_prof.recs.size();
    for (auto& r : g_prof.recs)
      for (auto e : r.ev) g_prof.pool.push_back(e);
    g_prof.recs.clear();
    if (ms)
      for (uint32_t i = 0; i < n; ++i) ms[i] = i < (uint32_t)HNTL_NUM_STAGES ? acc[i] : 0.0;
  });
}

hntl_status hntl_search(const hntl_index* index, const float* Q, uint32_t nq, const hntl_search_params* sp,
                        int32_t* ids, float* dist, void* stream) {
  return hntl_search_stages(index, Q, nq, sp, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                            nullptr, nullptr, nullptr, ids, dist, stream);
}

}  // extern "C"
