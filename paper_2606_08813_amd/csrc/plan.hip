// Batching form: search plans around the persistent fused kernel, HIP graph
// capture and replay, and the schedule autotuner with its tuning file.
//
// A plan owns one device allocation (the arena) cut into every buffer the
// search needs for batches of up to max_nq queries, so a run allocates
// nothing and its launch sequence can be captured once into a HIP graph:
//
//   reset (fill kernels: ticket, per-grain projection counters, per-query
//          bounds; graphs hold kernel nodes only)
//   routing          row norms, centroid distances (own MFMA GEMMs with a
//                    distance epilogue), top-P + exact re-score
//   bucketing        pairs grouped by grain, items numbered largest grain first
//   pair lists       per-pair list slots when grains are split into ranges
//   fused kernel     projection + scan + per-list top-C (persistent)
//   merge + rerank   pool = exact top C over the query's lists, FP32 rerank
//
// The batch size lives in device memory (written by a one-thread kernel
// before each run) and every kernel, the routing GEMMs included, skips rows
// past it, so one captured graph serves every batch size up to max_nq.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {

bool launch_fused_ct0(const FusedArgs*, int, int, int, int, int, hipStream_t);
bool launch_fused_ct1(const FusedArgs*, int, int, int, int, int, hipStream_t);
bool launch_fused_ct2(const FusedArgs*, int, int, int, int, int, hipStream_t);
bool launch_fused_ct3(const FusedArgs*, int, int, int, int, int, hipStream_t);
int fused_resident_ct0(int, int, int, int);
int fused_resident_ct1(int, int, int, int);
int fused_resident_ct2(int, int, int, int);
int fused_resident_ct3(int, int, int, int);

namespace {

__global__ void set_count_kernel(int32_t* __restrict__ p, int32_t v) {
  if (threadIdx.x == 0) *p = v;
}

bool fused_launch(int codes, const FusedArgs* a, int rp, int C, int qt, int nw, int grid, hipStream_t s) {
  switch (codes) {
    case HNTL_CODES_FP32: return launch_fused_ct0(a, rp, C, qt, nw, grid, s);
    case HNTL_CODES_BF16: return launch_fused_ct1(a, rp, C, qt, nw, grid, s);
    case HNTL_CODES_FP8_E4M3: return launch_fused_ct2(a, rp, C, qt, nw, grid, s);
    default: return launch_fused_ct3(a, rp, C, qt, nw, grid, s);
  }
}

int fused_resident(int codes, int rp, int C, int qt, int nw) {
  switch (codes) {
    case HNTL_CODES_FP32: return fused_resident_ct0(rp, C, qt, nw);
    case HNTL_CODES_BF16: return fused_resident_ct1(rp, C, qt, nw);
    case HNTL_CODES_FP8_E4M3: return fused_resident_ct2(rp, C, qt, nw);
    default: return fused_resident_ct3(rp, C, qt, nw);
  }
}

// Bytes of per-wave LDS of the fused kernel (lists + staged tangents).
size_t lds_per_wave(int rp, int C, int qt) {
  (void)C;
  const size_t lk = 64;  // the arrival stage of a register-resident list
  return (size_t)qt * lk * 8 + (((size_t)qt * rp + qt) * 4 + 7) / 8 * 8;
}

constexpr size_t LDS_LIMIT = 64 * 1024;
// one projection counter and 8 scan counters per launch, 256 bytes apart
constexpr int TICKET_INTS = 9 * 64;
constexpr int MIN_GRID = 8;  // every class of scan counters needs a workgroup
// search flags a plan honours (beyond HNTL_FLAG_SYNC)
constexpr int PLAN_STAGES = 5;  // route, bucket, projection launch, fused kernel, merge + rerank
constexpr uint32_t PLAN_FLAGS =
    HNTL_FLAG_PROJECT_BF16 | HNTL_FLAG_NO_PRUNE | HNTL_FLAG_ROUTE_BF16X3 | HNTL_FLAG_ROUTE_BF16 | HNTL_FLAG_MODE_A;
constexpr uint64_t MAX_LIST_BYTES = 4ull << 30;  // candidate-list storage of one plan

// Bump allocation over one block (base == nullptr: sizing pass).
struct Layout {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) / 256 * 256;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

// Grains by size, largest first (ties: lower grain id first); kept on the index.
std::mutex g_order_mu;
void ensure_grain_order(Index& ix) {
  std::lock_guard<std::mutex> lk(g_order_mu);
  if (ix.gorder) return;
  std::vector<int32_t> o(ix.G);
  for (uint32_t g = 0; g < ix.G; ++g) o[g] = (int32_t)g;
  std::stable_sort(o.begin(), o.end(), [&](int32_t a, int32_t b) {
    return ix.offsets_h[a + 1] - ix.offsets_h[a] > ix.offsets_h[b + 1] - ix.offsets_h[b];
  });
  int32_t* d = dev_alloc<int32_t>(&ix, ix.G);
  HIP_TRY(hipMemcpy(d, o.data(), sizeof(int32_t) * ix.G, hipMemcpyHostToDevice));
  ix.gorder = d;
}

std::string device_key(int dev) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string arch = p.gcnArchName;
  const size_t c = arch.find(':');
  if (c != std::string::npos) arch = arch.substr(0, c);
  return arch + "-cu" + std::to_string(p.multiProcessorCount);
}

std::string tune_key(const Index& ix, const hntl_search_params& sp, uint32_t nq) {
  std::ostringstream k;
  k << device_key(ix.device) << " N=" << ix.N << " d=" << ix.d << " G=" << ix.G << " r=" << ix.r
    << " maxgrain=" << ix.max_grain << " P=" << sp.P << " C=" << sp.C << " k=" << sp.k << " codes=" << sp.codes
    << " flags=" << (sp.flags & PLAN_FLAGS) << " route=" << sp.route << " mass=" << sp.mass
    << " nq=" << nq;
  return k.str();
}

}  // namespace

// ------------------------------------------------------------------ plan
struct Plan {
  Index* ix = nullptr;
  hntl_search_params sp{};
  uint32_t max_nq = 0;
  hntl_schedule sch{};
  uint32_t flags = 0;
  int device = 0;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  // batch I/O
  float* Q = nullptr;
  int32_t* ids = nullptr;
  float* dist = nullptr;
  int32_t* nq_dev = nullptr;
  // routing
  int32_t* probes = nullptr;
  RouteScratch route;
  // bucketing
  Buckets b{};
  int32_t* nsplit = nullptr;
  int32_t* lbase = nullptr;
  int32_t* qoff = nullptr;
  // fused kernel state
  FusedArgs* args_dev = nullptr;
  int32_t* ticket = nullptr;
  int32_t* proj_done = nullptr;  // one flag per projection item
  int64_t proj_items = 0;
  ItemDesc* items = nullptr;  // decoded work items of the fused kernel
  int64_t max_items = 0;
  uint32_t* qbound = nullptr;
  int32_t* err = nullptr;
  float* T = nullptr;
  float* epsq = nullptr;
  uint64_t* part = nullptr;
  uint64_t list_slots = 0;
  unsigned long long* scored = nullptr;  // eq. 6 scores of the last run
  // learned routing
  RouterScratch rs;
  // graph
  hipStream_t cap_stream = nullptr;
  std::vector<hipGraph_t> graphs;
  std::vector<hipGraphExec_t> execs;
  hipStream_t last_stream = nullptr;
  uint32_t wait_errors = 0;

  ~Plan() {
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(device);
    for (auto e : execs) (void)hipGraphExecDestroy(e);
    for (auto g : graphs) (void)hipGraphDestroy(g);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (arena) (void)hipFree(arena);
    (void)hipSetDevice(prev);
  }

  // Assigns every buffer from the arena (sizing pass when base is null).
  size_t layout(char* base) {
    const Index& x = *ix;
    const int64_t np = (int64_t)max_nq * sp.P;
    Layout L;
    L.base = base;
    Q = L.take<float>((size_t)max_nq * x.d);
    ids = L.take<int32_t>((size_t)max_nq * sp.k);
    dist = L.take<float>((size_t)max_nq * sp.k);
    nq_dev = L.take<int32_t>(1);
    probes = L.take<int32_t>(np);
    if (sp.route != HNTL_ROUTE_LEARNED) {
      const int form = route_form(sp.flags);
      const size_t n = route.layout(nullptr, x, max_nq, form);
      char* rb = L.take<char>(n);
      route.layout(rb, x, max_nq, form);
    }
    b.G = (int)x.G;
    b.gcount = L.take<int32_t>(x.G);
    b.gcount0 = L.take<int32_t>(x.G);
    b.gstart = L.take<int32_t>(x.G);
    b.cur0 = L.take<int32_t>(x.G);
    b.cur1 = L.take<int32_t>(x.G);
    b.order = L.take<int32_t>(np);
    for (int l = 0; l < 3; ++l) {
      b.lists.ioff[l] = L.take<int32_t>(x.G + 1);
      b.lists.lstart[l] = L.take<int32_t>(x.G);
      b.lists.lcount[l] = L.take<int32_t>(x.G);
    }
    b.lists.tile[LIST_SLOT0] = b.lists.tile[LIST_REST] = (int)sch.qt;  // scan item: qt pairs (one wave)
    // projection item: 16 pairs, one wave, inside the fused kernel; with a
    // separate projection launch, the shared-basis kernel's item where it applies
    b.lists.tile[LIST_ALL] = sch.proj ? project_tile(x, Q, (sp.flags & HNTL_FLAG_PROJECT_BF16) != 0) : 16;
    b.max_items[LIST_ALL] = (int)(np / b.lists.tile[LIST_ALL] + std::min<int64_t>(x.G, np) + 1);
    nsplit = L.take<int32_t>(x.G);
    lbase = L.take<int32_t>(np);
    qoff = L.take<int32_t>((size_t)max_nq + 1);
    args_dev = L.take<FusedArgs>(3);  // phases 0, 1, 2
    ticket = L.take<int32_t>(2 * TICKET_INTS);  // counters of each launch (phases 0/1 and 2)
    proj_items = (int64_t)((np + 15) / 16) + x.G;  // at most sum over grains of ceil(pairs / 16)
    proj_done = L.take<int32_t>(proj_items);
    max_items = proj_items + (int64_t)list_slots;  // projection items + at most one scan item per list
    items = L.take<ItemDesc>((size_t)max_items);
    qbound = L.take<uint32_t>(max_nq);
    err = L.take<int32_t>(1);
    T = L.take<float>((size_t)np * x.r);
    epsq = L.take<float>(np);
    part = L.take<uint64_t>((size_t)list_slots * sp.C);
    scored = L.take<unsigned long long>(1);
    if (sp.route == HNTL_ROUTE_LEARNED) {
      const size_t n = rs.layout(nullptr, x, max_nq, (int)sp.P);
      char* rb = L.take<char>(n);
      rs.layout(rb, x, max_nq, (int)sp.P);
    }
    return L.off;
  }

  const void* codes_ptr() const {
    switch (sp.codes) {
      case HNTL_CODES_FP32: return ix->codes;
      case HNTL_CODES_BF16: return ix->codes_bf16;
      case HNTL_CODES_FP8_E4M3: return ix->codes_fp8;
      default: return ix->codes_i16;
    }
  }

  FusedArgs make_args() const {
    const Index& x = *ix;
    FusedArgs a{};
    a.codes = codes_ptr();
    // int16 form: the per-grain steps in place of the FP8 scales, the decoded
    // residuals r_hat_i / rinv_g in place of eps_i
    a.scales = sp.codes == HNTL_CODES_INT16 ? x.i16_steps : x.scales;
    a.eps = sp.codes == HNTL_CODES_INT16 ? x.eps_i16 : x.eps;
    a.goff = x.goff;
    a.boff = x.boff;
    a.perm = x.perm;
    a.blo = x.blo;
    a.bhi = x.bhi;
    a.emin = x.emin;
    a.centroids = x.centroids;
    a.basis = x.basis;
    a.basis16 = x.basis_bf16;
    a.d = (int)x.d;
    a.r = (int)x.r;
    a.G = (int)x.G;
    a.P = (int)sp.P;
    a.C = (int)sp.C;
    a.Q = Q;
    for (int l = 0; l < 3; ++l) {
      a.ioff[l] = b.lists.ioff[l];
      a.lstart[l] = b.lists.lstart[l];
      a.lcount[l] = b.lists.lcount[l];
    }
    a.gorder = x.gorder;
    a.order = b.order;
    a.lbase = sch.range ? lbase : nullptr;
    a.R = (int)sch.range;
    a.ticket = ticket;
    a.proj_done = proj_done;
    a.qbound = qbound;
    a.err = err;
    a.T = T;
    a.epsq = epsq;
    a.part = part;
    a.scored = scored;
    a.proj_bf16 = (sp.flags & HNTL_FLAG_PROJECT_BF16) ? 1 : 0;
    a.proj_ext = sch.proj ? 1 : 0;
    a.items = items;
    a.prune = (sp.flags & HNTL_FLAG_NO_PRUNE) ? 0 : 1;
    return a;
  }

  // The launch sequence of one run (batch size already in nq_dev).  With
  // `ev` (6 events) the stage boundaries are recorded: route, bucketing,
  // separate projection launch (empty with proj = 0), fused kernel, merge +
  // rerank.
  void enqueue(hipStream_t s, hipEvent_t* ev = nullptr) {
    const Index& x = *ix;
    const int P = (int)sp.P, G = (int)x.G;
    if (ev) HIP_TRY(hipEventRecord(ev[0], s));
    FillList f{};
    f.seg[0] = FillSeg{ticket, 2 * TICKET_INTS, 0};
    f.seg[1] = FillSeg{reinterpret_cast<int32_t*>(scored), 2, 0};
    f.seg[2] = FillSeg{proj_done, proj_items, 0};
    f.seg[3] = FillSeg{reinterpret_cast<int32_t*>(qbound), (int64_t)max_nq, -1};
    f.seg[4] = FillSeg{b.gcount, G, 0};
    f.seg[5] = FillSeg{b.gcount0, G, 0};
    f.n = 6;
    launch_fill_multi(f, s);
    // routing reads the batch size from nq_dev: rows past it get probes -1
    if (sp.route == HNTL_ROUTE_LEARNED)
      launch_route_learned(x, Q, max_nq, P, sp.tau, probes, nullptr, rs, s, nq_dev, sp.mass);
    else
      launch_route_centroid(x, Q, max_nq, P, route, probes, nullptr, s, nq_dev);
    if (ev) HIP_TRY(hipEventRecord(ev[1], s));
    launch_bucket(probes, max_nq, P, G, b, s, x.gorder, nsplit, true);
    if (sch.range) launch_pair_lists(probes, max_nq, P, G, nsplit, lbase, qoff, s);
    launch_item_table(b.lists, x.gorder, G, (int)sch.qt, max_items, items, s);
    if (ev) HIP_TRY(hipEventRecord(ev[2], s));
    if (sch.proj) launch_project(x, Q, P, b, T, epsq, (sp.flags & HNTL_FLAG_PROJECT_BF16) != 0, x.gorder, s);
    if (ev) HIP_TRY(hipEventRecord(ev[3], s));
    for (int ph = sch.passes == 2 ? 1 : 0; ph <= (sch.passes == 2 ? 2 : 0); ++ph) {
      if (!fused_launch((int)sp.codes, args_dev + ph, (int)x.rp, (int)sp.C, (int)sch.qt, (int)sch.nw, (int)sch.grid,
                        s))
        throw ArgError{HNTL_EUNSUPPORTED, "no fused kernel for this rank / pool / schedule"};
      HIP_TRY(hipGetLastError());
    }
    if (ev) HIP_TRY(hipEventRecord(ev[4], s));
    launch_merge_rerank(x, Q, max_nq, P, (int)sp.C, (int)sp.k, probes, part, nullptr, nullptr, nullptr, ids, dist, s,
                        sch.range ? qoff : nullptr, (sp.flags & HNTL_FLAG_MODE_A) ? x.eps_id : nullptr, nq_dev);
    if (ev) HIP_TRY(hipEventRecord(ev[5], s));
  }

  void run(uint32_t nq, hipStream_t s) {
    hipLaunchKernelGGL(set_count_kernel, dim3(1), dim3(64), 0, s, nq_dev, (int32_t)nq);
    HIP_TRY(hipGetLastError());
    if (!execs.empty())
      HIP_TRY(hipGraphLaunch(execs[0], s));
    else
      enqueue(s);
    last_stream = s;
  }
};

namespace {

void check_plan_shape(const Index& ix, const hntl_search_params& sp) {
  if (sp.P < 1 || sp.P > ix.G) throw ArgError{HNTL_EINVAL, "need 1 <= P <= G"};
  if (sp.P > HNTL_MAX_P) throw ArgError{HNTL_EUNSUPPORTED, "P exceeds HNTL_MAX_P"};
  if (sp.k < 1 || sp.C < sp.k) throw ArgError{HNTL_EINVAL, "need 1 <= k <= C"};
  if (sp.C > HNTL_MAX_C) throw ArgError{HNTL_EUNSUPPORTED, "C exceeds HNTL_MAX_C"};
  if (sp.codes > HNTL_CODES_INT16) throw ArgError{HNTL_EINVAL, "unknown codes form"};
  if (sp.codes == HNTL_CODES_INT16 && (sp.flags & HNTL_FLAG_MODE_A))
    throw ArgError{HNTL_EUNSUPPORTED, "Mode A answers use the FP32 / BF16 / FP8 code forms"};
  if (!(ix.codes_mask & (1u << sp.codes))) throw ArgError{HNTL_ESTATE, "codes form not built for this index"};
  if ((sp.flags & HNTL_FLAG_PROJECT_BF16) && !ix.basis_bf16)
    throw ArgError{HNTL_ESTATE, "BF16 projection needs the BF16 basis (build a reduced-precision code form)"};
  if (sp.route > HNTL_ROUTE_LEARNED) throw ArgError{HNTL_EINVAL, "unknown route"};
  if (!(sp.mass >= 0.f && sp.mass <= 1.f)) throw ArgError{HNTL_EINVAL, "mass must lie in [0, 1]"};
  if (sp.route == HNTL_ROUTE_LEARNED && !(ix.router && ix.router->trained))
    throw ArgError{HNTL_ESTATE, "learned routing needs a trained router"};
  if (ix.d % 8 != 0) throw ArgError{HNTL_EUNSUPPORTED, "the fused kernel needs d % 8 == 0"};
  if (!(sp.flags & HNTL_FLAG_MODE_A) && !ix.X)
    throw ArgError{HNTL_ESTATE, "this index holds no raw vectors: only Mode A searches"};
  if (ix.rp != 16 && ix.rp != 32 && ix.rp != 48 && ix.rp != 64)
    throw ArgError{HNTL_EUNSUPPORTED, "the fused kernel needs a padded rank of 16, 32, 48 or 64"};
}

// Default schedule from the batch shape: few pairs per grain want short
// items spread over many workgroups; many pairs per grain want wide tiles.
hntl_schedule default_schedule(const Index& ix, const hntl_search_params& sp, uint32_t max_nq) {
  const double per_grain = (double)max_nq * sp.P / std::max<uint32_t>(1, ix.G);
  hntl_schedule s{};
  if (per_grain < 1.0) {
    s.qt = 1;
    s.nw = 1;
    s.range = 8;
  } else if (per_grain < 8.0) {
    s.qt = 1;
    s.nw = 4;
    s.range = 16;
  } else {
    s.qt = 4;
    s.nw = 4;
    s.range = 32;
  }
  while (s.nw > 1 && lds_per_wave((int)ix.rp, (int)sp.C, (int)s.qt) * s.nw > LDS_LIMIT) s.nw /= 2;
  s.grid = 0;
  s.passes = per_grain >= 8.0 ? 2 : 1;  // many pairs per grain: bound the other slots by slot 0 first
  return s;
}

Plan* make_plan(Index& ix, const hntl_search_params& sp, uint32_t max_nq, const hntl_schedule& sch_in,
                uint32_t plan_flags, hipStream_t s) {
  check_plan_shape(ix, sp);
  hntl_schedule sch = sch_in;
  if (!(sch.qt == 1 || sch.qt == 2 || sch.qt == 4 || sch.qt == 8))
    throw ArgError{HNTL_EINVAL, "schedule qt must be 1, 2, 4 or 8"};
  if (sch.nw < 1 || sch.nw > 8) throw ArgError{HNTL_EINVAL, "schedule nw must be 1..8"};
  if (sch.passes == 0) sch.passes = 1;
  if (sch.passes > 2) throw ArgError{HNTL_EINVAL, "schedule passes must be 1 or 2"};
  if (sch.proj > 1) throw ArgError{HNTL_EINVAL, "schedule proj must be 0 or 1"};
  if (lds_per_wave((int)ix.rp, (int)sp.C, (int)sch.qt) * sch.nw > LDS_LIMIT)
    throw ArgError{HNTL_EUNSUPPORTED, "schedule needs more than 64 KiB of LDS per workgroup"};
  ensure_grain_order(ix);
  if (route_form(sp.flags) != ROUTE_F32 && sp.route != HNTL_ROUTE_LEARNED) ensure_centroid_split(ix, s);
  if (sp.flags & HNTL_FLAG_MODE_A) ensure_eps_by_id(ix, s);
  std::unique_ptr<Plan> pl(new Plan());
  pl->ix = &ix;
  pl->sp = sp;
  pl->max_nq = max_nq;
  pl->flags = plan_flags;
  pl->device = ix.device;
  // list slots: per query at most the sum of its P largest split counts
  std::vector<int32_t> ns(ix.G);
  for (uint32_t g = 0; g < ix.G; ++g) {
    const int nb = ix.boff_h[g + 1] - ix.boff_h[g];
    ns[g] = sch.range ? std::max(1, (int)((nb + (int)sch.range - 1) / (int)sch.range)) : 1;
  }
  std::vector<int32_t> srt(ns);
  std::sort(srt.begin(), srt.end(), std::greater<int32_t>());
  uint64_t per_q = 0;
  for (uint32_t i = 0; i < sp.P; ++i) per_q += (uint64_t)srt[i];
  pl->list_slots = (uint64_t)max_nq * per_q;
  if (pl->list_slots >= (1ull << 31) || pl->list_slots * sp.C * sizeof(uint64_t) > MAX_LIST_BYTES)
    throw ArgError{HNTL_EUNSUPPORTED, "too many candidate lists for this schedule and batch size"};
  const uint64_t res = (uint64_t)fused_resident((int)sp.codes, (int)ix.rp, (int)sp.C, (int)sch.qt, (int)sch.nw);
  if (res == 0) throw ArgError{HNTL_EUNSUPPORTED, "no fused kernel for this rank / pool / schedule"};
  if (sch.grid == 0) {
    // as many workgroups as are resident at once, but no more waves than the
    // largest possible number of work items:
    // projection items + at most one scan item per (pair, block range)
    const uint64_t np = (uint64_t)max_nq * sp.P, gp = std::min<uint64_t>(ix.G, np);
    const uint64_t items = (np + 15) / 16 + gp + pl->list_slots;
    sch.grid = (uint32_t)std::min<uint64_t>(res, (items + sch.nw - 1) / sch.nw);
  }
  sch.grid = std::max<uint32_t>(sch.grid, MIN_GRID);
  pl->sch = sch;
  pl->arena_bytes = pl->layout(nullptr);
  HIP_TRY(hipMalloc((void**)&pl->arena, pl->arena_bytes));
  pl->layout(pl->arena);
  HIP_TRY(hipMemsetAsync(pl->Q, 0, sizeof(float) * (size_t)max_nq * ix.d, s));
  HIP_TRY(hipMemsetAsync(pl->err, 0, sizeof(int32_t), s));
  HIP_TRY(hipMemcpyAsync(pl->nsplit, ns.data(), sizeof(int32_t) * ix.G, hipMemcpyHostToDevice, s));
  FusedArgs a[3];
  for (int ph = 0; ph < 3; ++ph) {
    a[ph] = pl->make_args();
    a[ph].phase = ph;
    a[ph].ticket = pl->ticket + (ph == 2 ? TICKET_INTS : 0);
  }
  HIP_TRY(hipMemcpyAsync(pl->args_dev, a, sizeof(a), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (plan_flags & HNTL_PLAN_GRAPH) {
    // one graph serves every batch size up to max_nq (the size is read from
    // device memory by every kernel that depends on it)
    HIP_TRY(hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal));
    try {
      pl->enqueue(pl->cap_stream);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(pl->cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamEndCapture(pl->cap_stream, &g));
    pl->graphs.push_back(g);
    hipGraphExec_t e = nullptr;
    HIP_TRY(hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
    pl->execs.push_back(e);
  }
  return pl.release();
}

uint32_t read_wait_errors(Plan& pl) {
  int32_t e = 0;
  HIP_TRY(hipMemcpy(&e, pl.err, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (e) {
    pl.wait_errors += 1;
    HIP_TRY(hipMemset(pl.err, 0, sizeof(int32_t)));
  }
  return pl.wait_errors;
}

template <class F>
hntl_status guarded_call(F&& f) {
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

}  // namespace
}  // namespace hntl

struct hntl_plan {
  hntl::Plan* p;
};

using namespace hntl;

extern "C" {

hntl_status hntl_plan_create(hntl_index* index, const hntl_search_params* sp, uint32_t max_nq,
                             const hntl_schedule* sched, uint32_t plan_flags, void* stream, hntl_plan** out) {
  set_error("");
  if (!out) return fail(HNTL_EINVAL, "out is NULL");
  *out = nullptr;
  if (!index || !sp) return fail(HNTL_EINVAL, "null index or params");
  if (max_nq == 0) return fail(HNTL_EINVAL, "max_nq must be positive");
  return guarded_call([&] {
    Index& ix = index->ix;
    HIP_TRY(hipSetDevice(ix.device));
    const hntl_schedule sch = sched ? *sched : default_schedule(ix, *sp, max_nq);
    Plan* p = make_plan(ix, *sp, max_nq, sch, plan_flags, (hipStream_t)stream);
    *out = new hntl_plan{p};
  });
}

hntl_status hntl_plan_buffers(hntl_plan* plan, float** Q, int32_t** ids, float** dist) {
  set_error("");
  if (!plan) return fail(HNTL_EINVAL, "null plan");
  if (Q) *Q = plan->p->Q;
  if (ids) *ids = plan->p->ids;
  if (dist) *dist = plan->p->dist;
  return HNTL_OK;
}

hntl_status hntl_plan_run(hntl_plan* plan, uint32_t nq, void* stream) {
  set_error("");
  if (!plan) return fail(HNTL_EINVAL, "null plan");
  Plan& pl = *plan->p;
  if (nq > pl.max_nq) return fail(HNTL_EINVAL, "nq exceeds the plan's max_nq");
  return guarded_call([&] {
    HIP_TRY(hipSetDevice(pl.device));
    hipStream_t s = (hipStream_t)stream;
    pl.run(nq, s);
    if (pl.sp.flags & HNTL_FLAG_SYNC) {
      HIP_TRY(hipStreamSynchronize(s));
      HIP_TRY(hipGetLastError());
      const uint32_t before = pl.wait_errors;
      if (read_wait_errors(pl) != before) throw ArgError{HNTL_EDEVICE, "a fused-kernel wait gave up"};
    }
  });
}

hntl_status hntl_plan_search(hntl_plan* plan, const float* Q, uint32_t nq, int32_t* ids, float* dist,
                             void* stream) {
  set_error("");
  if (!plan) return fail(HNTL_EINVAL, "null plan");
  Plan& pl = *plan->p;
  if (nq > pl.max_nq) return fail(HNTL_EINVAL, "nq exceeds the plan's max_nq");
  if (nq == 0) return HNTL_OK;
  if (!Q || !ids || !dist) return fail(HNTL_EINVAL, "Q, ids and dist are required");
  return guarded_call([&] {
    HIP_TRY(hipSetDevice(pl.device));
    hipStream_t s = (hipStream_t)stream;
    const Index& ix = *pl.ix;
    if (Q != pl.Q)
      HIP_TRY(hipMemcpyAsync(pl.Q, Q, sizeof(float) * (size_t)nq * ix.d, hipMemcpyDeviceToDevice, s));
    pl.run(nq, s);
    if (ids != pl.ids)
      HIP_TRY(hipMemcpyAsync(ids, pl.ids, sizeof(int32_t) * (size_t)nq * pl.sp.k, hipMemcpyDeviceToDevice, s));
    if (dist != pl.dist)
      HIP_TRY(hipMemcpyAsync(dist, pl.dist, sizeof(float) * (size_t)nq * pl.sp.k, hipMemcpyDeviceToDevice, s));
    if (pl.sp.flags & HNTL_FLAG_SYNC) {
      HIP_TRY(hipStreamSynchronize(s));
      HIP_TRY(hipGetLastError());
      const uint32_t before = pl.wait_errors;
      if (read_wait_errors(pl) != before) throw ArgError{HNTL_EDEVICE, "a fused-kernel wait gave up"};
    }
  });
}

hntl_status hntl_plan_info_get(hntl_plan* plan, hntl_plan_info* out) {
  set_error("");
  if (!plan || !out) return fail(HNTL_EINVAL, "null pointer");
  Plan& pl = *plan->p;
  return guarded_call([&] {
    HIP_TRY(hipSetDevice(pl.device));
    if (pl.last_stream) HIP_TRY(hipStreamSynchronize(pl.last_stream));
    std::memset(out, 0, sizeof(*out));
    out->max_nq = pl.max_nq;
    out->sched = pl.sch;
    out->graph = pl.execs.empty() ? 0u : 1u;
    out->device_bytes = pl.arena_bytes;
    out->list_slots = pl.list_slots;
    out->wait_errors = read_wait_errors(pl);
  });
}

hntl_status hntl_plan_profile(hntl_plan* plan, uint32_t nq, uint32_t reps, double* stage_ms, uint64_t* scored,
                              void* stream) {
  set_error("");
  if (!plan || !stage_ms) return fail(HNTL_EINVAL, "null pointer");
  Plan& pl = *plan->p;
  if (nq > pl.max_nq) return fail(HNTL_EINVAL, "nq exceeds the plan's max_nq");
  if (reps == 0) return fail(HNTL_EINVAL, "reps must be positive");
  return guarded_call([&] {
    HIP_TRY(hipSetDevice(pl.device));
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ev[PLAN_STAGES + 1];
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    std::vector<double> acc(PLAN_STAGES, 0.0);
    unsigned long long sc = 0;
    try {
      for (uint32_t rep = 0; rep < reps; ++rep) {
        hipLaunchKernelGGL(set_count_kernel, dim3(1), dim3(64), 0, s, pl.nq_dev, (int32_t)nq);
        pl.enqueue(s, ev);
        HIP_TRY(hipEventSynchronize(ev[PLAN_STAGES]));
        for (int i = 0; i < PLAN_STAGES; ++i) {
          float t = 0.f;
          HIP_TRY(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
          acc[i] += t;
        }
        HIP_TRY(hipMemcpy(&sc, pl.scored, sizeof(sc), hipMemcpyDeviceToHost));
      }
    } catch (...) {
      for (auto& e : ev) (void)hipEventDestroy(e);
      throw;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    for (int i = 0; i < PLAN_STAGES; ++i) stage_ms[i] = acc[i] / reps;
    if (scored) *scored = sc;
    pl.last_stream = s;
  });
}

void hntl_plan_free(hntl_plan* plan) {
  if (!plan) return;
  delete plan->p;
  delete plan;
}

hntl_status hntl_tune(hntl_index* index, const hntl_search_params* sp, const float* Q, uint32_t nq,
                      const char* db_path, hntl_schedule* best, float* best_ms, void* stream) {
  set_error("");
  if (!index || !sp || !Q || !best) return fail(HNTL_EINVAL, "null pointer");
  if (nq == 0) return fail(HNTL_EINVAL, "nq must be positive");
  return guarded_call([&] {
    Index& ix = index->ix;
    HIP_TRY(hipSetDevice(ix.device));
    hipStream_t s = (hipStream_t)stream;
    check_plan_shape(ix, *sp);
    hntl_search_params spp = *sp;
    spp.flags &= PLAN_FLAGS;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float bms = 0.f;
    hntl_schedule bs{};
    bool have = false;
    const uint32_t qts[] = {1, 2, 4, 8}, nws[] = {1, 2, 4, 8}, ranges[] = {0, 8, 32, 64};
    for (uint32_t proj = 0; proj <= 1; ++proj)
    for (uint32_t passes = 1; passes <= 2; ++passes)
    for (uint32_t qt : qts)
      for (uint32_t nw : nws)
        for (uint32_t R : ranges) {
          if (lds_per_wave((int)ix.rp, (int)spp.C, (int)qt) * nw > LDS_LIMIT) continue;
          hntl_schedule c{qt, nw, R, 0, passes, proj};
          std::unique_ptr<Plan> pl;
          try {
            pl.reset(make_plan(ix, spp, nq, c, 0, s));
          } catch (const ArgError&) {
            continue;  // e.g. too many list slots for this range at this batch size
          } catch (const HipError& e) {
            if (e.code == hipErrorOutOfMemory || e.code == hipErrorMemoryAllocation) {
              (void)hipGetLastError();
              continue;
            }
            throw;
          }
          HIP_TRY(hipMemcpyAsync(pl->Q, Q, sizeof(float) * (size_t)nq * ix.d, hipMemcpyDeviceToDevice, s));
          pl->run(nq, s);  // warm-up
          std::vector<float> t;
          for (int rep = 0; rep < 5; ++rep) {
            HIP_TRY(hipEventRecord(e0, s));
            pl->run(nq, s);
            HIP_TRY(hipEventRecord(e1, s));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            t.push_back(ms);
          }
          HIP_TRY(hipStreamSynchronize(s));
          if (read_wait_errors(*pl) != 0) throw ArgError{HNTL_EDEVICE, "a fused-kernel wait gave up while tuning"};
          std::sort(t.begin(), t.end());
          const float med = t[t.size() / 2];
          if (!have || med < bms) {
            have = true;
            bms = med;
            bs = pl->sch;
            bs.grid = 0;  // resolved again on the device that loads the schedule
          }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!have) throw ArgError{HNTL_EUNSUPPORTED, "no candidate schedule could run"};
    *best = bs;
    if (best_ms) *best_ms = bms;
    if (db_path) {
      const std::string key = tune_key(ix, spp, nq);
      std::vector<std::string> lines;
      {
        std::ifstream in(db_path);
        std::string line;
        while (std::getline(in, line))
          if (!line.empty() && line.rfind(key + " |", 0) != 0) lines.push_back(line);
      }
      char buf[160];
      std::snprintf(buf, sizeof buf, " | qt=%u nw=%u range=%u passes=%u proj=%u | %.4f ms", bs.qt, bs.nw,
                    bs.range, bs.passes, bs.proj, bms);
      lines.push_back(key + buf);
      std::ofstream o(db_path, std::ios::trunc);
      if (!o) throw ArgError{HNTL_EINVAL, std::string("cannot write tuning file ") + db_path};
      for (auto& l : lines) o << l << "\n";
    }
  });
}

hntl_status hntl_schedule_lookup(const hntl_index* index, const hntl_search_params* sp, uint32_t max_nq,
                                 const char* db_path, hntl_schedule* out) {
  set_error("");
  if (!index || !sp || !db_path || !out) return fail(HNTL_EINVAL, "null pointer");
  return guarded_call([&] {
    hntl_search_params spp = *sp;
    spp.flags &= PLAN_FLAGS;
    const std::string key = tune_key(index->ix, spp, max_nq);
    std::ifstream in(db_path);
    std::string line;
    while (std::getline(in, line)) {
      if (line.rfind(key + " |", 0) != 0) continue;
      hntl_schedule s{};
      const int nf = std::sscanf(line.c_str() + key.size(), " | qt=%u nw=%u range=%u passes=%u proj=%u", &s.qt,
                                 &s.nw, &s.range, &s.passes, &s.proj);
      if (nf == 4 || nf == 5) {  // lines written before the proj field count as proj = 0
        s.grid = 0;
        *out = s;
        return;
      }
    }
    throw ArgError{HNTL_ESTATE, "no tuned schedule for this key"};
  });
}

}  // extern "C"
