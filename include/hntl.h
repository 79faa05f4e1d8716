/*
 * hntl.h - C ABI of the HNTL search library for AMD Instinct MI355X (gfx950).
 *
 * HNTL ("Hierarchical No-pointer Tangent-Local" search) answers approximate
 * k-nearest-neighbour queries in four steps (paper, Section 2.1 "Query
 * Execution Lifecycle", Mode B):
 *
 *   1. centroid routing   - the P grains whose centroids are closest to the
 *                           query (Section 2.1 step 1, Section 2.3)
 *   2. projection         - q' = q - mu_g, z_q = W_g^T q', eps_q = ||q' - W_g z_q||^2
 *                           for each probed grain (Section 2.2, eq. 1-4)
 *   3. Block-SoA scan     - D_i = ||z_q - z_i||^2 + eps_q + eps_i over every member
 *                           of every probed grain (eq. 6, Section 2.4), keeping the
 *                           C smallest (D, id) per query: the candidate pool
 *   4. exact rerank       - squared L2 against the raw float32 vectors of the pool,
 *                           top-k (Section 2.1 step 4, Mode B)
 *
 * The index is built by k-means grain partitioning plus a per-grain local PCA
 * basis of rank r (Section 2.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an hntl_status and never throws; on failure a
 *   thread-local message is available from hntl_last_error().
 * - Array arguments are plain pointers.  Pointers marked "device" must point to
 *   memory on the index's GPU; pointers marked "host or device" may be either
 *   (they are read with a unified-address copy).  The caller owns every array
 *   it passes; the library owns the index and everything inside it, including
 *   its own copy of the raw vectors used for rerank.
 * - Matrices are row-major, float32 unless stated.  Ids are int32 original row
 *   indices (N < 2^31); -1 pads a list that has fewer valid entries.
 * - Distances are squared Euclidean, float32.
 * - Ties are broken by the lower id (grain id for routing).
 * - "stream" is a hipStream_t passed as void* (NULL = the default stream).
 *   Search calls are asynchronous on that stream unless HNTL_FLAG_SYNC is set;
 *   outputs are valid after the stream synchronises.  Concurrent searches on
 *   one index are allowed (per-call scratch is stream-ordered).
 */
#ifndef HNTL_H_
#define HNTL_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hntl_status {
  HNTL_OK = 0,
  HNTL_EINVAL = -1,      /* invalid argument (sizes, null pointers, non-finite input) */
  HNTL_ENOMEM = -2,      /* device or host allocation failed */
  HNTL_EDEVICE = -3,     /* no usable GPU, or a HIP runtime error */
  HNTL_ESTATE = -4,      /* the index lacks what the call needs (e.g. codes form not built) */
  HNTL_EIO = -5,         /* a file could not be written or read, or failed its checks */
  HNTL_EUNSUPPORTED = -6 /* a size outside the compiled limits (see HNTL_MAX_*) */
} hntl_status;

/* Compiled limits. */
#define HNTL_MAX_R 64       /* tangent rank r */
#define HNTL_MAX_C 256      /* candidate pool C */
#define HNTL_MAX_P 48       /* probes P */
#define HNTL_BLOCK 64       /* Block-SoA block size B (vectors per block) */

/* Code storage of the tangent coordinates scanned in step 3. */
typedef enum hntl_codes {
  HNTL_CODES_FP32 = 0,
  HNTL_CODES_BF16 = 1,      /* bf16, round-to-nearest-even of the fp32 codes */
  HNTL_CODES_FP8_E4M3 = 2,  /* OCP e4m3fn of z / s_g, per-grain fp32 scale s_g = amax / 448 */
  HNTL_CODES_INT16 = 3      /* the paper's eq. 5: int16 z_hat = rint(fl32(z) * inv_g) with inv_g = fl32(32767 / amax_g),
                               uint16 r_hat_i = rint(fl32(eps_i) * rinv_g), rinv_g = fl32(65535 / max_i eps_i);
                               score (1 / inv_g)^2 sum_j (z_hat_q,j - z_hat_i,j)^2 (exact integer sum)
                               + r_hat_i / rinv_g + eps_q; a probed grain in which more than 25% of the
                               query's coordinates saturate is pruned (envelope filter).  The integer sum
                               is exact (64-bit); exact pruning uses the grain's code box in code space.
                               Mode B only */
} hntl_codes;

/* Search flags. */
#define HNTL_FLAG_SYNC 1u       /* synchronise the stream before returning, report device errors, and
                                   reject non-finite query values with HNTL_EINVAL */
#define HNTL_FLAG_CHECK_Q 2u    /* reject non-finite query values with HNTL_EINVAL (implies a sync);
                                   asynchronous calls without it do not check */
#define HNTL_FLAG_PROFILE 4u    /* record HIP events around each stage on the call's stream (see hntl_profile_read) */
#define HNTL_FLAG_NO_PRUNE 8u   /* scan every member of every probed grain (see below) */
#define HNTL_FLAG_PROJECT_BF16 16u /* projection on BF16 MFMA: q - mu_g (FP32) and W_g rounded to BF16 (nearest
                                      even), FP32 accumulation; eps_q stays FP32.  Needs an index with a
                                      reduced-precision code form (the BF16 bases are built with it) and d % 8 == 0 */
#define HNTL_FLAG_MODE_A 64u /* the paper's Mode A (Section 2.1): the answer comes from the index alone, no raw
                                vectors are read: the k smallest reconstruction distances
                                ||q - (mu_g + W_g z_i)||^2 = ||z_q - z_i||^2 + eps_q over the pool (eq. 2-4 and 6;
                                computed as the pool's eq. 6 score minus eps_i).  The returned distances are
                                these.  Needs the merged pool (not an injected one) */
/*
 * Centroid routing (Section 2.1 step 1).  The P probes are always the P
 * nearest centroids by FP32 direct differences ||q - mu_g||^2 (ties: lower g).
 * They are found from a shortlist of expansion distances
 * ||q||^2 + ||mu_g||^2 - 2 <q, mu_g> whose products run on MFMA in one of three
 * forms; every shortlist entry that the form's error bound leaves in reach of
 * the P-th is re-scored by direct differences (a row whose window passes the
 * shortlist's end is re-read whole), so the form changes speed, not probes.
 * Without either flag the products are FP32 MFMA.  Setting both is EINVAL.
 */
#define HNTL_FLAG_ROUTE_BF16X3 32u /* products on BF16 MFMA with each operand split into a BF16 high and low part
                                      (q_hi c_hi + q_hi c_lo + q_lo c_hi, FP32 accumulation, about 2^-16
                                      relative): three BF16 products.  Needs d % 8 == 0 */
#define HNTL_FLAG_ROUTE_BF16 128u  /* products on BF16 MFMA of bf16(q) . bf16(mu_g) (nearest even, FP32
                                      accumulation; error at most about 2^-8 (||q||^2 + ||mu||^2) / 2 per entry,
                                      a wider re-scored window): one BF16 product.  Needs d % 8 == 0 */
/*
 * Exact pruning.  By default the nearest probed grain of each query is scanned
 * first; its C-th best (D, id) key then bounds the other probed grains: their
 * candidates must beat it to enter the pool, and a grain is skipped outright
 * when a lower bound of eq. 6 over the grain (squared distance from z_q to the
 * bounding box of the grain's codes, plus eps_q, plus the grain's smallest
 * eps_i) exceeds it by a relative margin of 1e-4.  Pool and results are the
 * same as without pruning; HNTL_FLAG_NO_PRUNE scans everything.
 */

/* Stages timed by HNTL_FLAG_PROFILE, in order. */
#define HNTL_STAGE_ROUTE 0      /* centroid distances (MFMA) + top-P select */
#define HNTL_STAGE_BUCKET 1     /* grouping of (query, probe) pairs by grain */
#define HNTL_STAGE_PROJECT 2    /* projection GEMM + eps_q */
#define HNTL_STAGE_SCAN 3       /* Block-SoA scan + per-grain top-C */
#define HNTL_STAGE_RERANK 4     /* pool merge + exact rerank + top-k */
#define HNTL_NUM_STAGES 5

typedef struct hntl_index hntl_index; /* opaque */

/* Parameters of hntl_build. */
typedef struct hntl_build_params {
  uint32_t G;                 /* number of grains (k-means clusters), 1 <= G <= N */
  uint32_t r;                 /* tangent rank, 1 <= r <= min(d, HNTL_MAX_R) */
  uint32_t kmeans_iters;      /* maximum Lloyd iterations (0 = default 25) */
  uint32_t train_per_grain;   /* k-means trains on at most this many rows per grain (0 = default 256) */
  uint32_t eig_iters;         /* subspace iterations of the eigensolver (0 = default 40) */
  uint32_t codes_mask;        /* bit (1 << hntl_codes) for every code form to build; FP32 is always built */
  uint64_t seed;              /* seed of the build's counter-based random numbers */
  const float* init_centroids;/* optional G x d starting centroids (host or device); NULL = k-means++ */
} hntl_build_params;

/*
 * hntl_build - build an index from N raw vectors (Section 2.2: grains, local PCA
 * basis per grain, codes eq. 1-4, Block-SoA layout of Section 2.4).
 *   X       device, N x d float32, row-major.  Copied; the caller may free it after return.
 *   out     receives the new index; free it with hntl_index_free.
 * Synchronous.  Errors: EINVAL (null pointers, N == 0, d == 0, G > N, r > d),
 * EUNSUPPORTED (r > HNTL_MAX_R), ENOMEM, EDEVICE.
 */
hntl_status hntl_build(const float* X, uint64_t N, uint32_t d, const hntl_build_params* params,
                       void* stream, hntl_index** out);

/*
 * hntl_index_create - make an index from arrays in the stored format (import of an
 * index built elsewhere, e.g. exported earlier).  All pointers host or device.
 *   centroids  G x d          grain centroids mu_g
 *   basis      G x r x d      row j of grain g = column j of W_g (orthonormal columns)
 *   offsets    G + 1 int64    grain g owns grain-order positions [offsets[g], offsets[g+1])
 *   perm       N int32        grain-order position -> original row id (ascending inside a grain)
 *   codes      N x r          tangent coordinates z_i in grain order
 *   eps        N              residual energies eps_i in grain order (>= 0)
 *   X          N x d          raw vectors in original row order (copied for rerank), or NULL:
 *                             an index without raw vectors, which answers HNTL_FLAG_MODE_A
 *                             searches only (others fail with ESTATE)
 *   codes_mask as in hntl_build_params (derived reduced-precision codes to build)
 * Synchronous.  Errors: EINVAL (null pointer, inconsistent offsets/perm), EUNSUPPORTED, ENOMEM, EDEVICE.
 */
hntl_status hntl_index_create(uint64_t N, uint32_t d, uint32_t G, uint32_t r, const float* centroids,
                              const float* basis, const int64_t* offsets, const int32_t* perm,
                              const float* codes, const float* eps, const float* X, uint32_t codes_mask,
                              hntl_index** out);

/* Parameters of hntl_index_append (NULL = all defaults). */
typedef struct hntl_append_params {
  uint32_t split_max;         /* grains above this many members after the append are split (0 = never) */
  uint32_t eig_iters;         /* subspace iterations for the split grains' bases (0 = default 40) */
  uint64_t seed;              /* seed of the eigensolver's start vectors */
} hntl_append_params;

/*
 * hntl_index_append - a new index holding the rows of `base` plus n new rows
 * (Section 1 and the segment layer of Section 2 with Fig. 1: grains are
 * self-contained, so appending touches no other grain and no existing code).
 * `base` is not modified (an immutable segment); the result is independent of
 * it and both are freed separately.
 *   X       n x d float32 row-major, host or device; the new rows get ids
 *           N .. N + n - 1.  Copied.  n = 0 gives a copy of base.
 * Each new row joins the grain of its nearest centroid (FP32 distances, ties
 * to the lower grain) and is encoded by eq. 1-4 with that grain's stored
 * centroid and basis (FP64 arithmetic from the stored FP32 values); the
 * centroids, bases and codes of existing members are kept bit for bit.  With
 * split_max > 0, a grain holding more than split_max members is cut into
 * m = ceil(n_g / split_max) children: members ordered by their stored FP32
 * first code coordinate (ties by id) and cut into m runs whose sizes differ by
 * at most one; child 0 keeps the grain's number, children 1 .. m-1 get the
 * numbers G, G + 1, ... in ascending order of the grains split; every child
 * gets the exact FP64 mean of its members as centroid, its own local PCA basis
 * (as in hntl_build) and new codes.  The result holds the base's code forms
 * (codes_mask) and no learned router (train or import one again).
 * Synchronous.  Errors: EINVAL (null base/out, X NULL with n > 0),
 * EUNSUPPORTED (N + n >= 2^31; split_max > 0 on an index without raw
 * vectors), ENOMEM, EDEVICE.
 */
hntl_status hntl_index_append(const hntl_index* base, const float* X, uint64_t n,
                              const hntl_append_params* params, void* stream, hntl_index** out);

/*
 * hntl_index_save / hntl_index_load - an index as a directory of files (the
 * immutable segment of Section 2, Fig. 1, on disk): one NumPy .npy file per
 * stored-format array (centroids f4 G x d, basis f4 G x r x d, offsets i8 G+1,
 * perm i4 N, codes f4 N x r in grain order, eps f4 N), X.npy (f4 N x d) when
 * the index holds raw vectors, captured.npy (f8 G) when the build recorded it,
 * the learned router's arrays (router_W1.npy .. router_std.npy) when it has one,
 * and meta.json with the sizes, the code forms and a 64-bit FNV-1a checksum of
 * every file's data bytes.  save creates `dir` if needed and overwrites the
 * files; load reads what save wrote, verifies every checksum and shape, and
 * builds the index as hntl_index_create does (same checks), with the router and
 * captured record restored.  Host-side files; synchronous.
 * Errors: EINVAL (null pointers), EIO (unwritable or missing directory or file,
 * malformed header, shape or checksum mismatch), ENOMEM, EDEVICE, and the
 * errors of hntl_index_create for inconsistent arrays.
 */
hntl_status hntl_index_save(const hntl_index* index, const char* dir);
hntl_status hntl_index_load(const char* dir, hntl_index** out);

/*
 * hntl_index_export - copy the stored-format arrays out of an index.  Any pointer may
 * be NULL to skip that array; all are host or device, sized as in hntl_index_create.
 * scales receives the G per-grain FP8 scales (ESTATE if FP8 codes were not built).
 * Synchronous.
 */
hntl_status hntl_index_export(const hntl_index* index, float* centroids, float* basis, int64_t* offsets,
                              int32_t* perm, float* codes, float* eps, float* scales);

/*
 * hntl_index_export_codes - the reduced-precision codes of an index, unpacked to
 * N x r in grain order: uint16 BF16 bit patterns (codes = HNTL_CODES_BF16),
 * uint8 E4M3fn bit patterns (codes = HNTL_CODES_FP8_E4M3, value = code * scales[g],
 * scales: the G FP8 scales) or int16 codes z_hat (codes = HNTL_CODES_INT16,
 * scales: the G inv_g).  With codes = HNTL_CODES_INT16 | HNTL_EXPORT_RESIDUALS,
 * out receives the N uint16 residual codes r_hat_i (eq. 5, grain order) and
 * scales the G rinv_g.  out and scales are host or device and may be NULL.
 * Errors: EINVAL (FP32 requested, residuals of another form), ESTATE (form not
 * built).  Synchronous.
 */
#define HNTL_EXPORT_RESIDUALS 0x100u
hntl_status hntl_index_export_codes(const hntl_index* index, uint32_t codes, void* out, float* scales);

typedef struct hntl_index_info {
  uint64_t N;
  uint32_t d, G, r;
  uint32_t block;             /* Block-SoA block size B */
  uint32_t codes_mask;        /* code forms present */
  uint64_t n_blocks;          /* total Block-SoA blocks over all grains */
  uint64_t device_bytes;      /* device memory held by the index */
  double captured_variance;   /* mean over non-empty grains of the captured fraction (build only, else -1) */
  uint32_t kmeans_iters_run;  /* Lloyd iterations executed (build only) */
  uint32_t max_grain;         /* largest grain size */
} hntl_index_info;

hntl_status hntl_index_info_get(const hntl_index* index, hntl_index_info* out);

/* hntl_index_captured - per-grain captured-variance fraction (G floats, host). Build only. */
hntl_status hntl_index_captured(const hntl_index* index, double* out);

void hntl_index_free(hntl_index* index);

/* Parameters of a search. */
/* Routing of step 1. */
typedef enum hntl_route {
  HNTL_ROUTE_CENTROID = 0, /* the P grains with the closest centroids (Section 2.1 step 1) */
  HNTL_ROUTE_LEARNED = 1   /* the P grains with the largest learned-router scores (see hntl_router_train) */
} hntl_route;

typedef struct hntl_search_params {
  uint32_t P;       /* probes per query, 1 <= P <= min(G, HNTL_MAX_P) */
  uint32_t C;       /* candidate pool per query, k <= C <= HNTL_MAX_C */
  uint32_t k;       /* results per query, >= 1 */
  uint32_t codes;   /* hntl_codes form to scan */
  uint32_t flags;   /* HNTL_FLAG_* */
  uint32_t route;   /* hntl_route; LEARNED needs a trained or imported router (else ESTATE) */
  float tau;        /* learned routing only: a query whose largest softmax probability over the grains
                       is below tau is routed by centroids instead (0 = never) */
  float mass;       /* learned routing only, a probe budget: the top-P grains are kept up to and
                       including the first slot at which the cumulative softmax probability (over all
                       G router scores) reaches mass; later slots are probe -1 (not searched).
                       0 or 1 = all P slots; must lie in [0, 1].  Ignored by centroid routing */
} hntl_search_params;

/*
 * hntl_search - the whole query lifecycle for nq queries.
 *   Q     device, nq x d float32
 *   ids   device, nq x k int32  (original row ids, ascending distance, -1 padded)
 *   dist  device, nq x k float32 (squared L2; +inf where ids is -1)
 * nq == 0 is a no-op.  Errors: EINVAL, ESTATE (codes form not built), EUNSUPPORTED, EDEVICE.
 */
hntl_status hntl_search(const hntl_index* index, const float* Q, uint32_t nq, const hntl_search_params* sp,
                        int32_t* ids, float* dist, void* stream);

/*
 * hntl_search_noalloc - hntl_search for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  Same arguments, arithmetic and results as hntl_search
 * (the same kernels); the call's scratch (routing distances, bucketing
 * arrays, tangents, candidate lists) comes from one static device array of
 * HNTL_NOALLOC_SCRATCH_BYTES per GPU, held by the library until the process
 * ends, instead of the stream-ordered pool.  The call makes no hipMalloc or
 * hipFree; the caller still owns Q, ids and dist.
 *   - A call whose scratch would exceed HNTL_NOALLOC_SCRATCH_BYTES fails with
 *     EINVAL (the message states the bytes it needs): the scratch grows with
 *     nq x (G + P x (r + C x 2)) x 4 bytes plus a few G-sized arrays.
 *   - Derived index data is not made here: the BF16 routing forms need the
 *     index's split centroids and Mode A its eps by id, which the first
 *     hntl_search with the same flags makes; without them: ESTATE.
 *   - HNTL_FLAG_PROFILE is refused (EINVAL); HNTL_FLAG_CHECK_Q and
 *     HNTL_FLAG_SYNC synchronise the stream as in hntl_search.
 *   - Every call on one GPU uses that GPU's one array and leaves its contents
 *     behind; each call clears what it needs cleared.  Calls that overlap on
 *     one GPU (other streams or host threads) race on it: serialise them.
 */
#define HNTL_NOALLOC_SCRATCH_BYTES (64u << 20) /* 64 MiB per GPU */
hntl_status hntl_search_noalloc(const hntl_index* index, const float* Q, uint32_t nq, const hntl_search_params* sp,
                                int32_t* ids, float* dist, void* stream);

/*
 * hntl_search_stages - the same lifecycle with every stage's output observable and
 * every stage's input injectable, for stage-by-stage checking.  All pointers device;
 * any may be NULL.
 *   probes_in   nq x P int32   replaces step 1 (probe lists; each row distinct grain ids)
 *   probes_out  nq x P int32,  pdist_out nq x P float32 (squared distance to the centroid)
 *   tangent_in  nq x P x r float32 and epsq_in nq x P: replace step 2 (both or neither)
 *   tangent_out nq x P x r,    epsq_out nq x P
 *   pool_in     nq x C int32   replaces steps 1-3 (candidate pool ids, -1 padded)
 *   pool_out    nq x C int32,  pool_D_out nq x C float32 (eq. 6 score, +inf padded)
 *   ids, dist   as in hntl_search
 * When pool_in is given, Q, ids and dist are still required and steps 1-3 are skipped.
 */
hntl_status hntl_search_stages(const hntl_index* index, const float* Q, uint32_t nq,
                               const hntl_search_params* sp, const int32_t* probes_in,
                               int32_t* probes_out, float* pdist_out, const float* tangent_in,
                               const float* epsq_in, float* tangent_out, float* epsq_out,
                               const int32_t* pool_in, int32_t* pool_out, float* pool_D_out,
                               int32_t* ids, float* dist, void* stream);

/*
 * hntl_profile_read - per-stage device time of the searches issued by the calling
 * thread with HNTL_FLAG_PROFILE since the last read.  Waits for those events to
 * complete, then writes the summed milliseconds per stage into ms[0..n), the
 * number of timed calls into *calls and the number of eq. 6 scores computed
 * (query-grain pairs scanned times their grain sizes) into *scored (any of the
 * three may be NULL), and clears the record.  Stages skipped by stage injection
 * count 0 ms.
 */
hntl_status hntl_profile_read(double* ms, uint32_t n, uint32_t* calls, uint64_t* scored);

/* ------------------------------------------------------------------------
 * Batching form: persistent fused search plans
 * ------------------------------------------------------------------------
 * A plan fixes (index, search params, largest batch max_nq, schedule) and owns
 * every device buffer of the search, allocated once: the query, result and
 * scratch arrays.  Running a plan allocates nothing.  Steps 2-3 run as one
 * persistent fused project-scan-select kernel whose workgroups take work
 * items from a device queue, largest grain first; large grains are split into
 * block ranges, and every query shares one running bound on its pool between
 * the items (exact pruning, see HNTL_FLAG_NO_PRUNE).  With HNTL_PLAN_GRAPH the
 * plan captures its whole launch sequence (reset, routing, bucketing, fused
 * kernel, merge + rerank) into a HIP graph once, at creation, and every run
 * replays it: the batch size is read from device memory, so replays of one
 * plan need no host work beyond the launch.  Results equal those of
 * hntl_search with the same parameters (the pool is the exact top C of the
 * probed grains in both).
 *
 * A plan reads its index until it is freed; free every plan before its index.
 * Runs of one plan on different streams must not overlap (they share the
 * plan's buffers); different plans may run concurrently.
 */
typedef struct hntl_plan hntl_plan; /* opaque */

/* Work schedule of the fused kernel (picked by hntl_tune or given). */
typedef struct hntl_schedule {
  uint32_t qt;     /* pairs per wave in a scan item: 1, 2, 4 or 8 */
  uint32_t nw;     /* waves per workgroup, 1..8: a scan item holds nw * qt pairs of one grain */
  uint32_t range;  /* blocks of 64 vectors per scan item (0 = whole grain); larger grains
                      give one item per range, whose lists the merge joins */
  uint32_t grid;   /* workgroups of the persistent launch (0 = as many as are resident at once) */
  uint32_t passes; /* 1: every item in one launch; 2: projection and probe-slot-0 items in a first launch,
                      the other slots in a second one, which then start from each query's slot-0 bound
                      (0 = 1) */
  uint32_t proj;   /* 0: projection items run inside the fused kernel; 1: a grain-major projection
                      launch (16 pairs of one grain per single-wave workgroup) runs before it and
                      the fused kernel only scans and selects */
} hntl_schedule;

#define HNTL_PLAN_GRAPH 1u /* capture a HIP graph at creation; runs replay it */

/*
 * hntl_plan_create - a plan for batches of up to max_nq queries.
 *   index   the index (must outlive the plan); needs d % 8 == 0 and a padded rank
 *           8 * ceil(r / 8) of 16, 32, 48 or 64
 *   sp      search parameters as for hntl_search (flags: HNTL_FLAG_PROJECT_BF16,
 *           HNTL_FLAG_NO_PRUNE are honoured; HNTL_FLAG_SYNC applies to every run)
 *   sched   NULL = a default chosen from the batch shape
 *   stream  stream used for the one-time setup (and for graph capture through a
 *           private stream)
 * Errors: EINVAL, ESTATE, EUNSUPPORTED (shape outside the compiled kernels, or a
 * schedule whose workgroup needs more than 64 KiB of LDS), ENOMEM, EDEVICE.
 */
hntl_status hntl_plan_create(hntl_index* index, const hntl_search_params* sp, uint32_t max_nq,
                             const hntl_schedule* sched, uint32_t plan_flags, void* stream, hntl_plan** out);

/*
 * hntl_plan_buffers - the plan's own device buffers: Q (max_nq x d float32),
 * ids (max_nq x k int32), dist (max_nq x k float32).  Writing queries into Q and
 * calling hntl_plan_run avoids the copies of hntl_plan_search.  Any pointer may be NULL.
 */
hntl_status hntl_plan_buffers(hntl_plan* plan, float** Q, int32_t** ids, float** dist);

/*
 * hntl_plan_run - search the first nq rows of the plan's Q buffer (nq <= max_nq);
 * results land in the plan's ids / dist buffers (rows >= nq hold -1 / +inf).
 * Asynchronous on `stream` unless HNTL_FLAG_SYNC was given; then a wait that gave up
 * inside the fused kernel is reported as EDEVICE.
 */
hntl_status hntl_plan_run(hntl_plan* plan, uint32_t nq, void* stream);

/*
 * hntl_plan_search - copy nq queries (device) into the plan, run it, copy the
 * results out (device ids nq x k, dist nq x k).  Q, ids and dist may also be the
 * plan's own buffers (no copy then).
 */
hntl_status hntl_plan_search(hntl_plan* plan, const float* Q, uint32_t nq, int32_t* ids, float* dist,
                             void* stream);

typedef struct hntl_plan_info {
  uint32_t max_nq;
  hntl_schedule sched;     /* the schedule in use (grid resolved) */
  uint32_t graph;          /* 1 if runs replay a captured graph */
  uint64_t device_bytes;   /* the plan's device buffers */
  uint64_t list_slots;     /* capacity of per-(pair, range) candidate lists */
  uint32_t wait_errors;    /* waits that gave up since creation (0 in a healthy run) */
} hntl_plan_info;

/* hntl_plan_info_get - plan facts; synchronises the plan's last stream to read wait_errors. */
hntl_status hntl_plan_info_get(hntl_plan* plan, hntl_plan_info* out);

/*
 * hntl_plan_profile - run the plan reps times without its graph, with HIP events
 * between its stages on `stream`, and return the mean device milliseconds per stage
 * in stage_ms[0..5): routing, bucketing (with the resets), the separate projection
 * launch (schedule proj = 1; 0 otherwise), the fused project-scan-select kernel,
 * merge + rerank.  *scored (may be NULL) receives the
 * eq. 6 scores the last run computed.  The queries are the first nq rows of the
 * plan's Q buffer.  Synchronous.
 */
hntl_status hntl_plan_profile(hntl_plan* plan, uint32_t nq, uint32_t reps, double* stage_ms, uint64_t* scored,
                              void* stream);

void hntl_plan_free(hntl_plan* plan);

/*
 * hntl_tune - the autotuner.  Times every candidate schedule of the fused kernel
 * (proj in {0, 1} x passes in {1, 2} x qt in {1, 2, 4, 8} x nw in {1, 2, 4, 8} x range in
 * {0, 8, 32, 64}, those whose LDS fits) on the nq given queries (device, nq x d) and returns the fastest in *best
 * (*best_ms its median device time of one run).  With db_path != NULL the result is
 * also stored in that text file, one line per (device, index shape, search params,
 * batch size), replacing an older line of the same key; hntl_schedule_lookup reads it.
 */
hntl_status hntl_tune(hntl_index* index, const hntl_search_params* sp, const float* Q, uint32_t nq,
                      const char* db_path, hntl_schedule* best, float* best_ms, void* stream);

/*
 * hntl_schedule_lookup - the schedule stored by hntl_tune for this device, index
 * shape, search params and batch size max_nq.  ESTATE if the file has no such entry
 * (or does not exist).
 */
hntl_status hntl_schedule_lookup(const hntl_index* index, const hntl_search_params* sp, uint32_t max_nq,
                                 const char* db_path, hntl_schedule* out);

/* ------------------------------------------------------------------------
 * Learned router (an extension: the paper routes by centroid distance,
 * Section 2.3, and lists learned partitioning as future work, Section 4)
 * ------------------------------------------------------------------------
 * An MLP d -> hidden1 -> hidden2 -> G with GELU (exact erf form) maps a
 * standardised query xh = (q - mean) / std to one score per grain:
 *   s = W3 gelu(W2 gelu(W1 xh + b1) + b2) + b3.
 * Weights are FP32 with BF16 copies; the three GEMMs (and those of training)
 * run on BF16 MFMA with FP32 accumulation; each GEMM operand is rounded to
 * BF16 (nearest even).  Learned routing probes the P grains of largest score
 * (ties: lower grain id).
 */
#define HNTL_ROUTER_KEEP_WEIGHTS 1u /* continue from the index's current router (no initialisation,
                                       mean/std kept) */
#define HNTL_ROUTER_NO_SHUFFLE 2u   /* batches in input order (default: reshuffled every epoch) */

typedef struct hntl_router_params {
  uint32_t hidden1, hidden2; /* hidden widths (0 = 1024); multiples of 8 */
  uint32_t epochs;           /* passes over the training queries (0 = 1) */
  uint32_t batch;            /* rows per Adam step (0 = 1024); a partial last batch is dropped */
  uint32_t knn;              /* neighbours per training query forming its target (0 = 10, at most 16) */
  uint32_t flags;            /* HNTL_ROUTER_* */
  float lr;                  /* Adam step size (0 = 1e-3; beta1 0.9, beta2 0.999, eps 1e-8) */
  uint64_t seed;             /* initialisation and shuffling (counter-based generator) */
} hntl_router_params;

/*
 * hntl_router_train - train the index's router on n queries (device, n x d).
 * Target of query i: the grain distribution of its exact knn nearest rows of
 * the index (brute force on the GPU, see hntl_knn), or the given targets
 * (device, n x knn grain ids, each weighing 1 / knn).  Loss: mean softmax
 * cross-entropy; Adam on the FP32 masters.  Without HNTL_ROUTER_KEEP_WEIGHTS
 * the router is (re)initialised (He-style uniform) and mean / std are the
 * column statistics of the training queries.  epoch_loss (host, epochs floats)
 * may be NULL.  Synchronous.  Errors: EINVAL (n < batch), EUNSUPPORTED (sizes
 * not multiples of 8, knn > 16), ENOMEM, EDEVICE.
 */
hntl_status hntl_router_train(hntl_index* index, const float* Qtrain, uint32_t n, const int32_t* targets,
                              const hntl_router_params* params, float* epoch_loss, void* stream);

/*
 * hntl_router_set / hntl_router_export - import or read the router's FP32
 * weights: W1 hidden1 x d, b1 hidden1, W2 hidden2 x hidden1, b2 hidden2,
 * W3 G x hidden2, b3 G (row-major, out x in), mean and std (d).  Pointers are
 * host or device; export pointers may be NULL.  Synchronous.
 */
hntl_status hntl_router_set(hntl_index* index, uint32_t hidden1, uint32_t hidden2, const float* W1, const float* b1,
                            const float* W2, const float* b2, const float* W3, const float* b3, const float* mean,
                            const float* std);
hntl_status hntl_router_export(const hntl_index* index, uint32_t* hidden1, uint32_t* hidden2, float* W1, float* b1,
                               float* W2, float* b2, float* W3, float* b3, float* mean, float* std);

/* hntl_router_forward - router scores of nq queries (device nq x d) into scores (device nq x G). */
hntl_status hntl_router_forward(const hntl_index* index, const float* Q, uint32_t nq, float* scores, void* stream);

/*
 * hntl_router_grad - loss and gradients of the router at its current weights for
 * the batch X (device, n x d) with targets (device, n x kt grain ids), without
 * updating it: gW* / gb* (host or device, shaped like the weights; any may be NULL),
 * *loss (host).  Synchronous.
 */
hntl_status hntl_router_grad(hntl_index* index, const float* X, uint32_t n, const int32_t* targets, uint32_t kt,
                             float* loss, float* gW1, float* gb1, float* gW2, float* gb2, float* gW3, float* gb3,
                             void* stream);

/*
 * hntl_knn - exact k nearest raw vectors of the index for nq queries (device),
 * k <= 16: ids (device nq x k, original row ids, ascending distance, ties to the
 * lower id) and dist (device nq x k squared L2, may be NULL).  A 32-entry MFMA
 * expansion shortlist per query is re-scored by direct differences in FP32.
 */
hntl_status hntl_knn(const hntl_index* index, const float* Q, uint32_t nq, uint32_t k, int32_t* ids, float* dist,
                     void* stream);

/* Last error message of the calling thread ("" if none). */
const char* hntl_last_error(void);

/* Library version string. */
const char* hntl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HNTL_H_ */
