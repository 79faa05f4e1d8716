"""Benchmark of the HNTL search path on one MI355X.

Workload (default): the batching workload, 10,000,000 patch-mixture vectors,
d = 768, Zipf(1.1)-sized patches (16..20,000 members) over 8,192 patches;
index G = 8,192 k-means grains, r = 48; batches of 16,384 queries; P = 16,
C = 100, k = 10; FP32 codes.  A step is one full search of the batch (route,
bucket, project, scan + select, merge + rerank), inputs resident in HBM, run
by an autotuned search plan (the persistent fused project-scan-select kernel,
launch sequence replayed as a HIP graph; stage times come from eager profiled
runs with HIP events on the plan's stream).

Beside the headline (plain FP32 plan) the same JSON line carries, by default on
the batching workload:
  centroid_bf16  centroid routing with BF16 codes and BF16 projection, same P
                 and C (the precision form without the router)
  learned_bf16   the learned router (768-1024-1024-8192, trained first on
                 200,000 generated queries with brute-force kNN targets) with
                 BF16 codes and BF16 projection, same P and C, its Recall@10 on
                 the same query sample and its speed-up over the plain form
  scan_hbm       the scan in its HBM-bound regime: a 256-query batch, the fused
                 scan kernel's time against the unique code bytes of the
                 probed grains
  uneven_batches a seeded sequence of uneven batch sizes (1 .. 16,384,
                 65,536 queries in total) through one plan
  cpu_baseline   the CPU oracle (FP64 numpy) on a bounded query sample, over a
                 process pool on the host cores

Other forms are flags of the same script:
  --workload patch1M_d768_G1024_r32   the 1M-vector plain workload
  --form staged    hntl_search: one launch per stage
  --sched ...      a fixed plan schedule instead of the autotuner's
  --route learned  the learned router as the headline form
  --codes bf16|fp8 reduced-precision codes (BF16 MFMA projection by default)
  --codes int16    the paper's own int16 form (eq. 5, envelope filter, integer distances)
  --mode A         the answer from the index alone (no raw-vector rerank)
  --route-form     centroid routing's shortlist products (fp32, bf16, bf16x3)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "queries/sec and ns/vector scanned at Recall@10≥0.95; scan HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
# FP32 VALU without packed math (every HIP source is built with packed FP32
# off): 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA) x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 78.6
BF16_MFMA_PEAK_TFLOPS = 2500.0

# Measured DRAM traffic (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch, each scaled by its reading for a plain 1 GiB device copy) of
# kernels on given workloads; valid while the kernel's sources are unchanged
# (sha1 of the listed files).  Each entry names the profile summary it comes
# from.
_SCAN_SRC = ("paper_2606_08813_amd/csrc/fused_impl.h", "paper_2606_08813_amd/csrc/scan_impl.h",
             "paper_2606_08813_amd/csrc/hntl_device.h", "paper_2606_08813_amd/csrc/plan.hip",
             "paper_2606_08813_amd/csrc/bucket.hip")
_SHA = {
    "paper_2606_08813_amd/csrc/fused_impl.h": "077cb0221488c77b89f0cfbb719688a9350e9d16",
    "paper_2606_08813_amd/csrc/scan_impl.h": "08b1aa9c637b5afc8f01025d863320b4b9fa4998",
    "paper_2606_08813_amd/csrc/hntl_device.h": "8042d049177634c7c50bf9f741925e63359e7b21",
    "paper_2606_08813_amd/csrc/plan.hip": "7a6f9b44aa5f8ef18a7c9574b2ad2af57c79e889",
    "paper_2606_08813_amd/csrc/bucket.hip": "dc32fc07f95bbf8d60d3997767278e18c59cc518",
    "paper_2606_08813_amd/csrc/fused_ct0.hip": "dce4677b8d7025d96f78ce59f33911b619912e08",
    "paper_2606_08813_amd/csrc/fused_ct1.hip": "a15377c01ab0b4b06e0a90b3788ed3259d5aad97",
    "paper_2606_08813_amd/csrc/rerank.hip": "10c86c447d3bd19bc14c2dbd764d3fc5305ff15d",
    "paper_2606_08813_amd/csrc/project.hip": "ac70a7ba410f94fcf3a0388a38a0e5c439942fd7",
    "paper_2606_08813_amd/csrc/project_impl.h": "b7f2c4adb2e898712edc62fc094072e5ff0dab9b",
}


def _traffic(kernel, codes, batch, fetch_kib, write_kib, sources, profile, sched=None):
    return {"kernel": kernel, "workload": "zipf10M_d768_G8192_r48", "form": "plan", "codes": codes, "P": 16,
            "mode": "B", "batch": batch, "fetch_kib": fetch_kib, "write_kib": write_kib, "fetch_scale": 2.0,
            "write_scale": 1.0, "sources": {f: _SHA[f] for f in sources}, "profile": profile, "sched": sched}


# the fused scan's traffic depends on its tiles, ranges and passes (not on the
# waves per workgroup)
_WIDE = {"qt": 8, "range": 32, "passes": 1}
_NARROW = {"qt": 1, "range": 32, "passes": 2}


# per plan run: the fused scan launch(es), the separate projection launch, the
# merge + rerank launch (KiB per dispatch; the two-pass 256-query plan's two
# scan launches summed)
TRAFFIC = [
    _traffic("scan", "fp32", 16384, 2.196e6, 8.634e4, _SCAN_SRC + ("paper_2606_08813_amd/csrc/fused_ct0.hip",),
             "profiles/fused_scan_zipf10M_d768_G8192_r48_dram_counters.md", _WIDE),
    _traffic("scan", "fp32", 256, 7.962e4 + 1.121e5, 710.0 + 891.8,
             _SCAN_SRC + ("paper_2606_08813_amd/csrc/fused_ct0.hip",),
             "profiles/fused_scan_zipf10M_d768_G8192_r48_dram_counters.md", _NARROW),
    _traffic("scan", "bf16", 16384, 1.120e6, 8.752e4, _SCAN_SRC + ("paper_2606_08813_amd/csrc/fused_ct1.hip",),
             "profiles/fused_scan_zipf10M_d768_G8192_r48_dram_counters.md", _WIDE),
    _traffic("scan", "bf16", 256, 4.122e4 + 5.823e4, 709.9 + 891.6,
             _SCAN_SRC + ("paper_2606_08813_amd/csrc/fused_ct1.hip",),
             "profiles/fused_scan_zipf10M_d768_G8192_r48_dram_counters.md", _NARROW),
    _traffic("rerank", "fp32", 16384, 2.666e6, 3712.0, ("paper_2606_08813_amd/csrc/rerank.hip",),
             "profiles/merge_rerank_zipf10M_d768_G8192_r48_dram_counters.md"),
    _traffic("project", "fp32", 16384, 7.475e5, 5.759e4,
             ("paper_2606_08813_amd/csrc/project.hip", "paper_2606_08813_amd/csrc/project_impl.h"),
             "profiles/projection_zipf10M_d768_G8192_r48_counters.md"),
    _traffic("project", "bf16", 16384, 5.59e5, 5.745e4,
             ("paper_2606_08813_amd/csrc/project.hip", "paper_2606_08813_amd/csrc/project_impl.h"),
             "profiles/projection_zipf10M_d768_G8192_r48_counters.md"),
]


def measured_traffic(kernel, workload, form, codes, P, mode, batch, sched=None):
    import hashlib
    for t in TRAFFIC:
        if (kernel, workload, form, codes, P, mode, batch) != (t["kernel"], t["workload"], t["form"], t["codes"],
                                                               t["P"], t["mode"], t["batch"]):
            continue
        if t["sched"] and (sched is None or any(sched.get(k) != v for k, v in t["sched"].items())):
            return None  # counted under another schedule
        for src, sha in t["sources"].items():
            p = ROOT / src
            if not p.exists() or hashlib.sha1(p.read_bytes()).hexdigest() != sha:
                return None  # the kernel changed since the counters were taken
        return round((t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0)
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Measurement helpers (FP64 host arithmetic; the timed path never uses them).
def exact_knn(X, Qs, k, chunk=1 << 16, extra=32):
    """Exact k nearest rows of X (squared L2) for each row of Qs: a float64
    expansion over row chunks keeps k + extra candidates per query, which are
    re-scored by direct differences."""
    Qd = np.asarray(Qs, dtype=np.float64)
    qn = (Qd ** 2).sum(1)
    m = k + extra
    cand_i = np.zeros((len(Qd), 0), np.int64)
    cand_d = np.zeros((len(Qd), 0))
    for a in range(0, len(X), chunk):
        Xc = np.asarray(X[a:a + chunk], dtype=np.float64)
        D = qn[:, None] + (Xc ** 2).sum(1)[None, :] - 2.0 * (Qd @ Xc.T)
        ci = np.concatenate([cand_i, np.broadcast_to(np.arange(a, a + len(Xc)), D.shape)], 1)
        cd = np.concatenate([cand_d, D], 1)
        keep = np.argpartition(cd, min(m, cd.shape[1] - 1), axis=1)[:, :m]
        cand_i = np.take_along_axis(ci, keep, 1)
        cand_d = np.take_along_axis(cd, keep, 1)
    ids = np.empty((len(Qd), k), np.int64)
    for i in range(len(Qd)):
        dd = ((np.asarray(X[cand_i[i]], dtype=np.float64) - Qd[i]) ** 2).sum(1)
        o = np.lexsort((cand_i[i], dd))[:k]
        ids[i] = cand_i[i][o]
    return ids


def recall_at_k(ids, gt, k):
    return float(np.mean([len(set(a[:k].tolist()) & set(b[:k].tolist())) / k for a, b in zip(ids, gt)]))


def fp64_grain_scores(q, g, ex):
    """eq. 6 scores ||z_q - z_i||^2 + eps_q + eps_i of every member of grain g,
    from the stored centroid, basis, codes and eps in float64 (eq. 1-4 for q)."""
    mu = ex["centroids"][g].astype(np.float64)
    W = ex["basis"][g].astype(np.float64)
    qp = np.asarray(q, dtype=np.float64) - mu
    z = W @ qp
    e = qp - W.T @ z
    a, b = int(ex["offsets"][g]), int(ex["offsets"][g + 1])
    Z = ex["codes"][a:b].astype(np.float64)
    return ex["perm"][a:b], ((Z - z) ** 2).sum(1) + float(e @ e) + ex["eps"][a:b].astype(np.float64)


def uneven_batch_sizes(total=65536, seed=104):
    """Seeded uneven batch sizes: 1, 2, 7, 64, 500, 1000, 4096, 8192, 16384,
    then log-uniform draws in [1, 16384] until the sizes sum to `total` (the last
    one cut to fit)."""
    sizes = [1, 2, 7, 64, 500, 1000, 4096, 8192, 16384]
    rng = np.random.default_rng(seed)
    while sum(sizes) < total:
        sizes.append(int(np.exp(rng.uniform(0.0, np.log(16384.0)))))
    sizes[-1] -= sum(sizes) - total
    return [s for s in sizes if s > 0]


# ------------------------------------------------------- CPU oracle over a pool
# The pool is forked before anything touches the GPU; the workers read the
# corpus and queries inherited from the parent and the index from files the
# parent writes after the GPU build.  They run the oracle only.
_CPU = {}


def _cpu_worker_init():
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        from threadpoolctl import threadpool_limits
        _CPU["limit"] = threadpool_limits(1)
    except Exception:
        pass


def _cpu_worker_run(job):
    from oracle import search as osr
    path, idx, P, C, k, mode = job
    if _CPU.get("path") != path:
        _CPU["ex"] = {f[:-4]: np.load(os.path.join(path, f), mmap_mode="r") for f in os.listdir(path)
                      if f.endswith(".npy")}
        _CPU["path"] = path
    t0 = time.time()
    osr.search(_CPU["queries"][idx], _CPU["ex"], _CPU["corpus"], P, C, k, mode=mode)
    return len(idx), time.time() - t0


def start_cpu_pool(corpus_X, queries_X):
    import multiprocessing as mp
    n = max(1, min(len(os.sched_getaffinity(0)), 16))
    _CPU["corpus"] = corpus_X
    _CPU["queries"] = queries_X
    ctx = mp.get_context("fork")
    return ctx.Pool(n, initializer=_cpu_worker_init), n


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_cpu_baseline(pool, ncores, ex, nq, P, C, k, mode, seconds, scanned_per_query):
    """Wall time of the oracle over the pool on chunks of 8 sampled queries,
    stopping once `seconds` have passed; queries/s = completed / wall."""
    import shutil
    import tempfile
    d = tempfile.mkdtemp(prefix="hntl_oracle_", dir="/dev/shm" if os.path.isdir("/dev/shm") else None)
    try:
        for key in ("centroids", "basis", "offsets", "perm", "codes", "eps"):
            np.save(os.path.join(d, key + ".npy"), np.ascontiguousarray(ex[key]))
        order = np.random.default_rng(11).permutation(nq)
        jobs = [(d, order[i:i + 8], P, C, k, mode) for i in range(0, nq, 8)]
        done = 0
        t0 = time.time()
        for cnt, _ in pool.imap_unordered(_cpu_worker_run, jobs):
            done += cnt
            if time.time() - t0 > seconds:
                break
        wall = time.time() - t0
        pool.terminate()
        pool.join()
    finally:
        shutil.rmtree(d, ignore_errors=True)
    qps = done / wall
    return {"value": round(qps, 2), "unit": "queries/s", "cores": ncores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{done} of the {nq} queries in seeded random order (chunks of 8 over {ncores} worker "
                      f"processes, one thread each, until {seconds:g} s of wall time), the full lifecycle in float64 "
                      f"(numpy), same index and corpus; {wall:.1f} s",
            "ns_per_vector_scanned_per_core": round(wall * ncores / done / scanned_per_query * 1e9, 2)}


# ------------------------------------------------------------------- the GPU side
def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="zipf10M_d768_G8192_r48")
    ap.add_argument("--codes", choices=("fp32", "bf16", "fp8", "int16"), default="fp32")
    ap.add_argument("--recall-sample", type=int, default=200)
    ap.add_argument("--cpu-sample", type=int, default=-1,
                    help="0 skips the CPU oracle baseline; otherwise it runs for --cpu-seconds")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="wall seconds of the CPU oracle over the process pool")
    ap.add_argument("--no-profile", action="store_true", help="skip per-stage HIP event records")
    ap.add_argument("--no-prune", action="store_true", help="scan every member of every probed grain")
    ap.add_argument("--fp32-project", action="store_true",
                    help="with --codes bf16/fp8, keep the FP32 projection (default: BF16 MFMA projection)")
    ap.add_argument("--error-sample", type=int, default=100,
                    help="queries for the reduced-precision error report against FP64 scores of the stored index")
    ap.add_argument("--form", choices=("staged", "plan"), default="plan",
                    help="staged: hntl_search; plan: the persistent fused kernel in an autotuned, graph-replayed plan")
    ap.add_argument("--sched", default="",
                    help="plan schedule instead of autotuning, e.g. qt=4,nw=2,range=0,passes=2,proj=1")
    ap.add_argument("--route", choices=("centroid", "learned"), default="centroid",
                    help="learned: train the router first (router-train queries, brute-force kNN targets)")
    ap.add_argument("--P", type=int, default=0, help="probes per query (0 = the workload's)")
    ap.add_argument("--tau", type=float, default=0.0, help="learned routing: centroid fallback below this max prob")
    ap.add_argument("--mass", type=float, default=0.0,
                    help="learned routing: probe budget, stop at this cumulative softmax probability (0 = all P)")
    ap.add_argument("--compare-mass", type=float, default=0.99,
                    help="probe budget of the learned comparison's second line (0 = skip that line)")
    ap.add_argument("--mode", choices=("A", "B"), default="B",
                    help="B: exact rerank against the raw vectors; A: the answer from the index alone")
    ap.add_argument("--route-form", choices=("auto", "fp32", "bf16", "bf16x3"), default="auto",
                    help="centroid routing shortlist products: FP32 MFMA, one BF16 MFMA product, or three over "
                         "split BF16 operands (auto: bf16 when d % 8 == 0); the probes are picked by FP32 direct "
                         "differences either way")
    ap.add_argument("--router-train", type=int, default=200000, help="router training queries")
    ap.add_argument("--router-epochs", type=int, default=8)
    ap.add_argument("--compare", choices=("auto", "on", "off"), default="auto",
                    help="also time the learned router + BF16 codes + BF16 projection plan at the same P and C "
                         "(auto: on for the batching workload's default plain FP32 plan)")
    ap.add_argument("--hbm-sched", default="",
                    help="schedule of the HBM-regime plan instead of autotuning it (format of --sched)")
    ap.add_argument("--hbm-batch", type=int, default=-1,
                    help="queries of the scan's HBM-regime measurement (-1: 256 on the batching workload, 0: off)")
    ap.add_argument("--uneven", choices=("auto", "on", "off"), default="auto",
                    help="time the seeded uneven batch sequence through one plan (auto: on for the batching "
                         "workload's default plan)")
    ap.add_argument("--sweep", action="store_true",
                    help="also time every (P, C) of {1,2,4,8,16,32} x {k, 2k, 20, 64, 100, 200} as a tuned plan and "
                         "report the fastest with Recall@10 >= 0.95 on the recall sample (operating point)")
    ap.add_argument("--append-rows", type=int, default=0,
                    help="after the search timing, time hntl_index_append of this many new rows of the workload")
    ap.add_argument("--split-max", type=int, default=0, help="split_max of the timed append (0 = no splits)")
    ap.add_argument("--index-cache", default="",
                    help="directory: on a miss the built index's stored-format arrays are written there, on a "
                         "hit the index is made from them (hntl_index_create) instead of being built")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="run one plain device copy of this many GiB first (calibrates HBM counters)")
    return ap.parse_args()


def time_plan(hntl, torch, ix, Q, P, C, k, nq, codes, flags, rkw, steps, warmup, sched_arg=""):
    """Autotune (or take) a schedule, build a graph plan for nq queries and time
    `steps` replays; returns the plan, its ids / dist outputs and the timings."""
    stream = torch.cuda.current_stream()
    t0 = time.time()
    if sched_arg:
        sched = {kk: int(v) for kk, v in (kv.split("=") for kv in sched_arg.split(","))}
        sched = hntl.sched_dict(hntl._sched(dict({"grid": 0, "passes": 1, "proj": 0}, **sched)))
    else:
        sched, _ = hntl.hntl_tune(ix, Q, P, C, k, codes=codes, flags=flags, **rkw)
    tune_s = time.time() - t0
    plan = hntl.hntl_plan_create(ix, P, C, k, nq, codes=codes, flags=flags, sched=sched, graph=True, **rkw)
    ids = torch.empty((nq, k), dtype=torch.int32, device=Q.device)
    dist = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
    for _ in range(warmup):
        hntl.hntl_plan_search(plan, Q, out=(ids, dist))
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        hntl.hntl_plan_search(plan, Q, out=(ids, dist))
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    stage, scored = hntl.hntl_plan_profile(plan, nq, reps=3)
    stage = {("scan" if kk == "fused" else kk): v for kk, v in stage.items()}
    if not sched["proj"]:  # the projection runs inside the fused kernel: no stage of its own
        stage.pop("project")
    assert hntl.hntl_plan_info_get(plan)["wait_errors"] == 0
    return dict(plan=plan, ids=ids, dist=dist, ms=ms, stage=stage, scored=scored, sched=sched, tune_s=tune_s)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the search path runs on a single MI355X; sharding across GPUs is described, not built).",
              file=sys.stderr)
        sys.exit(2)
    from workloads import WORKLOADS
    W = WORKLOADS[args.workload]
    batching = W.name == "zipf10M_d768_G8192_r48"
    headline_plain = args.form == "plan" and args.route == "centroid" and args.codes == "fp32" and args.mode == "B"
    compare = args.compare == "on" or (args.compare == "auto" and batching and headline_plain)
    uneven = args.uneven == "on" or (args.uneven == "auto" and batching and headline_plain)
    hbm_batch = (256 if batching and args.form == "plan" else 0) if args.hbm_batch < 0 else args.hbm_batch

    t0 = time.time()
    corpus = W.corpus()
    queries = W.queries()
    log(f"[bench] generated {W.N}x{W.d} corpus + {W.nq} queries in {time.time() - t0:.1f}s")
    pool = None
    if args.cpu_sample != 0:  # forked now, before the GPU is touched
        pool, ncores = start_cpu_pool(corpus.X, queries.X)
        log(f"[bench] CPU oracle pool: {ncores} worker processes ({cpu_model()})")

    import torch
    from paper_2606_08813_amd import hntl

    if args.copy_gib > 0:  # a copy of known size: n bytes read, n bytes written
        n = int(args.copy_gib * (1 << 30)) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)  # one elementwise kernel: n bytes read, n bytes written
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {n * 4} bytes")
        del src, dst
        torch.cuda.empty_cache()
    dev = torch.device("cuda:0")
    X = torch.from_numpy(corpus.X).to(dev)
    Q = torch.from_numpy(queries.X).to(dev)
    torch.cuda.synchronize()

    t0 = time.time()
    codes_list = ["fp32"] + ([args.codes] if args.codes != "fp32" else []) + (["bf16"] if compare else [])
    codes_list = list(dict.fromkeys(codes_list))
    cache = Path(args.index_cache) / W.name if args.index_cache else None
    stored_names = ("centroids", "basis", "offsets", "perm", "codes", "eps")
    if cache is not None and all((cache / f"{nm}.npy").exists() for nm in stored_names):
        stored = {nm: np.load(cache / f"{nm}.npy") for nm in stored_names}
        ix = hntl.hntl_index_create(stored, X, codes=tuple(codes_list))
        del stored
        torch.cuda.synchronize()
        build_s = None
        info = hntl.hntl_index_info_get(ix)
        log(f"[bench] index made from the stored arrays in {cache} in {time.time() - t0:.1f}s")
    else:
        ix = hntl.hntl_build(X, W.G, W.r, seed=W.kmeans_seed, codes=tuple(codes_list))
        torch.cuda.synchronize()
        build_s = time.time() - t0
        info = hntl.hntl_index_info_get(ix)
        log(f"[bench] build {build_s:.1f}s, captured variance {info['captured_variance']:.4f}, "
            f"k-means iters {info['kmeans_iters_run']}, max grain {info['max_grain']}")
        if cache is not None:
            cache.mkdir(parents=True, exist_ok=True)
            for nm, a in hntl.hntl_index_export(ix).items():
                np.save(cache / f"{nm}.npy", a)
            log(f"[bench] stored arrays written to {cache}")
    del X
    torch.cuda.empty_cache()

    stream = torch.cuda.current_stream()
    P = args.P or W.P
    router = None
    if args.route == "learned" or compare:
        from workloads.configs import ROUTER_TRAIN_SEED
        t0 = time.time()
        Qtr = torch.from_numpy(W.queries(nq=args.router_train, query_seed=ROUTER_TRAIN_SEED).X).to(dev)
        losses = hntl.hntl_router_train(ix, Qtr, hidden=(1024, 1024), epochs=args.router_epochs, batch=1024, knn=10,
                                        lr=1e-3, seed=1)
        torch.cuda.synchronize()
        router = {"train_queries": args.router_train, "epochs": args.router_epochs, "hidden": [1024, 1024],
                  "train_s": round(time.time() - t0, 1), "epoch_loss": [round(float(x), 4) for x in losses],
                  "tau": args.tau}
        log(f"[bench] router trained in {router['train_s']}s, losses {router['epoch_loss']}")
        del Qtr
    flags = 0 if args.no_profile else hntl.HNTL_FLAG_PROFILE
    if args.no_prune:
        flags |= hntl.HNTL_FLAG_NO_PRUNE
    bf16_project = args.codes in ("bf16", "fp8") and not args.fp32_project
    if bf16_project:
        flags |= hntl.HNTL_FLAG_PROJECT_BF16
    route_form = None
    if args.route == "centroid":
        route_form = args.route_form if args.route_form != "auto" else ("bf16" if W.d % 8 == 0 else "fp32")
        flags |= {"fp32": 0, "bf16": hntl.HNTL_FLAG_ROUTE_BF16, "bf16x3": hntl.HNTL_FLAG_ROUTE_BF16X3}[route_form]
    if args.mode == "A":
        flags |= hntl.HNTL_FLAG_MODE_A
    rkw = dict(route=args.route, tau=args.tau, mass=args.mass)
    plan_mask = (hntl.HNTL_FLAG_PROJECT_BF16 | hntl.HNTL_FLAG_NO_PRUNE | hntl.HNTL_FLAG_ROUTE_BF16X3 |
                 hntl.HNTL_FLAG_ROUTE_BF16 | hntl.HNTL_FLAG_MODE_A)
    pflags = flags & plan_mask
    sched = None
    if args.form == "staged":
        ids = torch.empty((W.nq, W.k), dtype=torch.int32, device=dev)
        dist = torch.empty((W.nq, W.k), dtype=torch.float32, device=dev)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        for _ in range(args.warmup):
            hntl.hntl_search(ix, Q, P, W.C, W.k, codes=args.codes, flags=flags & ~hntl.HNTL_FLAG_PROFILE,
                             out=(ids, dist), **rkw)
        torch.cuda.synchronize()
        hntl.hntl_profile_read()  # drop warm-up records
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            hntl.hntl_search(ix, Q, P, W.C, W.k, codes=args.codes, flags=flags, out=(ids, dist), **rkw)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_per_step = ev0.elapsed_time(ev1) / args.steps
        stage_ms, calls, scored_total = hntl.hntl_profile_read()
        stage_avg = {kk: v / max(1, calls) for kk, v in stage_ms.items()}
        scored = scored_total // max(1, calls)  # eq. 6 scores actually computed per step
    else:
        r = time_plan(hntl, torch, ix, Q, P, W.C, W.k, W.nq, args.codes, pflags, rkw, args.steps, args.warmup,
                      args.sched)
        ids, dist, ms_per_step, stage_avg, scored, sched = r["ids"], r["dist"], r["ms"], r["stage"], r["scored"], r["sched"]
        log(f"[bench] schedule {sched} (tuning {r['tune_s']:.1f}s)")
        del r
    qps = W.nq / (ms_per_step / 1e3)
    log(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step, {qps:,.0f} queries/s; stages {stage_avg}")

    # work accounting from one staged run (probes -> vectors in the probed grains per step)
    o = hntl.hntl_search_stages(ix, Q, P, W.C, W.k, codes=args.codes,
                                flags=hntl.HNTL_FLAG_SYNC | (flags & plan_mask & ~hntl.HNTL_FLAG_NO_PRUNE), **rkw)
    probes = o["probes"].cpu().numpy()
    ex = hntl.hntl_index_export(ix)
    sizes = np.diff(ex["offsets"])
    scanned = int(sizes[probes[probes >= 0]].sum())
    ids_h = ids.cpu().numpy()

    # Recall@10 against exact brute force on a query sample
    rs = np.random.default_rng(7).choice(W.nq, size=min(args.recall_sample, W.nq), replace=False)
    t0 = time.time()
    gt = exact_knn(corpus.X, queries.X[rs], W.k)
    recall = recall_at_k(ids_h[rs], gt, W.k)
    log(f"[bench] Recall@10 on {len(rs)} sampled queries: {recall:.4f} (brute force {time.time() - t0:.1f}s)")

    # reduced-precision error report against FP64 (eq. 6 scores of the GPU's pool
    # entries from the stored FP32 index in float64, and final distances)
    precision = None
    if args.codes != "fp32" and args.error_sample > 0:
        es = np.random.default_rng(13).choice(W.nq, size=min(args.error_sample, W.nq), replace=False)
        probes_s = probes[es]
        pool_ids = o["pool_ids"].cpu().numpy()[es]
        pool_D = o["pool_D"].cpu().numpy()[es].astype(np.float64)
        rel = []
        for i in range(len(es)):
            m = {}
            for sl in range(P):
                if probes_s[i, sl] >= 0:
                    gi, gd = fp64_grain_scores(queries.X[es[i]], int(probes_s[i, sl]), ex)
                    m.update(zip(gi.tolist(), gd.tolist()))
            for pid, pd in zip(pool_ids[i], pool_D[i]):
                if pid >= 0:
                    ref = m[int(pid)]
                    rel.append(abs(pd - ref) / max(ref, 1e-12))
        rel = np.array(rel)
        fd = dist.cpu().numpy()[es].astype(np.float64)
        fi = ids_h[es]
        exact = ((corpus.X[fi].astype(np.float64) - queries.X[es][:, None, :].astype(np.float64)) ** 2).sum(-1)
        frel = np.abs(fd - exact) / np.maximum(exact, 1e-12)
        precision = {"codes": args.codes, "projection": "bf16" if bf16_project else "fp32",
                     "sample_queries": len(es),
                     "scan_score_rel_err_vs_fp64": {"median": float(np.median(rel)), "p99": float(np.quantile(rel, 0.99)),
                                                    "max": float(rel.max())},
                     "final_dist_rel_err_vs_fp64": {"median": float(np.median(frel)), "max": float(frel.max())}}
        log(f"[bench] precision report: {precision}")

    # rooflines per stage (algorithmic work per launch / average stage time)
    npairs = W.nq * P
    rp = (W.r + 7) // 8 * 8
    code_bytes = {"fp32": 4, "bf16": 2, "fp8": 1, "int16": 2}[args.codes]
    route_work = (2.0 * W.nq * (W.d * 1024 + 1024 * 1024 + 1024 * W.G) if args.route == "learned"
                  else 2.0 * W.nq * W.G * W.d * (3 if route_form == "bf16x3" else 1))
    route_bf16 = args.route == "learned" or route_form in ("bf16", "bf16x3")
    per_stage = {
        "route": dict(bound="mfma", work=route_work, unit="TFLOP/s",
                      peak=BF16_MFMA_PEAK_TFLOPS if route_bf16 else FP32_MFMA_PEAK_TFLOPS),
        "project": dict(bound="mfma", work=2.0 * npairs * W.r * W.d, unit="TFLOP/s",
                        peak=BF16_MFMA_PEAK_TFLOPS if bf16_project else FP32_MFMA_PEAK_TFLOPS),
        "scan": dict(bound="alu", work=3.0 * W.r * (scored or scanned), unit="TFLOP/s", peak=FP32_VALU_PEAK_TFLOPS),
        "rerank": dict(bound="hbm", work=(float(W.nq) * W.C * W.d * 4 if args.mode == "B" else W.nq * W.C * 4.0)
                       + W.nq * P * W.C * 8, unit="GB/s", peak=HBM_PEAK_GBS),
    }
    roof = {}
    for name, s in per_stage.items():
        t = stage_avg.get(name, 0.0) / 1e3
        if t <= 0:
            continue
        achieved = s["work"] / t / (1e12 if s["unit"] == "TFLOP/s" else 1e9)
        roof[name] = {"bound": s["bound"], "achieved": round(achieved, 3), "peak": s["peak"], "unit": s["unit"],
                      "frac": round(achieved / s["peak"], 4), "ms": round(stage_avg[name], 4)}
        tr = measured_traffic(name, W.name, args.form, args.codes if name != "project" else
                              ("bf16" if bf16_project else "fp32"), P, args.mode, W.nq, sched)
        if tr:  # the stage's DRAM bytes from counters on this kernel source
            roof[name]["traffic"] = tr
            roof[name]["dram_GBps"] = round(tr / t / 1e9, 1)
    dominant = max(roof, key=lambda n: roof[n]["ms"]) if roof else None
    scan_ms = stage_avg.get("scan", 0.0)

    # the scan in its HBM-bound regime: a small batch whose probed grains' codes
    # exceed the MALL, each probed grain's code blocks read once per pair tile
    scan_hbm = None
    if hbm_batch > 0 and args.form == "plan":
        nb = min(hbm_batch, W.nq)
        Qh = Q[:nb].contiguous()
        rh = time_plan(hntl, torch, ix, Qh, P, W.C, W.k, nb, args.codes, pflags, rkw, args.steps, 2, args.hbm_sched)
        ph = hntl.hntl_search_stages(ix, Qh, P, W.C, W.k, codes=args.codes,
                                     flags=hntl.HNTL_FLAG_SYNC | (pflags & ~hntl.HNTL_FLAG_NO_PRUNE), **rkw)["probes"]
        pg = np.unique(ph.cpu().numpy())
        pg = pg[pg >= 0]
        nblk = (sizes[pg] + 63) // 64
        unique_bytes = int(nblk.sum()) * 64 * (rp * code_bytes + 4)
        t_scan = rh["stage"]["scan"]
        traffic = measured_traffic("scan", W.name, "plan", args.codes, P, args.mode, nb, rh["sched"])
        scan_hbm = {"batch": nb, "schedule": rh["sched"], "scan_ms": round(t_scan, 4),
                    "probed_grains": int(len(pg)), "unique_code_bytes": unique_bytes,
                    "scored": int(rh["scored"]),
                    "achieved_GBps": round(unique_bytes / (t_scan / 1e3) / 1e9, 1),
                    "peak_GBps": HBM_PEAK_GBS,
                    "frac": round(unique_bytes / (t_scan / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                    "dram_traffic": traffic,
                    "dram_GBps": round(traffic / (t_scan / 1e3) / 1e9, 1) if traffic else None,
                    "ms_per_batch": round(rh["ms"], 4)}
        log(f"[bench] scan HBM regime ({nb} queries): {scan_hbm}")
        del rh

    # the seeded uneven batch sequence through one plan (graph replays)
    uneven_out = None
    if uneven and args.form == "plan":
        seq = uneven_batch_sizes(65536, seed=W.seed)
        Qu = torch.from_numpy(W.queries(nq=W.nq, query_seed=W.seed + 5000).X).to(dev)
        ru = time_plan(hntl, torch, ix, Qu, P, W.C, W.k, W.nq, args.codes, pflags, rkw, 1, 1, args.sched)
        plan_u = ru["plan"]
        views = [Qu[:nbq].contiguous() for nbq in seq]
        for v in views[:3]:
            hntl.hntl_plan_search(plan_u, v)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for v in views:
            hntl.hntl_plan_search(plan_u, v)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_u = ev0.elapsed_time(ev1)
        uneven_out = {"batches": len(seq), "queries": int(sum(seq)), "min_batch": int(min(seq)),
                      "max_batch": int(max(seq)), "seed": W.seed, "ms": round(ms_u, 3),
                      "queries_per_s": round(sum(seq) / (ms_u / 1e3), 1), "schedule": ru["sched"]}
        log(f"[bench] uneven batches: {uneven_out}")
        del ru, plan_u, Qu, views

    # the learned router + BF16 codes + BF16 projection at the same P and C,
    # and centroid routing with the same BF16 codes and projection (what the
    # precision form gives without the router)
    learned = None
    centroid_bf16 = None
    if compare:
        fl_l = hntl.HNTL_FLAG_PROJECT_BF16
        fl_c = fl_l | (pflags & (hntl.HNTL_FLAG_ROUTE_BF16 | hntl.HNTL_FLAG_ROUTE_BF16X3))  # the headline's shortlist
        rc = time_plan(hntl, torch, ix, Q, P, W.C, W.k, W.nq, "bf16", fl_c, {}, args.steps, args.warmup)
        rec_c = recall_at_k(rc["ids"].cpu().numpy()[rs], gt, W.k)
        centroid_bf16 = {"form": "plan", "route": "centroid", "codes": "bf16", "projection": "bf16", "P": P,
                         "C": W.C, "value": round(W.nq / (rc["ms"] / 1e3), 1), "ms_per_step": round(rc["ms"], 4),
                         "recall_at_10": round(rec_c, 4),
                         "stage_ms": {kk: round(v, 4) for kk, v in rc["stage"].items()}, "schedule": rc["sched"],
                         "speedup_vs_plain_fp32": round(ms_per_step / rc["ms"], 4)}
        log(f"[bench] centroid + BF16: {centroid_bf16}")
        del rc
        rl = time_plan(hntl, torch, ix, Q, P, W.C, W.k, W.nq, "bf16", fl_l, dict(route="learned", tau=args.tau),
                       args.steps, args.warmup)
        rec_l = recall_at_k(rl["ids"].cpu().numpy()[rs], gt, W.k)
        learned = {"form": "plan", "route": "learned", "codes": "bf16", "projection": "bf16", "P": P, "C": W.C,
                   "value": round(W.nq / (rl["ms"] / 1e3), 1), "ms_per_step": round(rl["ms"], 4),
                   "recall_at_10": round(rec_l, 4), "stage_ms": {kk: round(v, 4) for kk, v in rl["stage"].items()},
                   "schedule": rl["sched"], "speedup_vs_plain_fp32": round(ms_per_step / rl["ms"], 4),
                   "vectors_scored_per_step": int(rl["scored"])}
        log(f"[bench] learned + BF16: {learned}")
        del rl
        if args.compare_mass > 0:
            # the same with the router's probability-mass probe budget
            mkw = dict(route="learned", tau=args.tau, mass=args.compare_mass)
            rm = time_plan(hntl, torch, ix, Q, P, W.C, W.k, W.nq, "bf16", fl_l, mkw, args.steps, args.warmup)
            rec_m = recall_at_k(rm["ids"].cpu().numpy()[rs], gt, W.k)
            pm = hntl.hntl_search_stages(ix, Q, P, W.C, W.k, codes="bf16", flags=hntl.HNTL_FLAG_SYNC | fl_l,
                                         **mkw)["probes"]
            learned["probe_budget"] = {
                "mass": args.compare_mass, "value": round(W.nq / (rm["ms"] / 1e3), 1),
                "ms_per_step": round(rm["ms"], 4), "recall_at_10": round(rec_m, 4),
                "mean_probes_per_query": round(float((pm >= 0).sum().item()) / W.nq, 3),
                "stage_ms": {kk: round(v, 4) for kk, v in rm["stage"].items()}, "schedule": rm["sched"],
                "speedup_vs_plain_fp32": round(ms_per_step / rm["ms"], 4)}
            log(f"[bench] learned + BF16 + probe budget: {learned['probe_budget']}")
            del rm, pm

    # CPU oracle over the process pool, on the same index (timing only)
    cpu = None
    if pool is not None:
        cpu = run_cpu_baseline(pool, ncores, ex, W.nq, P, W.C, W.k, args.mode, args.cpu_seconds, scanned / W.nq)
        log(f"[bench] CPU oracle: {cpu['value']} queries/s on {cpu['cores']} processes")

    # operating point: the fastest (P, C) of the grid at Recall@10 >= 0.95 (plans, tuned per point)
    sweep = None
    if args.sweep and args.form == "plan":
        pts = []
        for Ps in (1, 2, 4, 8, 16, 32):
            if Ps > W.G:
                continue
            for Cs in sorted({W.k, 2 * W.k, 20, 64, 100, 200}):
                if Cs < W.k:
                    continue
                rr = time_plan(hntl, torch, ix, Q, Ps, Cs, W.k, W.nq, args.codes, pflags, rkw,
                               max(3, args.steps // 2), 2)
                rec = recall_at_k(rr["ids"].cpu().numpy()[rs], gt, W.k)
                pts.append({"P": Ps, "C": Cs, "queries_per_s": round(W.nq / (rr["ms"] / 1e3), 1),
                            "recall_at_10": round(rec, 4)})
                log(f"[bench] sweep P={Ps} C={Cs}: {pts[-1]['queries_per_s']:,.0f} q/s, Recall@10 {rec:.4f}")
                del rr
        ok = [p for p in pts if p["recall_at_10"] >= 0.95]
        best = max(ok, key=lambda p: p["queries_per_s"]) if ok else None
        sweep = {"grid": pts, "operating_point": best, "recall_sample": int(len(rs))}
        log(f"[bench] operating point {best}")

    # incremental segment: a new index = this one plus appended rows (build side, timed separately)
    append = None
    if args.append_rows > 0:
        Xa = torch.from_numpy(W.queries(nq=args.append_rows, query_seed=4242).X).to(dev)
        times = []
        for _ in range(2):  # the first call also loads the append's code objects
            torch.cuda.synchronize()
            t0 = time.time()
            ix2 = hntl.hntl_index_append(ix, Xa, split_max=args.split_max, seed=1)
            torch.cuda.synchronize()
            times.append(time.time() - t0)
            G2 = ix2.G
            del ix2
            torch.cuda.empty_cache()
        t = min(times)
        append = {"rows": args.append_rows, "base_rows": W.N, "split_max": args.split_max, "grains_after": G2,
                  "seconds": round(t, 4), "rows_per_s": round(args.append_rows / t, 1)}
        log(f"[bench] append of {args.append_rows} rows: {t * 1e3:.1f} ms, {G2 - W.G} new grains")
        del Xa

    out = {
        "metric": METRIC,
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp8": "fp8", "int16": "i16"}[args.codes],
        "data": "synthetic",
        "config": {"workload": W.name, "N": W.N, "d": W.d, "G": W.G, "r": W.r, "queries_per_step": W.nq,
                   "P": P, "C": W.C, "k": W.k, "codes": args.codes,
                   "projection": "bf16" if bf16_project else "fp32", "form": args.form, "route": args.route,
                   "route_shortlist": route_form, "mode": args.mode, "schedule": sched},
        "recall_at_10": round(recall, 4),
        # per vector actually scored (exact pruning skips most members of non-nearest grains)
        "scan_ns_per_vector_scored": round(scan_ms * 1e6 / scored, 6) if (scan_ms and scored) else None,
        "ns_per_vector_scored": round(ms_per_step * 1e6 / scored, 6) if scored else None,
        "ns_per_vector_scanned": round(ms_per_step * 1e6 / scanned, 6),
        "vectors_scored_per_step": scored,
        "vectors_in_probed_grains_per_step": scanned,
        "prune": not args.no_prune,
        "stage_ms": {kk: round(v, 4) for kk, v in stage_avg.items()},
        "build_s": None if build_s is None else round(build_s, 2),
        "captured_variance": round(info["captured_variance"], 5),
        "roofline": dict(roof.get(dominant, {}), kernel=dominant,
                         traffic=measured_traffic(dominant, W.name, args.form, args.codes, P, args.mode, W.nq,
                                                  sched))
        if dominant else None,
        "stage_rooflines": roof,
        "scan_hbm": scan_hbm,
        "centroid_bf16": centroid_bf16,
        "learned_bf16": learned,
        "uneven_batches": uneven_out,
        "cpu_baseline": cpu,
        "precision": precision,
        "router": router,
    }
    if append is not None:
        out["append"] = append
    if sweep is not None:
        out["sweep"] = sweep
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
