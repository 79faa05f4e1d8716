"""Named synthetic workloads (sizes, search parameters, seeds).

Only input shapes and seeds live here.  Seeds: data seed per workload, queries
use data seed + 1000, k-means uses data seed + 2000.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from . import patch_mixture as pm


@dataclass(frozen=True)
class Workload:
    name: str
    N: int
    d: int
    n_patches: int
    G: int
    r: int
    nq: int
    P: int
    C: int
    k: int
    seed: int
    zipf: bool = False
    byte_valued: bool = False  # SIFT1M-shaped stand-in: non-negative byte-valued components
    codes: tuple = ("fp32",)
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def query_seed(self):
        return self.seed + 1000

    @property
    def kmeans_seed(self):
        return self.seed + 2000

    def corpus(self, threads=None):
        if self.zipf:
            return pm.zipf_mixture(self.N, self.d, self.n_patches, self.seed, threads=threads)
        m = pm.uniform_mixture(self.N, self.d, self.n_patches, self.seed, threads=threads)
        return pm.byte_valued(m) if self.byte_valued else m

    def queries(self, nq=None, threads=None, query_seed=None):
        nq = self.nq if nq is None else nq
        qs = self.query_seed if query_seed is None else query_seed
        if self.zipf:
            sizes = pm.zipf_sizes(self.N, self.n_patches, 1.1, 16, 20000, self.seed)
            return pm.zipf_queries(nq, self.d, sizes, self.seed, qs, threads=threads)
        m = pm.uniform_queries(nq, self.d, self.n_patches, self.seed, qs, threads=threads)
        return pm.byte_valued(m) if self.byte_valued else m


# 10k vectors, d=768, 64 patches; G=64 grains, r=32; 1,000 queries, P=4, C=20, k=10
SMALL_10K = Workload("patch10k_d768_G64_r32", N=10_000, d=768, n_patches=64, G=64, r=32,
                     nq=1000, P=4, C=20, k=10, seed=101)

# 1M vectors, d=768, 1,024 patches; G=1,024, r=32; 10,000 queries, P=8, C=64, k=10
SCALE_1M = Workload("patch1M_d768_G1024_r32", N=1_000_000, d=768, n_patches=1024, G=1024, r=32,
                    nq=10_000, P=8, C=64, k=10, seed=102)

# same data as SCALE_1M with BF16 and FP8-e4m3 codes
PRECISION_1M = Workload("patch1M_d768_G1024_r32_bf16_fp8", N=1_000_000, d=768, n_patches=1024,
                        G=1024, r=32, nq=10_000, P=8, C=64, k=10, seed=102,
                        codes=("bf16", "fp8"))

# 10M vectors, Zipf(1.1) patch sizes 16..20,000 over 8,192 patches; G=8,192, r=48
ZIPF_10M = Workload("zipf10M_d768_G8192_r48", N=10_000_000, d=768, n_patches=8192, G=8192, r=48,
                    nq=16_384, P=16, C=100, k=10, seed=104, zipf=True)

# SIFT1M-shaped stand-in (the data set itself is not available): 1M x 128
# non-negative byte-valued vectors from 1,024 patches; G=1,024, r=16;
# 10,000 queries, P=16, C=100, k=10
SIFTLIKE_1M = Workload("siftlike1M_d128_G1024_r16", N=1_000_000, d=128, n_patches=1024, G=1024, r=16,
                       nq=10_000, P=16, C=100, k=10, seed=105, byte_valued=True)

# its small parity case: 20k x 128, 64 patches; G=64, r=16; 500 queries, P=8, C=50
SIFTLIKE_20K = Workload("siftlike20k_d128_G64_r16", N=20_000, d=128, n_patches=64, G=64, r=16,
                        nq=500, P=8, C=50, k=10, seed=106, byte_valued=True)

WORKLOADS = {w.name: w for w in (SMALL_10K, SCALE_1M, PRECISION_1M, ZIPF_10M, SIFTLIKE_1M, SIFTLIKE_20K)}

ROUTER_TRAIN_SEED = 3005
ROUTER_HELDOUT_SEED = 3006
