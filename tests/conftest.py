import hashlib
import os
import sys
from pathlib import Path

import numpy as np
import pytest

ROOT = Path(__file__).resolve().parents[1]
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))

CACHE = ROOT / "tests" / ".cache"


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def _oracle_hash():
    h = hashlib.sha1()
    for p in sorted((ROOT / "oracle").glob("*.py")) + sorted((ROOT / "workloads").glob("*.py")):
        h.update(p.read_bytes())
    return h.hexdigest()[:12]


def cached_oracle_index(tag, build_fn):
    """Stored arrays of an oracle-built index, cached on disk keyed by the oracle source."""
    CACHE.mkdir(parents=True, exist_ok=True)
    path = CACHE / f"{tag}_{_oracle_hash()}.npz"
    if path.exists():
        with np.load(path, allow_pickle=False) as z:
            return {k: z[k] for k in z.files}
    stored = build_fn()
    tmp = path.with_suffix(".tmp.npz")
    np.savez(tmp, **stored)
    os.replace(tmp, path)
    return stored


@pytest.fixture(scope="session")
def small10k():
    """The 10k-vector patch-mixture workload: corpus, queries, oracle index, ground truth."""
    from workloads import SMALL_10K as W
    from oracle import brute, index as oi

    m = W.corpus()
    q = W.queries()

    def mk():
        idx = oi.build(m.X, W.G, W.r, W.kmeans_seed)
        st = idx.stored()
        st["captured"] = idx.captured
        return st

    stored = cached_oracle_index("small10k", mk)
    gt = cached_oracle_index("small10k_gt", lambda: dict(zip(("ids", "dist"), brute.knn(m.X, q.X, 10))))
    return dict(W=W, X=m.X, labels=m.labels, Q=q.X, stored=stored, gt_ids=gt["ids"], gt_dist=gt["dist"])
