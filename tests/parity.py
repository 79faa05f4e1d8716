"""The parity rule between the GPU path and the oracle.

For a ranked list of length m (probes, pool or results) per query:

* tau = the oracle's m-th (last valid) distance;
* every GPU id missing from the oracle's list must have an oracle distance
  <= tau * (1 + rel);
* every oracle id missing from the GPU's list must have an oracle distance
  >= tau * (1 - rel);
* where the two lists differ at a position, the oracle distances of the two
  ids there must agree within rel (a swap of near-tied neighbours);
* every returned distance must satisfy |d_gpu - d_oracle(id)| <= dtol *
  max(d_oracle(id), floor).

rel = 1e-5 (near-tie window), dtol = 1e-4 (FP32 distance tolerance).
"""
from __future__ import annotations

import numpy as np

REL = 1e-5
DTOL = 1e-4


def check_lists(gpu_ids, gpu_d, orc_ids, orc_d, orc_dist_of, rel=REL, dtol=DTOL, floor=1e-9, what="list"):
    """orc_dist_of(row, ids) -> oracle distances of arbitrary ids for that row.

    Returns (n_rows_differing_by_near_ties, n_rows) and raises AssertionError
    with a description on the first violation."""
    gpu_ids = np.asarray(gpu_ids)
    gpu_d = np.asarray(gpu_d, dtype=np.float64)
    orc_ids = np.asarray(orc_ids)
    orc_d = np.asarray(orc_d, dtype=np.float64)
    differing = 0
    for i in range(orc_ids.shape[0]):
        ov = orc_ids[i] >= 0
        gv = gpu_ids[i] >= 0
        if ov.sum() != gv.sum():
            raise AssertionError(f"{what} row {i}: {gv.sum()} valid GPU entries vs {ov.sum()} oracle")
        if not ov.any():
            continue
        o_ids = orc_ids[i][ov]
        g_ids = gpu_ids[i][gv]
        if len(set(g_ids.tolist())) != len(g_ids):
            raise AssertionError(f"{what} row {i}: duplicate ids {g_ids}")
        tau = orc_d[i][ov][-1]
        gd_orc = np.asarray(orc_dist_of(i, g_ids), dtype=np.float64)
        fl = max(floor, 0.0)
        err = np.abs(gpu_d[i][gv] - gd_orc)
        lim = dtol * np.maximum(gd_orc, fl)
        if (err > lim).any():
            j = int(np.argmax(err - lim))
            raise AssertionError(f"{what} row {i}: distance of id {g_ids[j]} gpu {gpu_d[i][gv][j]!r} "
                                 f"oracle {gd_orc[j]!r}")
        if np.any(np.diff(gpu_d[i][gv]) < 0):
            raise AssertionError(f"{what} row {i}: GPU list not ascending")
        if np.array_equal(o_ids, g_ids):
            continue
        differing += 1
        so, sg = set(o_ids.tolist()), set(g_ids.tolist())
        for gid, gdo in zip(g_ids, gd_orc):
            if gid not in so and gdo > tau * (1 + rel) + fl:
                raise AssertionError(f"{what} row {i}: GPU id {gid} (oracle dist {gdo!r}) beyond tau {tau!r}")
        od_map = dict(zip(o_ids.tolist(), orc_d[i][ov].tolist()))
        for oid in o_ids:
            if oid not in sg and od_map[oid] < tau * (1 - rel) - fl:
                raise AssertionError(f"{what} row {i}: oracle id {oid} ({od_map[oid]!r}) missing, tau {tau!r}")
        od = orc_d[i][ov]
        for pos in np.nonzero(o_ids != g_ids)[0]:
            if abs(gd_orc[pos] - od[pos]) > rel * max(abs(od[pos]), fl) + fl:
                raise AssertionError(f"{what} row {i} pos {pos}: gpu id {g_ids[pos]} ({gd_orc[pos]!r}) vs "
                                     f"oracle id {o_ids[pos]} ({od[pos]!r})")
    return differing, orc_ids.shape[0]
