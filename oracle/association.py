"""Oracle for target association (Algorithm 3, with the side preference of Section 3).

TEST INFRASTRUCTURE ONLY: used by the tests; the library never imports it.

Brute force over all pairs, in the algorithm's order:
  1. every source s marks each target within its danger radius (|t - s| <= r_s) as
     endangered;
  2. every center c, in index order, claims each endangered target within
     r_c (1 + tol) whose side preference it meets (a target's side 0 accepts any center;
     otherwise the center's side must equal it) if it is closer than every center that
     claimed the target before, so equal distances stay with the lower index;
  3. endangered targets no center claimed are flagged.
Result per target: the center index, -1 (not endangered) or -2 (flagged).

Distances are compared squared, ((dx*dx + dy*dy) + dz*dz) <= r*r, in FP64; numpy performs
each elementwise product and sum separately, with no fused multiply-add.
"""

from __future__ import annotations

import numpy as np

FAR = -1
UNMATCHED = -2


def _d2(t, p):
    dx = t[:, None, 0] - p[None, :, 0]
    dy = t[:, None, 1] - p[None, :, 1]
    dz = t[:, None, 2] - p[None, :, 2]
    return (dx * dx + dy * dy) + dz * dz


def associate_targets(src_xyz, src_danger, ctr_xyz, ctr_radius, tgt_xyz, tol=0.0,
                      ctr_side=None, tgt_side=None, chunk=256):
    src_xyz = np.asarray(src_xyz, dtype=np.float64).reshape(-1, 3)
    ctr_xyz = np.asarray(ctr_xyz, dtype=np.float64).reshape(-1, 3)
    tgt_xyz = np.asarray(tgt_xyz, dtype=np.float64).reshape(-1, 3)
    rs = np.asarray(src_danger, dtype=np.float64)
    rs2 = rs * rs
    rc = np.asarray(ctr_radius, dtype=np.float64) * (1.0 + tol)
    rc2 = rc * rc
    nt = tgt_xyz.shape[0]
    out = np.full(nt, FAR, dtype=np.int64)
    for a in range(0, nt, chunk):
        t = tgt_xyz[a:a + chunk]
        # stage 1: endangered targets
        if src_xyz.shape[0] == 0:
            continue
        endangered = np.any(_d2(t, src_xyz) <= rs2[None, :], axis=1)
        if not np.any(endangered):
            continue
        # stage 2: the closest admissible center (first index among equals)
        rows = np.nonzero(endangered)[0]
        res = np.full(len(rows), UNMATCHED, dtype=np.int64)
        if ctr_xyz.shape[0] > 0:
            d2 = _d2(t[rows], ctr_xyz)
            ok = d2 <= rc2[None, :]
            if tgt_side is not None:
                ts = np.asarray(tgt_side)[a:a + chunk][rows]
                cs = np.asarray(ctr_side)
                ok &= (ts[:, None] == 0) | (cs[None, :] == ts[:, None])
            d2 = np.where(ok, d2, np.inf)
            best = np.argmin(d2, axis=1)  # first occurrence of the minimum
            has = np.any(ok, axis=1)
            res[has] = best[has]
        out[a + rows] = res  # stage 3: the rest stay flagged
    return out
