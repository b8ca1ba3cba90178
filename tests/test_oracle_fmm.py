"""Pins for the Tier B oracle (GIGAQBX steps, own tree and lists).

* With nmax >= N the tree is one box, every source is in List 1, and Tier B must equal
  Tier A (direct QBX) to rounding.
* Partition: from any center, the near lists, the W-far subtrees, and the V subtrees and
  X-far boxes of the owner and its ancestors reach every source leaf exactly once.
* Structural consequences the paper states for Lists 3 and 4 (Section 5.2.3), the
  monotonicity of the adequate-separation relation, the bound |List 2| <= 875
  (Appendix C) and the suspended-center radius bound.
* Acceleration error vs Tier A stays below (3/4)^(p_fmm+1) (the bound column of Table 3)
  and decreases as p_fmm grows (Theorem 1).
"""

import math

import numpy as np
import pytest

import oracle as O
from oracle.gigaqbx import SQRT3, OracleFMM
from workloads import workload_tiny

pytestmark = pytest.mark.usefixtures("oracle_lib")

CASES = {
    "S-l1": dict(level=1, order=2, kernel="S", p_qbx=3, p_fmm=6, nmax=32),
    "D-l1": dict(level=1, order=2, kernel="D", p_qbx=3, p_fmm=6, nmax=32),
    "S-l2-tf05": dict(level=2, order=1, kernel="S", p_qbx=2, p_fmm=5, nmax=24, tcf=0.5),
    "D-l2-flat": dict(level=2, order=1, kernel="D", p_qbx=2, p_fmm=5, nmax=40, curved=False),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def fmm(request):
    w = workload_tiny(**CASES[request.param])
    return OracleFMM(w)


def _tier_a(w):
    pot, _ = O.direct_qbx(w.kernel, w.p_qbx, w.src_xyz, O.strengths(w)[0], w.ctr_xyz, w.tgt_xyz,
                          w.tgt_center, nrm=w.src_normal)
    return pot


def test_single_box_equals_direct():
    w = workload_tiny(level=1, order=2, kernel="D", p_qbx=4, p_fmm=4, nmax=10 ** 9)
    F = OracleFMM(w)
    assert F.tree.nboxes == 1
    tids, pot, _ = F.evaluate()
    ref = _tier_a(w)
    assert np.max(np.abs(pot - ref[tids])) <= 1e-13 * np.max(np.abs(ref))


def test_partition_every_source_leaf_once(fmm):
    for b in fmm.list_owner_boxes():
        missing, multi = fmm.partition_check(b)
        assert not missing and not multi, (b, missing, multi)


def test_every_list_exercised(fmm):
    L = fmm.lists
    tb = fmm.target_boxes()
    ob = fmm.list_owner_boxes()
    sizes = {nm: sum(len(L.get(nm, b)) for b in (tb if nm in ("U", "Wclose", "Wfar", "Xclose") else ob))
             for nm in ("U", "V", "Wclose", "Wfar", "Xclose", "Xfar")}
    assert all(v > 0 for v in sizes.values()), sizes


def test_list3_list4_structure(fmm):
    t, L = fmm.tree, fmm.lists
    for b in fmm.target_boxes():
        for d in L.W(b):
            assert t.h[d] < t.h[b]  # strictly smaller
            sep = float(np.max(np.abs(t.center[d] - t.center[b]))) - t.h[d] - t.h[b]
            assert sep >= 2 * t.h[d]  # separated by at least the width of d
    for b in fmm.list_owner_boxes():
        for d in L.X(b):
            assert t.h[d] >= t.h[b]  # at least as large as b
            sep = float(np.max(np.abs(t.center[d] - t.center[b]))) - t.h[d] - t.h[b]
            assert sep >= 2 * t.h[b]  # separated by at least the width of b
            # List entries are restricted to boxes holding sources, so b itself can only
            # appear in W(d) when its subtree has sources
            assert b in L.W(d) or d in L.T(b) or t.sub_src[b] == 0


def test_list_bounds(fmm):
    t, L = fmm.tree, fmm.lists
    for b in fmm.list_owner_boxes():
        assert len(L.V(b)) <= 875
        assert len(L.X(b)) <= 125
        assert len(L.Xclose(b)) <= 250
        assert len(L.Xfar(b)) <= 375


def test_monotonicity_of_adequate_separation(fmm):
    t = fmm.tree
    rng = np.random.default_rng(0)
    boxes = rng.choice(t.nboxes, size=min(60, t.nboxes), replace=False)
    for a in boxes:
        pa = t.parent[a]
        if pa < 0:
            continue
        for b in boxes:
            if t.prec_tcr(pa, b):
                assert t.prec_tcr(a, b)
            if t.tcr_prec(pa, b):
                assert t.tcr_prec(a, b)


def test_center_confinement(fmm):
    t, w = fmm.tree, fmm.w
    for c in range(w.n_ctr):
        b = t.ctr_owner[c]
        d = w.ctr_xyz[c] - t.center[b]
        if b != 0:
            assert np.linalg.norm(d) + w.ctr_radius[c] <= SQRT3 * t.h[b] * (1 + t.tcf) * (1 + 1e-15)
        if not t.is_leaf[b]:
            # a suspended center could not fit its child: r_c > sqrt(3)|b| t_f / 2
            assert w.ctr_radius[c] > SQRT3 * t.h[b] * t.tcf / 2


@pytest.mark.parametrize("kernel", ["S", "D"])
def test_acceleration_error_bound_and_decay(kernel):
    w = workload_tiny(level=1, order=2, kernel=kernel, p_qbx=3, p_fmm=6, nmax=32)
    ref = _tier_a(w)
    errs = []
    for p in (3, 6, 10, 14):
        F = OracleFMM(w, p_fmm=p)
        tids, pot, _ = F.evaluate()
        e = np.max(np.abs(pot - ref[tids])) / np.max(np.abs(ref))
        assert e <= 0.75 ** (p + 1)
        errs.append(e)
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs


def test_sampled_equals_full(fmm):
    """Evaluating a subset of centers gives the same numbers as the full run."""
    tids, pot, _ = fmm.evaluate()
    rng = np.random.default_rng(1)
    cs = np.sort(rng.choice(fmm.w.n_ctr, 17, replace=False))
    t2, p2, _ = fmm.evaluate(centers=cs)
    full = dict(zip(tids.tolist(), pot.tolist()))
    for t, v in zip(t2.tolist(), p2.tolist()):
        assert abs(full[t] - v) <= 1e-14 * max(1.0, abs(v))


def test_list_split_sums_to_total(fmm):
    tids, pot, _ = fmm.evaluate()
    parts = 0.0
    for nm in ("U", "V", "Wclose", "Wfar", "Xclose", "Xfar"):
        _, p1, _ = fmm.evaluate(lists=(nm,))
        parts = parts + p1
    assert np.max(np.abs(parts - pot)) <= 1e-12 * np.max(np.abs(pot))


@pytest.mark.parametrize("thr", [8, 40, 10 ** 6])
def test_remark4_partition_and_value(thr):
    """Remark 4 moves small List 3 far boxes to direct evaluation: the partition still holds
    and the result moves toward direct QBX (never away from it by more than the bound)."""
    w = workload_tiny(level=1, order=2, kernel="D", p_qbx=3, p_fmm=6, nmax=32)
    F0 = OracleFMM(w)
    F = OracleFMM(w, wfar_direct_max=thr)
    for b in F.list_owner_boxes():
        missing, multi = F.partition_check(b)
        assert not missing and not multi
    moved = sum(len(F0.lists.Wfar(b)) - len(F.lists.Wfar(b)) for b in F.target_boxes())
    assert moved > 0
    if thr >= 10 ** 6:
        assert all(len(F.lists.Wfar(b)) == 0 for b in F.target_boxes())
    ref = _tier_a(w)
    tids, pot, _ = F.evaluate()
    assert np.max(np.abs(pot - ref[tids])) / np.max(np.abs(ref)) <= 0.75 ** (w.p_fmm + 1)


# --- the l_inf target confinement region (cost comparison of Section 6) --------------------

@pytest.mark.parametrize("case", ["S-l1", "D-l2-flat", "S-l2-tf05"])
def test_linf_tcr_partition_confinement_and_accuracy(case):
    """With the box-shaped TCR the lists still reach every source leaf exactly once, every
    owned center's ball lies in its box's TCR, the box TCR sits inside the ball TCR (so
    fewer centers descend), and the result stays within the acceleration bound."""
    w = workload_tiny(**CASES[case])
    F = OracleFMM(w, tcr_norm="linf")
    t = F.tree
    for b in F.list_owner_boxes():
        missing, multi = F.partition_check(b)
        assert not missing and not multi, (b, missing, multi)
    for c in range(w.n_ctr):
        b = t.ctr_owner[c]
        if b != 0:
            d = w.ctr_xyz[c] - t.center[b]
            assert np.max(np.abs(d)) + w.ctr_radius[c] <= t.h[b] * (1 + t.tcf) * (1 + 1e-15)
            # the box TCR lies inside the ball TCR of the same box
            assert np.linalg.norm(d) + w.ctr_radius[c] <= SQRT3 * t.h[b] * (1 + t.tcf) * (1 + 1e-15)
    ref = _tier_a(w)
    tids, pot, _ = F.evaluate()
    assert np.max(np.abs(pot - ref[tids])) / np.max(np.abs(ref)) <= 0.75 ** (w.p_fmm + 1)


def test_linf_prec_tcr_is_the_box_distance():
    w = workload_tiny(**CASES["S-l1"])
    t = OracleFMM(w, tcr_norm="linf").tree
    for a in range(t.nboxes):
        for b in range(t.nboxes):
            dinf = np.max(np.abs(t.center[a] - t.center[b]))
            assert t.prec_tcr(a, b) == (dinf - t.h[b] * (1 + t.tcf) >= 3 * t.h[a])


# --- conventional targets (Algorithm 5 Stages 3, 5(b) and 9 for point targets) -------------

def _point_direct(w, tids, d=0):
    x = w.tgt_xyz[tids]
    pot, _ = O.direct_qbx(w.kernel, 0, w.src_xyz, O.strengths(w)[d], x, x,
                          np.arange(len(tids)), nrm=w.src_normal)
    return pot


@pytest.mark.parametrize("kernel", ["S", "D"])
def test_point_targets_single_box_and_accuracy(kernel):
    from workloads import add_point_targets

    w = add_point_targets(workload_tiny(level=1, order=2, kernel=kernel, p_qbx=3, p_fmm=8,
                                        nmax=10 ** 9), n_out=40, n_in=20)
    F = OracleFMM(w)
    tids, pot = F.evaluate_points()
    assert len(tids) == 60
    ref = _point_direct(w, tids)
    assert np.max(np.abs(pot - ref)) <= 1e-13 * np.max(np.abs(ref))  # one box: all direct
    w = add_point_targets(workload_tiny(level=2, order=2, kernel=kernel, p_qbx=3, p_fmm=8,
                                        nmax=24), n_out=120, n_in=60)
    F = OracleFMM(w)
    for b in F.list_owner_boxes():
        missing, multi = F.partition_check(b)
        assert not missing and not multi
    tids, pot = F.evaluate_points()
    ref = _point_direct(w, tids)
    err = np.max(np.abs(pot - ref)) / np.max(np.abs(ref))
    assert err <= 0.75 ** (w.p_fmm + 1)
    # and the QBX targets are unaffected by the extra points being in the tree
    t2, p2, _ = F.evaluate()
    assert np.all(w.tgt_center[t2] >= 0)


@pytest.mark.parametrize("case", ["S-l1", "D-l2-flat", "S-l2-tf05"])
def test_level_restriction_balance_refinement_and_accuracy(case):
    """The level-restricted tree (the remark on List 3 complexity): no two touching leaves
    differ by two or more levels unless the coarser one cannot split; it refines the plain
    tree (every plain box is still there, with the same particles below it); the lists
    still reach every source leaf exactly once; and the result stays within the
    acceleration bound.  The check of "touching" is a separate brute force over exact
    dyadic box geometry."""
    w = workload_tiny(**CASES[case])
    plain = OracleFMM(w).tree
    F = OracleFMM(w, level_restrict=True)
    t = F.tree
    assert t.nboxes > plain.nboxes  # these trees are not balanced to begin with
    keys = {t.key(b) for b in range(t.nboxes)}
    assert all(plain.key(b) in keys for b in range(plain.nboxes))
    leaves = np.nonzero(t.is_leaf)[0]
    for i in leaves:
        for j in leaves:
            if t.level[j] < t.level[i] + 2:
                continue
            gap = np.abs(t.center[i] - t.center[j]) - (t.h[i] + t.h[j])
            if np.all(gap <= 0):  # closed cubes meet: i must be unable to split
                assert len(t.own_src[i]) == 0 and len(t.own_tgt[i]) == 0, (i, j)
    for b in F.list_owner_boxes():
        missing, multi = F.partition_check(b)
        assert not missing and not multi, (b, missing, multi)
    ref = _tier_a(w)
    tids, pot, _ = F.evaluate()
    assert np.max(np.abs(pot - ref[tids])) / np.max(np.abs(ref)) <= 0.75 ** (w.p_fmm + 1)
