"""Pins of the target-association oracle (Algorithm 3 with side preference) on cases
whose answer is fixed by hand: inclusive danger and center radii on exactly representable
distances, the tolerance widening a center ball, the closest-center rule and its tie
break, side preference, and the empty cases; then, on a discretized surface, properties
that hold for any correct association (every base node is reached from its own side, far
points are never endangered, the chosen center is admissible and no admissible center is
closer)."""

import numpy as np

from oracle.association import FAR, UNMATCHED, associate_targets
from workloads import workload_tiny

O3 = np.zeros((1, 3))


def test_danger_zone_is_inclusive():
    src = O3
    tg = np.array([[0.5, 0, 0], [1.0, 0, 0], [1.0 + 2.0 ** -40, 0, 0], [0, 0, -1.0]])
    got = associate_targets(src, [1.0], np.zeros((0, 3)), [], tg)
    assert got.tolist() == [UNMATCHED, UNMATCHED, FAR, UNMATCHED]


def test_closest_center_tie_and_tolerance():
    src = O3
    ctr = np.array([[0.5, 0, 0], [-0.25, 0, 0], [0.0, 0.5, 0]])
    rad = [0.5, 0.5, 0.5]
    tg = np.array([[0.25, 0, 0],     # 0.25 from c0, 0.5 from c1: c0
                   [0.0, 0, 0],      # 0.5 from c0 and c2, 0.25 from c1: c1
                   [0.25, 0.25, 0],  # equidistant from c0 and c2 (sqrt(1/8)): lower index
                   [1.0625, 0, 0]])  # 0.5625 from c0: outside r, inside r (1 + 1/8)
    got = associate_targets(src, [2.0], ctr, rad, tg)
    assert got.tolist() == [0, 1, 0, UNMATCHED]
    got = associate_targets(src, [2.0], ctr, rad, tg, tol=0.125)
    assert got.tolist() == [0, 1, 0, 0]


def test_side_preference():
    src = O3
    ctr = np.array([[0.1, 0, 0], [-0.5, 0, 0]])
    side = np.array([1, -1], dtype=np.int8)
    tg = np.array([[0.0, 0, 0]] * 3)
    tside = np.array([0, -1, 1], dtype=np.int8)
    got = associate_targets(src, [1.0], ctr, [1.0, 1.0], tg, ctr_side=side, tgt_side=tside)
    assert got.tolist() == [0, 1, 0]
    tside = np.array([-1, -1, -1], dtype=np.int8)
    got = associate_targets(src, [1.0], ctr, [1.0, 0.25], tg, ctr_side=side, tgt_side=tside)
    assert got.tolist() == [UNMATCHED] * 3


def test_empty_inputs():
    tg = np.array([[0.0, 0, 0], [5.0, 0, 0]])
    assert associate_targets(np.zeros((0, 3)), [], O3, [1.0], tg).tolist() == [FAR, FAR]
    assert associate_targets(O3, [1.0], O3, [1.0], np.zeros((0, 3))).shape == (0,)


def _admissible(t, c, r, tol):
    d = t - c
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2] <= (r * (1.0 + tol)) ** 2


def test_surface_properties():
    w = workload_tiny(level=2, order=2, kernel="S", nmax=32)
    rng = np.random.default_rng(3)
    nodes = w.src_xyz
    # base nodes from each side (their own center lies at distance r)
    tg = np.concatenate([nodes, nodes, 3.0 * np.ones((4, 3)),
                         rng.uniform(-1.3, 1.3, (400, 3))])
    side = np.concatenate([np.ones(len(nodes)), -np.ones(len(nodes)), np.zeros(404)]).astype(np.int8)
    tol = 1e-9
    got = associate_targets(w.src_xyz, w.src_radius, w.ctr_xyz, w.ctr_radius, tg, tol=tol,
                            ctr_side=w.ctr_side, tgt_side=side)
    n = len(nodes)
    assert np.all(got[:2 * n] >= 0)  # every node is endangered by itself and has a center
    assert np.all(w.ctr_side[got[:n]] == 1) and np.all(w.ctr_side[got[n:2 * n]] == -1)
    assert np.all(got[2 * n:2 * n + 4] == FAR)
    for i in np.nonzero(got >= 0)[0]:
        c = got[i]
        assert _admissible(tg[i], w.ctr_xyz[c], w.ctr_radius[c], tol)
        d = np.linalg.norm(w.ctr_xyz - tg[i], axis=1)
        ok = d <= w.ctr_radius * (1 + tol) * (1 + 1e-12)
        if side[i] != 0:
            ok &= w.ctr_side == side[i]
        assert d[c] <= d[ok].min() * (1 + 1e-12)
    # a volume point far from every source (further than the largest danger radius from
    # all of them) is never endangered; one on a node always is
    far = np.min(np.linalg.norm(tg[2 * n:, None] - nodes[None], axis=2), axis=1) > w.src_radius.max()
    assert np.all(got[2 * n:][far] == FAR)
