"""Pins of the geometry-processing oracle (stage-1 and stage-2 refinement, Section 3,
Algorithms 1 and 2) on cases whose outcome follows from the definitions by hand:

* the stretch factor of a flat equilateral triangle is its edge length, for any vertex
  order, and a midpoint child has half of its parent's;
* two concentric unit spheres 0.3 apart: a center at r from one sheet has the other sheet
  at about 0.3 - r, so Algorithm 1 must shrink r below 0.3 / (2 - eps), about 0.152
  (eta <= 0.304); a level-1 mesh (eta about 0.65-0.86) needs exactly two bisections of
  every element;
* one smooth sphere: Algorithm 1 changes nothing;
* a sphere refined on one cap: Algorithm 2 bisects the coarse elements at the fringe and
  nothing far from it;
* principal curvatures of an ellipsoid at its pole and rim (closed forms), and the scaled
  curvature of a sphere of radius 1/2, which is exactly twice the stretch factor;
and the postconditions of both algorithms, checked by a plain all-pairs test on samples.
"""

import numpy as np
import pytest

import oracle.refinement as R
from workloads import icosphere

EPS = 0.025


def sphere(P):
    return P / np.sqrt(P[..., 0] ** 2 + P[..., 1] ** 2 + P[..., 2] ** 2)[..., None]


def two_spheres(P):
    """Parameter points far out (|P| > 5) map to the sphere of radius 1.3, the rest to the
    unit sphere (piecewise constant factor, so tangents stay exact)."""
    n = np.sqrt(P[..., 0] ** 2 + P[..., 1] ** 2 + P[..., 2] ** 2)
    rad = np.where(np.real(n) > 5.0, 1.3, 1.0)
    return P / n[..., None] * rad[..., None]


def ico_elems(level, scale=1.0):
    v, f = icosphere(level)
    return [(scale * v[a], scale * v[b], scale * v[c]) for a, b, c in f]


def brute_any(q, r, p, strict):
    d = q[:, None, :] - p[None, :, :]
    d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    rr = (r * r)[:, None]
    return np.any(d2 < rr if strict else d2 <= rr, axis=1)


def test_stretch_factor_of_flat_triangles():
    flat = lambda P: P  # noqa: E731
    A, B, C = np.array([0.0, 0, 0]), np.array([2.0, 0, 0]), np.array([1.0, np.sqrt(3.0), 0])
    for tri in [(A, B, C), (B, C, A), (C, A, B)]:
        assert R.stretch(flat, *tri, 4) == pytest.approx(2.0, rel=1e-14)
    kids = R.bisect([(A, B, C)], [True])
    assert len(kids) == 4
    for k in kids:
        assert R.stretch(flat, *k, 4) == pytest.approx(1.0, rel=1e-14)
    # a stretched triangle: eta follows the longest direction of the map
    S = np.diag([3.0, 1.0, 1.0])
    assert R.stretch(lambda P: P @ S.T, A, B, C, 2) == pytest.approx(6.0, rel=1e-14)


def test_stage1_two_concentric_spheres():
    elems = ico_elems(1) + ico_elems(1, scale=10.0)
    eta0 = np.array([R.stretch(two_spheres, *e, 4) for e in elems])
    assert eta0.min() > 0.6 and eta0.max() < 0.9
    out, rounds = R.stage1(two_spheres, elems, 4, eps=EPS, kappa_max=None)
    eta = np.array([R.stretch(two_spheres, *e, 4) for e in out])
    bound = 2 * 0.3 / (2 - EPS)
    assert rounds == 2 and len(out) == 16 * len(elems)
    assert eta.max() < bound and eta.min() > bound / 2
    # postcondition on a sample of centers, by all pairs
    xyz, elem, r, c = R._centers(two_spheres, out, 4)
    pick = np.random.default_rng(0).choice(c.shape[0], 1500, replace=False)
    assert not brute_any(c[pick], (1 - EPS) * r[pick], xyz, strict=True).any()


def test_stage1_leaves_a_smooth_sphere_alone():
    elems = ico_elems(2)  # eta <= 0.45: scaled curvature below 0.8 as well
    out, rounds = R.stage1(sphere, elems, 4, eps=EPS)
    assert rounds == 0 and len(out) == len(elems)


def test_stage2_refines_the_fringe_of_a_refined_cap():
    elems = ico_elems(1)
    top = [np.mean([e[0][2], e[1][2], e[2][2]]) > 0 for e in elems]
    elems = R.bisect(elems, top)
    cap = [np.mean([e[0][2], e[1][2], e[2][2]]) > 0.2 for e in elems]
    elems = R.bisect(elems, cap)
    el1, r1 = R.stage1(sphere, elems, 4, eps=EPS, kappa_max=None)
    assert r1 == 0 and len(el1) == len(elems)
    el2, r2 = R.stage2(sphere, el1, 4)
    assert r2 >= 1 and len(el2) > len(el1)
    # far from the cap (z < -0.5) nothing changes; every stage-2 element lies in a stage-1 one
    low1 = sorted(tuple(np.round(np.concatenate(e), 12)) for e in el1 if max(e[0][2], e[1][2], e[2][2]) < -0.5)
    low2 = sorted(tuple(np.round(np.concatenate(e), 12)) for e in el2 if max(e[0][2], e[1][2], e[2][2]) < -0.5)
    assert low1 == low2
    # postcondition by all pairs on a sample of stage-2 nodes
    _, _, _, ctr = R._centers(sphere, el1, 4)
    xyz, _, elem = R.nodes(sphere, el2, 4)
    eta = np.array([R.stretch(sphere, *e, 4) for e in el2])
    pick = np.random.default_rng(1).choice(xyz.shape[0], 2000, replace=False)
    assert not brute_any(xyz[pick], 0.375 * eta[elem[pick]], ctr, strict=False).any()


def _ref_point(A, B, C, P):
    """Reference coordinates (x, y) of the parameter point P on the element's plane."""
    M = np.stack([B - A, C - B], axis=1)
    xy, *_ = np.linalg.lstsq(M, P - A, rcond=None)
    return xy


def test_principal_curvatures_of_an_ellipsoid():
    """Semi-axes (1, 1, c): at the pole both principal curvatures are c; at the rim they
    are 1/c^2 (across) and 1 (along); outward normals make them negative."""
    c = 0.3
    ell = lambda P: sphere(P) * np.array([1.0, 1.0, c])  # noqa: E731
    A, B, C = np.array([0.1, 0.0, 1.0]), np.array([-0.05, 0.087, 1.0]), np.array([-0.05, -0.087, 1.0])
    x, y = _ref_point(A, B, C, np.array([0.0, 0.0, 1.0]))
    k = R.principal_curvatures(ell, A, B, C, [x], [y])[0]
    assert np.allclose(k, [-c, -c], rtol=1e-7)
    A, B, C = np.array([1.0, 0.1, 0.0]), np.array([1.0, -0.05, 0.087]), np.array([1.0, -0.05, -0.087])
    x, y = _ref_point(A, B, C, np.array([1.0, 0.0, 0.0]))
    k = R.principal_curvatures(ell, A, B, C, [x], [y])[0]
    assert np.allclose(k, [-1.0 / c ** 2, -1.0], rtol=1e-7)


def test_scaled_curvature_of_a_sphere_and_its_refinement():
    """On a sphere of radius 1/2 the principal curvatures are 2, so kappa = 2 eta.  The
    criterion is scale-free: the icosahedron's elements (kappa about 1.3) all exceed 0.8
    and one bisection brings every element below it."""
    half = lambda P: 0.5 * sphere(P)  # noqa: E731
    for e in ico_elems(1)[:5]:
        assert R.scaled_curvature(half, *e, 4) == pytest.approx(2.0 * R.stretch(half, *e, 4), rel=1e-7)
    elems = ico_elems(0)
    kap = np.array([R.scaled_curvature(half, *e, 4) for e in elems])
    assert kap.min() > 0.8
    out, rounds = R.stage1(half, elems, 4, eps=EPS, kappa_max=0.8)
    assert rounds == 1 and len(out) == 4 * len(elems)
    assert max(R.scaled_curvature(half, *e, 4) for e in out) <= 0.8
