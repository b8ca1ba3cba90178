"""Oracle for geometry processing: stage-1 and stage-2 refinement (Section 3, Algorithms 1
and 2) by brute force.

TEST INFRASTRUCTURE ONLY: used by the tests; the library never imports it.

Independent of the library's implementation: the stretch factor is the largest singular
value from numpy's SVD of the Jacobian of the map from the bi-unit equilateral reference
triangle, the quadrature nodes are built here from Gauss-Legendre points, the proximity
tests compare all pairs, and elements are bisected into their four midpoint triangles
(which halves the stretch factor).  Distances are compared squared, ((dx*dx + dy*dy) +
dz*dz) against r*r, in FP64 (a k-d tree narrows the candidate pairs first).
"""

from __future__ import annotations

import math

import numpy as np

SQ3 = math.sqrt(3.0)
# reference equilateral triangle (edge 2) and the triangle {0 <= y <= x <= 1}
_REF = np.array([[-1.0, -1.0 / SQ3], [1.0, -1.0 / SQ3], [0.0, 2.0 / SQ3]])
_TRI = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0]])


def _equilateral_to_tri():
    """Linear part G of the affine map taking _REF's vertices to _TRI's."""
    D = np.stack([_REF[1] - _REF[0], _REF[2] - _REF[0]], axis=1)
    E = np.stack([_TRI[1] - _TRI[0], _TRI[2] - _TRI[0]], axis=1)
    return E @ np.linalg.inv(D)


def rule(order):
    """Collapsed Gauss-Legendre nodes on {0 <= y <= x <= 1}: x = u, y = u v."""
    pts, wts = [], []
    gu, wu = np.polynomial.legendre.leggauss(order + 1)
    gv, wv = np.polynomial.legendre.leggauss((order + 2) // 2)
    for a in range(order + 1):
        u = (gu[a] + 1.0) / 2.0
        for b in range((order + 2) // 2):
            v = (gv[b] + 1.0) / 2.0
            pts.append((u, u * v))
            wts.append(wu[a] / 2.0 * wv[b] / 2.0 * u)
    p = np.array(pts)
    return p[:, 0], p[:, 1], np.array(wts)


def element_geometry(surface, A, B, C, x, y):
    """Points and tangents (d/dx, d/dy) at reference points of one element."""
    P = A[None, :] + x[:, None] * (B - A)[None, :] + y[:, None] * (C - B)[None, :]
    h = 1e-30
    F = np.asarray(surface(P.astype(complex))).real
    Fx = np.asarray(surface(P + 1j * h * (B - A)[None, :])).imag / h
    Fy = np.asarray(surface(P + 1j * h * (C - B)[None, :])).imag / h
    return F, Fx, Fy


def stretch(surface, A, B, C, order):
    """eta_k = max over the element's nodes and vertices of 2 sigma_1(J G)."""
    x, y, _ = rule(order)
    x = np.concatenate([x, [0.0, 1.0, 1.0]])
    y = np.concatenate([y, [0.0, 0.0, 1.0]])
    _, Fx, Fy = element_geometry(surface, A, B, C, x, y)
    G = _equilateral_to_tri()
    best = 0.0
    for i in range(x.shape[0]):
        J = np.stack([Fx[i], Fy[i]], axis=1) @ G
        best = max(best, 2.0 * np.linalg.svd(J, compute_uv=False)[0])
    return best


def nodes(surface, elems, order):
    x, y, w = rule(order)
    xyz, nrm, elem = [], [], []
    for k, (A, B, C) in enumerate(elems):
        F, Fx, Fy = element_geometry(surface, A, B, C, x, y)
        cr = np.cross(Fx, Fy)
        xyz.append(F)
        nrm.append(cr / np.linalg.norm(cr, axis=1)[:, None])
        elem += [k] * x.shape[0]
    return np.concatenate(xyz), np.concatenate(nrm), np.array(elem)


def bisect(elems, mark):
    out = [e for e, m in zip(elems, mark) if not m]
    kids = []
    for (A, B, C), m in zip(elems, mark):
        if m:
            ab, bc, ca = (A + B) / 2.0, (B + C) / 2.0, (C + A) / 2.0
            kids.append([(A, ab, ca), (ab, B, bc), (ca, bc, C), (bc, ca, ab)])
    for j in range(4):  # children grouped by position, like the library's ordering
        out += [k[j] for k in kids]
    return out


def any_within(q, r, p, strict):
    """For each query q_i: is some p_j within r_i (< if strict, else <=)?  A k-d tree only
    lists candidates (a slightly wider ball); the exact squared comparison decides."""
    from scipy.spatial import cKDTree

    hit = np.zeros(q.shape[0], dtype=bool)
    if p.shape[0] == 0:
        return hit
    kd = cKDTree(p)
    cand = kd.query_ball_point(q, r * (1.0 + 1e-9) + 1e-300)
    for i, js in enumerate(cand):
        if not js:
            continue
        d = p[js] - q[i]
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        rr = r[i] * r[i]
        hit[i] = bool(np.any(d2 < rr if strict else d2 <= rr))
    return hit


def _centers(surface, elems, order):
    xyz, nrm, elem = nodes(surface, elems, order)
    eta = np.array([stretch(surface, *e, order) for e in elems])
    r = eta[elem] / 2.0
    c = np.empty((2 * xyz.shape[0], 3))
    c[0::2] = xyz + r[:, None] * nrm
    c[1::2] = xyz - r[:, None] * nrm
    return xyz, elem, np.repeat(r, 2), c


def stage1(surface, elems, order, eps=0.025, max_rounds=30):
    """Algorithm 1; returns (elements, rounds)."""
    for rounds in range(max_rounds + 1):
        xyz, elem, r, c = _centers(surface, elems, order)
        hit = any_within(c, (1.0 - eps) * r, xyz, strict=True)
        mark = np.zeros(len(elems), dtype=bool)
        mark[elem[np.nonzero(hit)[0] // 2]] = True
        if not mark.any() or rounds == max_rounds:
            return elems, rounds
        elems = bisect(elems, mark)


def stage2(surface, elems1, order, margin=0.375, max_rounds=30):
    """Algorithm 2 from the stage-1 elements (centers fixed); returns (elements, rounds)."""
    _, _, _, ctr = _centers(surface, elems1, order)
    elems = list(elems1)
    for rounds in range(max_rounds + 1):
        xyz, _, elem = nodes(surface, elems, order)
        eta = np.array([stretch(surface, *e, order) for e in elems])
        hit = any_within(xyz, margin * eta[elem], ctr, strict=False)
        mark = np.zeros(len(elems), dtype=bool)
        mark[elem[hit]] = True
        if not mark.any() or rounds == max_rounds:
            return elems, rounds
        elems = bisect(elems, mark)
