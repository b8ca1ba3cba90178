"""Oracle for geometry processing: stage-1 refinement (Algorithm 1 and the scaled-curvature
criterion of Section 3) and stage-2 refinement (Algorithm 2) by brute force.

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
    """Points and tangents (d/dx, d/dy) at reference points; A, B, C are one element's
    vertices (3,) or a batch of elements (n, 3), giving arrays (..., n_points, 3)."""
    A, B, C = (np.asarray(v, dtype=float) for v in (A, B, C))
    x, y = np.asarray(x, dtype=float), np.asarray(y, dtype=float)
    e1, e2 = (B - A)[..., None, :], (C - B)[..., None, :]
    P = A[..., None, :] + x[:, None] * e1 + y[:, None] * e2
    h = 1e-30
    F = np.asarray(surface(P.astype(complex))).real
    Fx = np.asarray(surface(P + 1j * h * e1)).imag / h
    Fy = np.asarray(surface(P + 1j * h * e2)).imag / h
    return F, Fx, Fy


def _check_points(order):
    x, y, _ = rule(order)
    return np.concatenate([x, [0.0, 1.0, 1.0]]), np.concatenate([y, [0.0, 0.0, 1.0]])


def _stretch_at(Fx, Fy):
    """2 sigma_1(J G) at every point (SVD of the stacked 3 x 2 Jacobians)."""
    J = np.stack([Fx, Fy], axis=-1) @ _equilateral_to_tri()
    return 2.0 * np.linalg.svd(J, compute_uv=False)[..., 0]


def stretch(surface, A, B, C, order):
    """eta_k = max over the element's nodes and vertices of 2 sigma_1(J G) (one element or a
    batch)."""
    x, y = _check_points(order)
    _, Fx, Fy = element_geometry(surface, A, B, C, x, y)
    return np.max(_stretch_at(Fx, Fy), axis=-1)


def principal_curvatures(surface, A, B, C, x, y, h=1e-3):
    """(k1, k2) at reference points: eigenvalues of the shape operator I^-1 II, with the
    second derivatives of the map from fourth-order central differences of point
    positions (the mixed one from the second derivative along the diagonal)."""
    x, y = np.asarray(x, dtype=float), np.asarray(y, dtype=float)

    def d2(ex, ey):  # second derivative along the reference direction (ex, ey)
        f = [element_geometry(surface, A, B, C, x + k * h * ex, y + k * h * ey)[0]
             for k in (-2, -1, 0, 1, 2)]
        return (-f[4] + 16 * f[3] - 30 * f[2] + 16 * f[1] - f[0]) / (12 * h * h)

    _, Fx, Fy = element_geometry(surface, A, B, C, x, y)
    fxx, fyy = d2(1, 0), d2(0, 1)
    fxy = 0.5 * (d2(1, 1) - fxx - fyy)
    n = np.cross(Fx, Fy)
    n /= np.linalg.norm(n, axis=-1)[..., None]
    dot = lambda a, b: np.sum(a * b, axis=-1)  # noqa: E731
    I1 = np.stack([np.stack([dot(Fx, Fx), dot(Fx, Fy)], -1), np.stack([dot(Fx, Fy), dot(Fy, Fy)], -1)], -2)
    I2 = np.stack([np.stack([dot(fxx, n), dot(fxy, n)], -1), np.stack([dot(fxy, n), dot(fyy, n)], -1)], -2)
    return np.sort(np.real(np.linalg.eigvals(np.linalg.solve(I1, I2))), axis=-1)


def scaled_curvature(surface, A, B, C, order):
    """kappa_k = max over nodes and vertices of max(|k1|, |k2|) * 2 sigma_1(J G) (one
    element or a batch)."""
    x, y = _check_points(order)
    k = principal_curvatures(surface, A, B, C, x, y)
    _, Fx, Fy = element_geometry(surface, A, B, C, x, y)
    return np.max(np.max(np.abs(k), axis=-1) * _stretch_at(Fx, Fy), axis=-1)


def _batch(elems):
    return tuple(np.array([e[i] for e in elems]) for i in range(3))


def nodes(surface, elems, order):
    x, y, w = rule(order)
    F, Fx, Fy = element_geometry(surface, *_batch(elems), x, y)
    cr = np.cross(Fx, Fy)
    nrm = cr / np.linalg.norm(cr, axis=-1)[..., None]
    return F.reshape(-1, 3), nrm.reshape(-1, 3), np.repeat(np.arange(len(elems)), x.shape[0])


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
    eta = stretch(surface, *_batch(elems), order)
    r = eta[elem] / 2.0
    c = np.empty((2 * xyz.shape[0], 3))
    c[0::2] = xyz + r[:, None] * nrm
    c[1::2] = xyz - r[:, None] * nrm
    return xyz, elem, np.repeat(r, 2), c


def stage1(surface, elems, order, eps=0.025, kappa_max=0.8, max_rounds=30):
    """Stage 1: Algorithm 1 and, unless kappa_max is None, the scaled-curvature criterion;
    returns (elements, rounds)."""
    for rounds in range(max_rounds + 1):
        xyz, elem, r, c = _centers(surface, elems, order)
        hit = any_within(c, (1.0 - eps) * r, xyz, strict=True)
        mark = np.zeros(len(elems), dtype=bool)
        mark[elem[np.nonzero(hit)[0] // 2]] = True
        if kappa_max is not None:
            mark |= scaled_curvature(surface, *_batch(elems), order) > kappa_max
        if not mark.any() or rounds == max_rounds:
            return elems, rounds
        elems = bisect(elems, mark)


def stage2(surface, elems1, order, margin=0.375, max_rounds=30):
    """Algorithm 2 from the stage-1 elements (centers fixed); returns (elements, rounds)."""
    _, _, _, ctr = _centers(surface, elems1, order)
    elems = list(elems1)
    for rounds in range(max_rounds + 1):
        xyz, _, elem = nodes(surface, elems, order)
        eta = stretch(surface, *_batch(elems), order)
        hit = any_within(xyz, margin * eta[elem], ctr, strict=False)
        mark = np.zeros(len(elems), dtype=bool)
        mark[elem[hit]] = True
        if not mark.any() or rounds == max_rounds:
            return elems, rounds
        elems = bisect(elems, mark)
