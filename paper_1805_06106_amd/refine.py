"""Geometry processing for user meshes: stage-1 and stage-2 refinement (Section 3,
Algorithms 1 and 2) and the oversampled stage-2 quadrature discretization.

A mesh is a set of triangles given in a parameter space (vertices A, B, C per element, as
3-vectors) and a smooth map `surface` from parameter points to the surface.  The map takes
arrays of points (..., 3) and must accept complex input: tangents are taken by complex-step
differentiation, so they are exact to rounding.  A flat mesh uses the identity map.

Element size (the stretch factor of Section 3): with the element mapped from the bi-unit
equilateral reference triangle, eta(x) = 2 sigma_1(Jacobian at x) and eta_k is its largest
value over the element (taken over its quadrature nodes and vertices).  Expansion radius
r_k = eta_k / 2 (stage 1).  "Bisecting" an element splits it into the four triangles of its
edge midpoints in parameter space, which halves eta_k; the mesh need not stay conforming.

* Stage 1 (truncation): a center c = x +- r_k n of a node x on element k whose ball of
  radius (1 - eps) r_k holds another source point strictly inside marks element k
  (Algorithm 1, eps = 0.025), and so does a scaled curvature max(|k1|, |k2|) eta(x) above
  0.8 at a node (the scaled-curvature criterion); marked elements are bisected until none
  is marked.
* Stage 2 (quadrature resolution): starting from the stage-1 elements, with the stage-1
  centers fixed, a stage-2 element with a source point within 0.5 (3/4) eta of some center
  is bisected, until none is.
* The stage-2 quadrature discretization uses a higher-order rule on the stage-2 elements.

The proximity queries run on the GPU through the library (`gq_points_near`); the rest is
bookkeeping on the host.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import _capi as C

# affine map from the bi-unit equilateral reference triangle (-1, -1/sqrt3), (1, -1/sqrt3),
# (0, 2/sqrt3) onto {0 <= y <= x <= 1} (vertices (0,0), (1,0), (1,1)): its linear part
_EQ = np.array([[0.5, 0.5 / math.sqrt(3.0)], [0.0, 1.0 / math.sqrt(3.0)]])


def collapsed_rule(order: int):
    """(x, y, w) on {0 <= y <= x <= 1}: an (order+1) x (order+2)//2 Gauss-Legendre grid in
    (u, v) mapped by (x, y) = (u, u v), exact for total degree order + 1; weights sum to
    1/2."""
    nu, nv = order + 1, (order + 2) // 2
    gu, wu = np.polynomial.legendre.leggauss(nu)
    gv, wv = np.polynomial.legendre.leggauss(nv)
    u, v = np.meshgrid(0.5 * (gu + 1.0), 0.5 * (gv + 1.0), indexing="ij")
    wuu, wvv = np.meshgrid(0.5 * wu, 0.5 * wv, indexing="ij")
    return u.ravel(), (u * v).ravel(), (wuu * wvv * u).ravel()


@dataclass
class ParamMesh:
    A: np.ndarray  # (n_elem, 3) parameter-space vertices
    B: np.ndarray
    C: np.ndarray
    surface: object  # callable (..., 3) -> (..., 3), complex-capable
    parent: np.ndarray | None = None  # element of the mesh this one was refined from

    @property
    def n_elem(self):
        return self.A.shape[0]

    def _map(self, x, y):
        """Surface points and tangents d/dx, d/dy at reference points (x, y), per element."""
        P = (self.A[:, None, :] + x[None, :, None] * (self.B - self.A)[:, None, :]
             + y[None, :, None] * (self.C - self.B)[:, None, :])
        h = 1e-30
        F = np.asarray(self.surface(P.astype(np.complex128))).real
        Fx = np.asarray(self.surface(P + 1j * h * (self.B - self.A)[:, None, :])).imag / h
        Fy = np.asarray(self.surface(P + 1j * h * (self.C - self.B)[:, None, :])).imag / h
        return F, Fx, Fy

    def nodes(self, order: int):
        """Quadrature nodes of every element: xyz, unit normals, weights (area element
        included) and the element index of each node, element-major."""
        x, y, w = collapsed_rule(order)
        F, Fx, Fy = self._map(x, y)
        cr = np.cross(Fx, Fy)
        area = np.linalg.norm(cr, axis=2)
        return {"xyz": F.reshape(-1, 3), "normal": (cr / area[..., None]).reshape(-1, 3),
                "weight": (w[None, :] * area).ravel(),
                "elem": np.repeat(np.arange(self.n_elem), x.shape[0])}

    def _stretch_points(self, order: int):
        x, y, _ = collapsed_rule(order)
        return np.concatenate([x, [0.0, 1.0, 1.0]]), np.concatenate([y, [0.0, 0.0, 1.0]])

    def scaled_curvature(self, order: int, h: float = 1e-5):
        """kappa_k: the largest max(|k1|, |k2|) eta(x) over the element's nodes and vertices,
        k1, k2 the principal curvatures (the scaled-curvature criterion of Section 3).  The
        second derivatives are central differences of the exact first derivatives."""
        x, y = self._stretch_points(order)
        _, Fx, Fy = self._map(x, y)
        _, Fxp, Fyp = self._map(x + h, y)
        _, Fxm, Fym = self._map(x - h, y)
        _, Fxq, Fyq = self._map(x, y + h)
        _, Fxr, Fyr = self._map(x, y - h)
        Fxx = (Fxp - Fxm) / (2 * h)
        Fyy = (Fyq - Fyr) / (2 * h)
        Fxy = 0.5 * ((Fyp - Fym) / (2 * h) + (Fxq - Fxr) / (2 * h))
        nrm = np.cross(Fx, Fy)
        nrm /= np.linalg.norm(nrm, axis=2)[..., None]
        E, Fm, Gm = (np.sum(a * b, axis=2) for a, b in ((Fx, Fx), (Fx, Fy), (Fy, Fy)))
        L, M, N = (np.sum(a * nrm, axis=2) for a in (Fxx, Fxy, Fyy))
        det = E * Gm - Fm * Fm
        H = (E * N - 2.0 * Fm * M + Gm * L) / (2.0 * det)
        K = (L * N - M * M) / det
        kmax = np.abs(H) + np.sqrt(np.maximum(H * H - K, 0.0))
        return np.max(kmax * self._stretch(Fx, Fy), axis=1)

    @staticmethod
    def _stretch(Fx, Fy):
        """2 sigma_1 of the Jacobian of the equilateral-reference map, per point."""
        a = Fx * _EQ[0, 0] + Fy * _EQ[1, 0]
        b = Fx * _EQ[0, 1] + Fy * _EQ[1, 1]
        g11 = np.sum(a * a, axis=2)
        g22 = np.sum(b * b, axis=2)
        g12 = np.sum(a * b, axis=2)
        lam = 0.5 * (g11 + g22) + np.sqrt(0.25 * (g11 - g22) ** 2 + g12 * g12)
        return 2.0 * np.sqrt(lam)

    def element_size(self, order: int):
        """eta_k: the largest stretch factor 2 sigma_1 of the equilateral-reference map over
        the element's order-`order` nodes and its vertices."""
        x, y = self._stretch_points(order)
        _, Fx, Fy = self._map(x, y)
        # columns of J M, M the equilateral map; sigma_1^2 = largest eigenvalue of the Gram
        return np.max(self._stretch(Fx, Fy), axis=1)

    def bisect(self, mark):
        """A mesh with each marked element replaced by its four midpoint children (children
        appended after the unmarked elements, in element order); `parent` maps every
        element to its element in self."""
        mark = np.asarray(mark, dtype=bool)
        keep = np.nonzero(~mark)[0]
        cut = np.nonzero(mark)[0]
        A, B, Cc = self.A[cut], self.B[cut], self.C[cut]
        ab, bc, ca = 0.5 * (A + B), 0.5 * (B + Cc), 0.5 * (Cc + A)
        # the same orientation as the parent: (A, ab, ca), (ab, B, bc), (ca, bc, C), (bc, ca, ab)
        kids = [(A, ab, ca), (ab, B, bc), (ca, bc, Cc), (bc, ca, ab)]
        nA = np.concatenate([self.A[keep]] + [k[0] for k in kids])
        nB = np.concatenate([self.B[keep]] + [k[1] for k in kids])
        nC = np.concatenate([self.C[keep]] + [k[2] for k in kids])
        par = np.concatenate([keep] + [cut] * 4)
        return ParamMesh(nA, nB, nC, self.surface, par)


def centers(mesh: ParamMesh, order: int, eta=None):
    """QBX centers of the mesh's nodes: node i has the exterior center 2i (x + r n) and the
    interior center 2i+1 (x - r n), r = eta_k / 2 of its element."""
    nd = mesh.nodes(order)
    eta = mesh.element_size(order) if eta is None else eta
    r = 0.5 * eta[nd["elem"]]
    c = np.empty((2 * r.shape[0], 3))
    c[0::2] = nd["xyz"] + r[:, None] * nd["normal"]
    c[1::2] = nd["xyz"] - r[:, None] * nd["normal"]
    return nd, np.repeat(r, 2), c


def refine_stage1(mesh: ParamMesh, order: int, eps: float = 0.025, kappa_max=0.8,
                  max_rounds: int = 30, stream=None):
    """Stage-1 refinement: bisect elements whose expansion balls of radius (1 - eps) r_k
    hold a source point strictly inside (Algorithm 1), or, unless kappa_max is None, whose
    scaled curvature exceeds kappa_max (0.8 in the paper), until none does.  Returns
    (mesh, rounds, origin) with origin[k] the input element that element k came from."""
    origin = np.arange(mesh.n_elem)
    for rounds in range(max_rounds + 1):
        nd, r, c = centers(mesh, order)
        hit = C.gq_points_near(c, (1.0 - eps) * r, nd["xyz"], strict=True, stream=stream)
        mark = np.zeros(mesh.n_elem, dtype=bool)
        mark[nd["elem"][np.nonzero(hit)[0] // 2]] = True
        if kappa_max is not None:
            mark |= mesh.scaled_curvature(order) > kappa_max
        if not mark.any() or rounds == max_rounds:
            return mesh, rounds, origin
        mesh = mesh.bisect(mark)
        origin = origin[mesh.parent]
    return mesh, max_rounds, origin


def refine_stage2(mesh1: ParamMesh, order: int, margin: float = 0.5 * 0.75,
                  max_rounds: int = 30, stream=None):
    """Algorithm 2: from the stage-1 mesh (whose centers stay fixed), bisect stage-2 elements
    having a source point within margin * eta of some center, until none does.  Returns
    (mesh2, rounds, origin) with origin[k] the stage-1 element of stage-2 element k."""
    _, _, ctr = centers(mesh1, order)
    mesh = ParamMesh(mesh1.A, mesh1.B, mesh1.C, mesh1.surface)
    origin = np.arange(mesh.n_elem)
    for rounds in range(max_rounds + 1):
        nd = mesh.nodes(order)
        eta = mesh.element_size(order)
        hit = C.gq_points_near(nd["xyz"], margin * eta[nd["elem"]], ctr, strict=False,
                               stream=stream)
        mark = np.zeros(mesh.n_elem, dtype=bool)
        mark[nd["elem"][hit]] = True
        if not mark.any() or rounds == max_rounds:
            return mesh, rounds, origin
        mesh = mesh.bisect(mark)
        origin = origin[mesh.parent]
    return mesh, max_rounds, origin


def discretize(mesh: ParamMesh, order: int = 4, quad_order: int = 8, eps: float = 0.025,
               kappa_max=0.8, stream=None):
    """Stage 1 and 2 refinement of `mesh` and its stage-2 quadrature discretization.

    Returns a dict: the stage-1 nodes (targets, with their two centers each: ctr 2i exterior,
    2i+1 interior, and radii), the quadrature sources (xyz, normal, weight) on the stage-2
    elements with the order-`quad_order` rule, both meshes and the round counts."""
    m1, rounds1, _ = refine_stage1(mesh, order, eps=eps, kappa_max=kappa_max, stream=stream)
    eta1 = m1.element_size(order)
    nd1, r, ctr = centers(m1, order, eta1)
    m2, rounds2, origin2 = refine_stage2(m1, order, stream=stream)
    q = m2.nodes(quad_order)
    return {"stage1": m1, "stage2": m2, "stage2_parent": origin2, "rounds": (rounds1, rounds2),
            "node_xyz": nd1["xyz"], "node_normal": nd1["normal"], "node_weight": nd1["weight"],
            "ctr_xyz": ctr, "ctr_radius": r,
            "src_xyz": q["xyz"], "src_normal": q["normal"], "src_w": q["weight"],
            "src_elem": q["elem"]}
