"""Synthetic surfaces, quadrature nodes and densities for the Laplace QBX workloads.

Everything here is input data: positions, weights, normals, QBX centers and radii,
target positions, the target-to-center map and densities.  The surfaces follow the
paper's test family (Section 6, the 'urchin' surfaces defined through a real spherical
harmonic bump) on a projected icosahedral mesh; the paper's own meshes and node rules are
not available, so these seeded stand-ins are used instead.

Conventions (one source node per quadrature node, two QBX centers per node):
  * center 2i   = x_i + r_i n_i  (exterior side, '+')
  * center 2i+1 = x_i - r_i n_i  (interior side, '-')
  * target k sits at the base node x_{k//2} and is evaluated through center k
  * r_i is half the largest chord between the three mapped vertices of node i's element
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------------------
# Icosahedral meshes
# ----------------------------------------------------------------------------------------


def _icosahedron():
    g = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for a in (-1.0, 1.0):
        for b in (-g, g):
            v.append((0.0, a, b))
            v.append((a, b, 0.0))
            v.append((b, 0.0, a))
    v = np.array(v, dtype=np.float64)
    v /= np.linalg.norm(v, axis=1)[:, None]
    # faces: triples whose pairwise distances equal the edge length
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    edge = np.min(d[d > 1e-12])
    adj = np.abs(d - edge) < 1e-9
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            for k in range(j + 1, 12):
                if adj[i, k] and adj[j, k]:
                    f = [i, j, k]
                    a, b, c = v[f]
                    if np.dot(np.cross(b - a, c - b), a + b + c) < 0:
                        f = [i, k, j]
                    faces.append(f)
    assert len(faces) == 20
    return v, np.array(faces, dtype=np.int64)


def icosphere(level: int):
    """Vertices on the unit sphere and outward-oriented triangles (20 * 4**level)."""
    v, f = _icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(level):
        cache = {}
        newf = []

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                p = (np.array(verts[i]) + np.array(verts[j])) * 0.5
                p /= np.linalg.norm(p)
                verts.append(tuple(p))
                cache[key] = len(verts) - 1
            return cache[key]

        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            newf += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        f = np.array(newf, dtype=np.int64)
    return np.array(verts, dtype=np.float64), f


# ----------------------------------------------------------------------------------------
# Duffy-collapsed Gauss-Legendre rule on the reference triangle {0 <= y <= x <= 1}
# ----------------------------------------------------------------------------------------


def duffy_rule(order: int):
    """(x, y, w) of an (order+1) x (order+2)//2 collapsed Gauss-Legendre rule.

    (u, v) in [0,1]^2 maps to (x, y) = (u, u v) with Jacobian u.  The rule integrates
    polynomials of total degree order+1 exactly on the reference triangle (area 1/2).
    """
    nu, nv = order + 1, (order + 2) // 2
    gu, wu = np.polynomial.legendre.leggauss(nu)
    gv, wv = np.polynomial.legendre.leggauss(nv)
    gu, wu = 0.5 * (gu + 1.0), 0.5 * wu
    gv, wv = 0.5 * (gv + 1.0), 0.5 * wv
    U, V = np.meshgrid(gu, gv, indexing="ij")
    WU, WV = np.meshgrid(wu, wv, indexing="ij")
    x = U.ravel()
    y = (U * V).ravel()
    w = (WU * WV * U).ravel()
    return x, y, w


# ----------------------------------------------------------------------------------------
# Real spherical harmonics as polynomials (complex-step friendly)
# ----------------------------------------------------------------------------------------


def _legendre_poly_part(k: int, m: int, z, r2):
    """r^(k-m) * d^m/dx^m P_k(z/r), a polynomial in z and r^2 (no Condon-Shortley phase)."""
    t_prev = None
    t = np.ones_like(z) * float(np.prod(np.arange(1, 2 * m, 2))) if m > 0 else np.ones_like(z)
    if k == m:
        return t
    t_prev, t = t, (2 * m + 1) * z * t
    for kk in range(m + 2, k + 1):
        t_prev, t = t, ((2 * kk - 1) * z * t - (kk + m - 1) * r2 * t_prev) / (kk - m)
    return t


def _cos_sin_m(m: int, x, y):
    c, s = np.ones_like(x), np.zeros_like(x)
    for _ in range(m):
        c, s = x * c - y * s, x * s + y * c
    return c, s


def _norm_factor(k: int, m: int) -> float:
    return math.sqrt((2 * k + 1) / (4 * math.pi) * math.factorial(k - m) / math.factorial(k + m))


def re_ylm_unnormalized_dir(k: int, m: int, P):
    """Re Y_k^m(P/|P|) with the paper's normalization and no Condon-Shortley phase.

    P may be complex (complex-step differentiation); the formula only uses +, -, *, / and
    sqrt.
    """
    x, y, z = P[..., 0], P[..., 1], P[..., 2]
    r2 = x * x + y * y + z * z
    r = np.sqrt(r2)
    c, _ = _cos_sin_m(m, x, y)
    return _norm_factor(k, m) * _legendre_poly_part(k, m, z, r2) * c / r**k


def real_sh_basis(lmax: int, xhat: np.ndarray) -> np.ndarray:
    """Orthonormal real spherical harmonics at unit vectors, shape ((lmax+1)^2, N).

    Row order: for l = 0..lmax, m = -l..l.  m > 0: sqrt(2) Re Y_l^m, m = 0: Y_l^0,
    m < 0: sqrt(2) Im Y_l^|m|.
    """
    x, y, z = xhat[:, 0], xhat[:, 1], xhat[:, 2]
    r2 = np.ones_like(z)
    out = np.empty(((lmax + 1) ** 2, xhat.shape[0]))
    cs = [_cos_sin_m(m, x, y) for m in range(lmax + 1)]
    for l in range(lmax + 1):
        for m in range(0, l + 1):
            t = _legendre_poly_part(l, m, z, r2) * _norm_factor(l, m)
            c, s = cs[m]
            if m == 0:
                out[l * l + l] = t
            else:
                out[l * l + l + m] = math.sqrt(2.0) * t * c
                out[l * l + l - m] = math.sqrt(2.0) * t * s
    return out


# ----------------------------------------------------------------------------------------
# Surface maps
# ----------------------------------------------------------------------------------------


@dataclass
class SurfaceSpec:
    curved: bool = True          # False: flat triangles of the icosphere
    bump_k: int = 0              # radial bump rho = 1 + a Re Y_k^m
    bump_m: int = 0
    bump_a: float = 0.0
    scale: tuple = (1.0, 1.0, 1.0)


def _surface_map(spec: SurfaceSpec, P):
    """Map a (possibly complex) point of the flat mesh to the surface."""
    if not spec.curved:
        return P
    nrm = np.sqrt(P[..., 0] ** 2 + P[..., 1] ** 2 + P[..., 2] ** 2)
    phat = P / nrm[..., None]
    rho = np.ones_like(nrm)
    if spec.bump_a != 0.0:
        rho = rho + spec.bump_a * re_ylm_unnormalized_dir(spec.bump_k, spec.bump_m, P)
    out = phat * rho[..., None]
    return out * np.asarray(spec.scale, dtype=np.float64)


def _map_and_jacobian(spec, A, B, C, x, y):
    """Surface points and the two tangent vectors d/dx, d/dy (complex-step, exact)."""
    P = A[:, None, :] + x[None, :, None] * (B - A)[:, None, :] + y[None, :, None] * (C - B)[:, None, :]
    h = 1e-30
    F = _surface_map(spec, P.astype(np.complex128)).real
    Fx = _surface_map(spec, P + 1j * h * (B - A)[:, None, :]).imag / h
    Fy = _surface_map(spec, P + 1j * h * (C - B)[:, None, :]).imag / h
    return P, F, Fx, Fy


# ----------------------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------------------


@dataclass
class Workload:
    name: str
    kernel: str                  # "S" single layer, "D" double layer
    p_qbx: int
    p_fmm: int
    nmax: int
    tcf: float
    src_xyz: np.ndarray          # (N_S, 3)
    src_w: np.ndarray            # (N_S,)   final quadrature weights (area element included)
    src_normal: np.ndarray       # (N_S, 3) unit outward normals
    src_dir: np.ndarray          # (N_S, 3) unit-sphere parameter point of each node
    ctr_xyz: np.ndarray          # (N_C, 3)
    ctr_radius: np.ndarray       # (N_C,)
    tgt_xyz: np.ndarray          # (N_T, 3)
    tgt_center: np.ndarray       # (N_T,) int64
    density: np.ndarray          # (n_densities, N_S), or node values with `interp`
    meta: dict = field(default_factory=dict)
    # Oversampled quadrature (optional): the sources are the quadrature nodes of n_elem
    # elements, element-major, and `density` holds values at each element's n_node
    # interpolation nodes; interp (n_quad, n_node) maps one element's node values to its
    # quadrature nodes.
    interp: np.ndarray | None = None
    n_elem: int = 0
    node_xyz: np.ndarray | None = None     # (n_elem * n_node, 3)
    node_normal: np.ndarray | None = None  # (n_elem * n_node, 3)
    # Element size data for target association: each source's danger radius (half its
    # element's size) and each center's side (+1 exterior, -1 interior).
    src_radius: np.ndarray | None = None
    ctr_side: np.ndarray | None = None

    @property
    def n_src(self):
        return self.src_xyz.shape[0]

    @property
    def n_ctr(self):
        return self.ctr_xyz.shape[0]

    @property
    def n_tgt(self):
        return self.tgt_xyz.shape[0]


def _nodes(level: int, order: int, spec: SurfaceSpec):
    verts, faces = icosphere(level)
    A, B, C = verts[faces[:, 0]], verts[faces[:, 1]], verts[faces[:, 2]]
    x, y, w = duffy_rule(order)
    P, F, Fx, Fy = _map_and_jacobian(spec, A, B, C, x, y)
    cr = np.cross(Fx, Fy)
    area = np.linalg.norm(cr, axis=2)
    weights = (w[None, :] * area).ravel()
    normals = (cr / area[..., None]).reshape(-1, 3)
    pts = F.reshape(-1, 3)
    # unit-sphere weights and directions (used only to smooth densities)
    unit = SurfaceSpec(curved=True)
    _, Fu, Fux, Fuy = _map_and_jacobian(unit, A, B, C, x, y)
    uw = (w[None, :] * np.linalg.norm(np.cross(Fux, Fuy), axis=2)).ravel()
    pdir = Fu.reshape(-1, 3)
    # element radius: half the largest chord between mapped vertices
    tri = np.stack([A, B, C], axis=1)
    mv = _surface_map(spec, tri.astype(np.complex128)).real
    chords = np.stack([
        np.linalg.norm(mv[:, 0] - mv[:, 1], axis=1),
        np.linalg.norm(mv[:, 1] - mv[:, 2], axis=1),
        np.linalg.norm(mv[:, 2] - mv[:, 0], axis=1),
    ], axis=1)
    rk = 0.5 * chords.max(axis=1)
    radius = np.repeat(rk, x.shape[0])
    return pts, weights, normals, pdir, uw, radius, faces.shape[0]


def _density_lowpass(rng, n_dens, pdir, unit_w, lmax=16):
    """Uniform(-1,1) node values smoothed by projection onto real Y_l^m, l <= lmax."""
    n = pdir.shape[0]
    return _lowpass_project([rng.uniform(-1.0, 1.0, n) for _ in range(n_dens)], pdir, unit_w,
                            lmax)


def _lowpass_project(raw, pdir, unit_w, lmax=16):
    n = pdir.shape[0]
    n_dens = len(raw)
    out = np.empty((n_dens, n))
    nb = (lmax + 1) ** 2
    coef = np.zeros((n_dens, nb))
    chunk = 1 << 17
    for s in range(0, n, chunk):
        Yb = real_sh_basis(lmax, pdir[s:s + chunk])
        for d in range(n_dens):
            coef[d] += Yb @ (unit_w[s:s + chunk] * raw[d][s:s + chunk])
    for s in range(0, n, chunk):
        Yb = real_sh_basis(lmax, pdir[s:s + chunk])
        out[:, s:s + chunk] = coef @ Yb
    return out


def _density_random_sh(rng, n_dens, pdir, lmax=4):
    nb = (lmax + 1) ** 2
    Yb = real_sh_basis(lmax, pdir)
    coef = rng.standard_normal((n_dens, nb))
    return coef @ Yb


def make_workload(name, *, level, order, spec: SurfaceSpec, kernel, p_qbx, p_fmm,
                  nmax=512, tcf=0.9, seed=0, n_densities=1, density="lowpass"):
    pts, w, nrm, pdir, uw, rk, ntri = _nodes(level, order, spec)
    n = pts.shape[0]
    ctr = np.empty((2 * n, 3))
    ctr[0::2] = pts + rk[:, None] * nrm
    ctr[1::2] = pts - rk[:, None] * nrm
    crad = np.repeat(rk, 2)
    tgt = np.repeat(pts, 2, axis=0)
    tgt_center = np.arange(2 * n, dtype=np.int64)
    rng = np.random.default_rng(seed)
    if density == "lowpass":
        dens = _density_lowpass(rng, n_densities, pdir, uw)
    elif density == "sh4":
        dens = _density_random_sh(rng, n_densities, pdir)
    elif density == "ones":
        dens = np.ones((n_densities, n))
    else:
        raise ValueError(density)
    return Workload(
        name=name, kernel=kernel, p_qbx=p_qbx, p_fmm=p_fmm, nmax=nmax, tcf=tcf,
        src_xyz=pts, src_w=w, src_normal=nrm, src_dir=pdir,
        ctr_xyz=ctr, ctr_radius=crad, tgt_xyz=tgt, tgt_center=tgt_center,
        density=np.ascontiguousarray(dens),
        meta=dict(level=level, order=order, n_triangles=ntri, seed=seed,
                  curved=spec.curved, bump=(spec.bump_k, spec.bump_m, spec.bump_a),
                  scale=spec.scale, density=density),
        src_radius=rk.copy(), ctr_side=np.tile(np.array([1, -1], dtype=np.int8), n),
    )


def interior_lattice(order: int):
    """Reference coordinates (x, y) on {0 <= y <= x <= 1} of the interior points of the
    degree-(order+3) barycentric lattice: a scaled principal lattice of degree `order`,
    (order+1)(order+2)/2 points, unisolvent for polynomials of total degree <= order, none
    on an edge (so no node is shared between elements)."""
    n = order + 3
    lam = np.array([(a, b, n - a - b) for a in range(1, n) for b in range(1, n - a)
                    if n - a - b >= 1], dtype=np.float64) / n
    # vertices (0,0), (1,0), (1,1) carry barycentric weights lam[:, 0], lam[:, 1], lam[:, 2]
    return lam[:, 1] + lam[:, 2], lam[:, 2]


def subdivided_rule(order: int, sub: int):
    """The collapsed Gauss-Legendre rule of `order` on each of the sub^2 congruent
    sub-triangles of the reference triangle: (x, y, w), weights summing to 1/2."""
    xr, yr, wr = duffy_rule(order)
    pts, wts = [], []
    for i in range(sub):
        for j in range(i + 1):
            v0 = np.array([i, j]) / sub
            tris = [(v0, np.array([i + 1, j]) / sub, np.array([i + 1, j + 1]) / sub)]
            if j < i:
                tris.append((v0, np.array([i + 1, j + 1]) / sub, np.array([i, j + 1]) / sub))
            for a, b, c in tris:
                pts.append(a[None] + xr[:, None] * (b - a)[None] + yr[:, None] * (c - b)[None])
                wts.append(wr / sub ** 2)
    p = np.concatenate(pts)
    return p[:, 0], p[:, 1], np.concatenate(wts)


def lattice_interpolation(order: int, xq, yq):
    """Matrix (len(xq), n_node) taking values at interior_lattice(order) to the values of
    their degree-`order` interpolating polynomial at the points (xq, yq)."""
    xn, yn = interior_lattice(order)
    mono = [(i, j) for i in range(order + 1) for j in range(order + 1 - i)]
    vn = np.stack([xn ** i * yn ** j for i, j in mono], axis=1)
    vq = np.stack([xq ** i * yq ** j for i, j in mono], axis=1)
    return np.linalg.solve(vn.T, vq.T).T


def oversampled_workload(name, *, level, spec: SurfaceSpec, kernel, p_qbx, p_fmm,
                         node_order=4, quad_order=4, sub=4, sides="both", nmax=512, tcf=0.9,
                         seed=0, n_densities=1):
    """A surface discretized as the paper's stage-2 pair (Section 3): the density lives on a
    unisolvent node set per element (interior_lattice(node_order)) and the layer potential
    uses an oversampled quadrature on the same elements (subdivided_rule(quad_order, sub)).

    Sources are the quadrature nodes (element-major); each density node gets its QBX
    center(s) at distance r_k (half the largest chord of its element) along the normal:
    sides "both" gives centers 2i (exterior) and 2i+1 (interior) with targets at the node,
    "interior" or "exterior" one center per node and target i at node i (a square
    operator).  Densities: random combinations of real Y_l^m, l <= 4, at the nodes' sphere
    directions (seed `seed`)."""
    verts, faces = icosphere(level)
    A, B, C = verts[faces[:, 0]], verts[faces[:, 1]], verts[faces[:, 2]]
    ne = faces.shape[0]
    xn, yn = interior_lattice(node_order)
    xq, yq, wq = subdivided_rule(quad_order, sub)
    interp = lattice_interpolation(node_order, xq, yq)
    _, Fn, Fnx, Fny = _map_and_jacobian(spec, A, B, C, xn, yn)
    crn = np.cross(Fnx, Fny)
    node = Fn.reshape(-1, 3)
    node_nrm = (crn / np.linalg.norm(crn, axis=2)[..., None]).reshape(-1, 3)
    _, Fq, Fqx, Fqy = _map_and_jacobian(spec, A, B, C, xq, yq)
    crq = np.cross(Fqx, Fqy)
    arq = np.linalg.norm(crq, axis=2)
    src = Fq.reshape(-1, 3)
    src_nrm = (crq / arq[..., None]).reshape(-1, 3)
    src_w = (wq[None, :] * arq).ravel()
    _, Fu, _, _ = _map_and_jacobian(SurfaceSpec(curved=True), A, B, C, xq, yq)
    _, Fun, _, _ = _map_and_jacobian(SurfaceSpec(curved=True), A, B, C, xn, yn)
    tri = np.stack([A, B, C], axis=1)
    mv = _surface_map(spec, tri.astype(np.complex128)).real
    chords = np.stack([np.linalg.norm(mv[:, 0] - mv[:, 1], axis=1),
                       np.linalg.norm(mv[:, 1] - mv[:, 2], axis=1),
                       np.linalg.norm(mv[:, 2] - mv[:, 0], axis=1)], axis=1)
    rk = np.repeat(0.5 * chords.max(axis=1), xn.shape[0])
    nn = node.shape[0]
    if sides == "both":
        ctr = np.empty((2 * nn, 3))
        ctr[0::2] = node + rk[:, None] * node_nrm
        ctr[1::2] = node - rk[:, None] * node_nrm
        crad = np.repeat(rk, 2)
        tgt = np.repeat(node, 2, axis=0)
        side = np.tile(np.array([1, -1], dtype=np.int8), nn)
    elif sides in ("interior", "exterior"):
        sgn = -1.0 if sides == "interior" else 1.0
        ctr = node + sgn * rk[:, None] * node_nrm
        crad = rk.copy()
        tgt = node.copy()
        side = np.full(nn, int(sgn), dtype=np.int8)
    else:
        raise ValueError(sides)
    rng = np.random.default_rng(seed)
    dens = _density_random_sh(rng, n_densities, Fun.reshape(-1, 3))
    return Workload(
        name=name, kernel=kernel, p_qbx=p_qbx, p_fmm=p_fmm, nmax=nmax, tcf=tcf,
        src_xyz=src, src_w=src_w, src_normal=src_nrm, src_dir=Fu.reshape(-1, 3),
        ctr_xyz=ctr, ctr_radius=crad, tgt_xyz=tgt,
        tgt_center=np.arange(ctr.shape[0], dtype=np.int64),
        density=np.ascontiguousarray(dens),
        meta=dict(level=level, node_order=node_order, quad_order=quad_order, sub=sub,
                  n_triangles=ne, seed=seed, sides=sides, curved=spec.curved,
                  bump=(spec.bump_k, spec.bump_m, spec.bump_a), scale=spec.scale),
        interp=interp, n_elem=ne, node_xyz=node, node_normal=node_nrm,
        src_radius=np.repeat(rk[::xn.shape[0]], xq.shape[0]), ctr_side=side)


def workload_c1(nmax=512, n_densities=1, p_fmm=10, p_qbx=3, kernel="S"):
    """Unit sphere as 320 flat triangles, 15-node rule, S, p_qbx=3, p_fmm=10, seed 1."""
    return make_workload("sphere320-flat", level=2, order=4, spec=SurfaceSpec(curved=False),
                         kernel=kernel, p_qbx=p_qbx, p_fmm=p_fmm, nmax=nmax, seed=1,
                         n_densities=n_densities, density="sh4")


def workload_c2(n_densities=1, seed=2, nmax=512):
    """Urchin rho = 1 + 0.2 Re Y_8^4 on 20480 curved triangles, 28-node rule, D, 5/15."""
    return make_workload("urchin8-20480", level=5, order=6,
                         spec=SurfaceSpec(curved=True, bump_k=8, bump_m=4, bump_a=0.2),
                         kernel="D", p_qbx=5, p_fmm=15, nmax=nmax, seed=seed,
                         n_densities=n_densities, density="lowpass")


def workload_c4(n_densities=1, seed=4, nmax=512):
    """Ellipsoid (3,1,1) with the Y_8^4 bump on 81920 triangles, 28-node rule, S, 8/20."""
    return make_workload("ellipsoid-urchin-81920", level=6, order=6,
                         spec=SurfaceSpec(curved=True, bump_k=8, bump_m=4, bump_a=0.2,
                                          scale=(3.0, 1.0, 1.0)),
                         kernel="S", p_qbx=8, p_fmm=20, nmax=nmax, seed=seed,
                         n_densities=n_densities, density="lowpass")


def add_point_targets(w: Workload, n_out=200, n_in=100, r_out=(1.4, 2.0), r_in=(0.2, 0.55),
                      seed=11) -> Workload:
    """A copy of w with conventional targets appended (tgt_center = -1): n_out points at
    radii r_out (outside the surface) and n_in at radii r_in (inside), uniform in
    direction."""
    import dataclasses

    rng = np.random.default_rng(seed)

    def shell(n, lo, hi):
        v = rng.standard_normal((n, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        return v * rng.uniform(lo, hi, n)[:, None]

    pts = np.concatenate([shell(n_out, *r_out), shell(n_in, *r_in)])
    return dataclasses.replace(
        w, name=w.name + f"+{len(pts)}pt",
        tgt_xyz=np.concatenate([w.tgt_xyz, pts]),
        tgt_center=np.concatenate([w.tgt_center, np.full(len(pts), -1, dtype=np.int64)]),
        meta=dict(w.meta, point_targets=len(pts)))


def c3_surface_params(i: int):
    """Surface i (0..63) of the 64-surface batch: bump order k ~ U{2..10} with m = k // 2,
    amplitude ~ U(0.05, 0.25), icosphere level ~ U{3..6}; seeded by 3000 + i."""
    rng = np.random.default_rng(3000 + i)
    k = int(rng.integers(2, 11))
    amp = float(rng.uniform(0.05, 0.25))
    level = int(rng.integers(3, 7))
    return k, k // 2, amp, level


def workload_c3(i: int, n_densities=8, nmax=512):
    """Surface i of the 64-urchin batch: 28-node rule, D, 5/15; density d of surface i is
    the smoothed recipe seeded by 3000 + 64 + 8 i + d."""
    k, m, amp, level = c3_surface_params(i)
    spec = SurfaceSpec(curved=True, bump_k=k, bump_m=m, bump_a=amp)
    w = make_workload(f"urchin{k}-{20 * 4 ** level}-s{i}", level=level, order=6, spec=spec,
                      kernel="D", p_qbx=5, p_fmm=15, nmax=nmax, seed=3000 + i, n_densities=1,
                      density="ones")
    raw = [np.random.default_rng(3000 + 64 + 8 * i + d).uniform(-1.0, 1.0, w.n_src)
           for d in range(n_densities)]
    w.density = np.ascontiguousarray(_lowpass_project(raw, w.src_dir, _unit_weights(level, 6)))
    w.meta["density"] = "lowpass"
    return w


def fresh_densities(w: Workload, count: int, seed0: int = 5000):
    """`count` new densities on w's nodes by the urchin recipe (uniform(-1, 1) node values
    smoothed by projection onto real Y_l^m, l <= 16); density i is seeded by seed0 + i."""
    raw = [np.random.default_rng(seed0 + i).uniform(-1.0, 1.0, w.n_src) for i in range(count)]
    uw = _unit_weights(w.meta["level"], w.meta["order"])
    return np.ascontiguousarray(_lowpass_project(raw, w.src_dir, uw))


def _unit_weights(level, order):
    verts, faces = icosphere(level)
    A, B, C = verts[faces[:, 0]], verts[faces[:, 1]], verts[faces[:, 2]]
    x, y, w = duffy_rule(order)
    _, _, Fux, Fuy = _map_and_jacobian(SurfaceSpec(curved=True), A, B, C, x, y)
    return (w[None, :] * np.linalg.norm(np.cross(Fux, Fuy), axis=2)).ravel()


def workload_tiny(level=1, order=2, kernel="S", p_qbx=3, p_fmm=6, nmax=32, tcf=0.9,
                  curved=True, bump=(3, 1, 0.15), seed=7, n_densities=1, density="lowpass"):
    """Small curved surfaces that still produce several tree levels and every list."""
    spec = SurfaceSpec(curved=curved, bump_k=bump[0], bump_m=bump[1], bump_a=bump[2])
    return make_workload(f"tiny-l{level}-o{order}", level=level, order=order, spec=spec,
                         kernel=kernel, p_qbx=p_qbx, p_fmm=p_fmm, nmax=nmax, tcf=tcf,
                         seed=seed, n_densities=n_densities, density=density)
