"""Pins for the Tier A oracle (direct QBX) against closed forms.

* Unit sphere: S[Y_l^m] = Y/(2l+1) on the surface; D[Y_l^m] has one-sided limits
  -(l+1)/(2l+1) Y (inside) and l/(2l+1) Y (outside); D[1] = -1 inside, 0 outside
  (Gauss's law).  The interior potential of S and D is a polynomial of degree l, so the
  interior QBX result carries only quadrature error; the exterior side also carries the
  O(r^(p+1)) truncation error of Lemma 1.
* Flat triangle: the double layer of density 1 is -Omega/(4 pi), Omega the signed solid
  angle (van Oosterom-Strackee).
* Evaluation at the center itself reduces the QBX expansion to its n = 0 term, the point
  value of the discretized potential.
"""

import math

import numpy as np
import pytest

import oracle as O
from workloads.geometry import SurfaceSpec, duffy_rule, make_workload, real_sh_basis

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _sphere_case(q, kernel, l, m, n_sample=96, seed=3):
    """Sources: curved unit sphere, level 4, 28 nodes/triangle (16x finer than the
    centers' level-2 mesh); centers/targets: level 2, 15 nodes/triangle."""
    fine = make_workload("fine", level=4, order=6, spec=SurfaceSpec(curved=True), kernel=kernel,
                         p_qbx=q, p_fmm=q, density="ones")
    coarse = make_workload("coarse", level=2, order=4, spec=SurfaceSpec(curved=True),
                           kernel=kernel, p_qbx=q, p_fmm=q, density="ones")
    idx = l * l + l + m
    dens = real_sh_basis(l, fine.src_xyz)[idx] if l >= 0 else np.ones(fine.n_src)
    rng = np.random.default_rng(seed)
    cids = np.sort(rng.choice(coarse.n_ctr, n_sample, replace=False))
    tgt = coarse.tgt_xyz[cids]
    pot, _ = O.direct_qbx(kernel, q, fine.src_xyz, fine.src_w * dens, coarse.ctr_xyz[cids], tgt,
                          np.arange(len(cids)), nrm=fine.src_normal)
    exterior = (cids % 2) == 0
    yt = real_sh_basis(max(l, 0), tgt)[idx] if l >= 0 else np.ones(len(cids))
    return pot, yt, exterior


@pytest.mark.parametrize("l,m", [(0, 0), (2, 1), (3, -2)])
def test_single_layer_sphere_eigenrelation(l, m):
    q = 5
    pot, y, ext = _sphere_case(q, "S", l, m)
    ref = y / (2 * l + 1)
    scale = np.abs(ref).max() if l > 0 else 1.0
    err_in = np.abs(pot[~ext] - ref[~ext]).max() / scale
    err_out = np.abs(pot[ext] - ref[ext]).max() / scale
    assert err_in < 1e-7
    assert err_out < 1e-3


@pytest.mark.parametrize("l,m", [(1, 0), (2, 1)])
def test_double_layer_sphere_eigenrelation(l, m):
    q = 3
    pot, y, ext = _sphere_case(q, "D", l, m)
    inside = -(l + 1) / (2 * l + 1) * y
    outside = l / (2 * l + 1) * y
    scale = np.abs(y).max()
    assert np.abs(pot[~ext] - inside[~ext]).max() / scale < 1e-6
    assert np.abs(pot[ext] - outside[ext]).max() / scale < 5e-3


def test_gauss_law_double_layer():
    pot, _, ext = _sphere_case(3, "D", -1, 0)
    assert np.abs(pot[~ext] + 1.0).max() < 1e-6
    assert np.abs(pot[ext]).max() < 1e-5


def _solid_angle(a, b, c, x):
    r1, r2, r3 = a - x, b - x, c - x
    n1, n2, n3 = np.linalg.norm(r1), np.linalg.norm(r2), np.linalg.norm(r3)
    num = np.dot(r1, np.cross(r2, r3))
    den = n1 * n2 * n3 + np.dot(r1, r2) * n3 + np.dot(r1, r3) * n2 + np.dot(r2, r3) * n1
    return 2.0 * math.atan2(num, den)


@pytest.mark.parametrize("x", [np.array([0.3, 0.2, 0.4]), np.array([0.5, 0.1, -0.35]),
                               np.array([-0.2, 0.6, 0.5])])
def test_double_layer_flat_triangle_solid_angle(x):
    A, B, C = np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.0, 0.0]), np.array([0.6, 0.8, 0.0])
    u, v, w = duffy_rule(40)
    pts = A + u[:, None] * (B - A) + v[:, None] * (C - B)
    n = np.cross(B - A, C - B)
    area2 = np.linalg.norm(n)
    n = n / area2
    wts = w * area2
    pot, _ = O.direct_qbx("D", 0, pts, wts, x[None, :], x[None, :], np.array([0]),
                          nrm=np.repeat(n[None, :], len(pts), axis=0))
    ref = -_solid_angle(A, B, C, x) / (4 * math.pi)
    assert abs(pot[0] - ref) < 1e-9


def test_evaluation_at_center_is_point_sum():
    rng = np.random.default_rng(0)
    src = rng.standard_normal((200, 3))
    qs = rng.standard_normal(200)
    ctr = np.array([[0.1, 0.2, 0.05], [3.0, -1.0, 0.5]])
    pot, _ = O.direct_qbx("S", 6, src, qs, ctr, ctr, np.array([0, 1]))
    for i in range(2):
        ref = np.sum(qs / (4 * math.pi * np.linalg.norm(src - ctr[i], axis=1)))
        assert abs(pot[i] - ref) < 1e-13 * np.sum(np.abs(qs))


def test_direct_qbx_is_linear_and_matches_explicit_sum():
    """Tier A = evaluation of the sum of per-source local expansions (the quadrature sum of
    the QBX coefficient integral); checks the batched path against the one-source path."""
    rng = np.random.default_rng(1)
    src = rng.standard_normal((30, 3)) * 2
    nrm = rng.standard_normal((30, 3))
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    qs = rng.standard_normal(30)
    c = np.array([[0.2, -0.1, 0.3]])
    t = c + np.array([[0.05, 0.02, -0.01]])
    for kern in ("S", "D"):
        pot, _ = O.direct_qbx(kern, 4, src, qs, c, t, np.array([0]), nrm=nrm)
        L = np.zeros(25, dtype=complex)
        for j in range(30):
            L += O.p2l(kern, 4, src[j], [qs[j]], c[0], nrm=nrm[j])
        assert abs(pot[0] - O.eval_local(4, L, c[0], t[0])) < 1e-14 * np.abs(L).max()


# --- adjoint double layer S' = d/dn_t S (the Neumann operator) -----------------------------

def _sphere_sprime(q, l, m, n_sample=64, seed=4):
    fine = make_workload("fine", level=4, order=6, spec=SurfaceSpec(curved=True), kernel="S",
                         p_qbx=q, p_fmm=q, density="ones")
    coarse = make_workload("coarse", level=2, order=4, spec=SurfaceSpec(curved=True),
                           kernel="S", p_qbx=q, p_fmm=q, density="ones")
    idx = l * l + l + m
    dens = real_sh_basis(l, fine.src_xyz)[idx]
    rng = np.random.default_rng(seed)
    cids = np.sort(rng.choice(coarse.n_ctr, n_sample, replace=False))
    tgt = coarse.tgt_xyz[cids]
    tn = coarse.src_normal[cids // 2]  # outward normal at each target's base node
    d = O.direct_qbx_sprime(q, fine.src_xyz, fine.src_w * dens, coarse.ctr_xyz[cids], tgt,
                            np.arange(len(cids)), tn)
    return d, real_sh_basis(l, tgt)[idx], (cids % 2) == 0


@pytest.mark.parametrize("l,m", [(1, 0), (2, 1), (3, -2)])
def test_sprime_sphere_eigenrelation(l, m):
    """S[Y_l] is r^l Y/(2l+1) inside and r^-(l+1) Y/(2l+1) outside the unit sphere, so its
    radial derivative on the surface is l/(2l+1) Y from inside and -(l+1)/(2l+1) Y from
    outside."""
    d, y, ext = _sphere_sprime(5, l, m)
    scale = np.abs(y).max()
    assert np.abs(d[~ext] - l / (2 * l + 1) * y[~ext]).max() / scale < 1e-6
    assert np.abs(d[ext] + (l + 1) / (2 * l + 1) * y[ext]).max() / scale < 5e-3


def test_local_normal_derivative_matches_finite_differences():
    rng = np.random.default_rng(8)
    p = 6
    src = rng.uniform(-1, 1, (20, 3)) * 0.3 + np.array([2.0, 0.5, -1.0])
    c = np.array([0.1, -0.2, 0.05])
    L = O.p2l("S", p, src, rng.standard_normal(20), c)
    for _ in range(5):
        t = c + rng.uniform(-0.3, 0.3, 3)
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        h = 1e-3
        f = [O.eval_local(p, L, c, t + k * h * n) for k in (-2, -1, 1, 2)]
        fd = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)
        assert abs(O.local_normal_derivative(p, L, c, t, n) - fd) <= 1e-9 * max(1.0, abs(fd))
