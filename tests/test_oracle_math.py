"""Pins for the oracle's special functions, expansions and translations.

Each test checks the oracle against something other than itself: a library routine, a
closed form, an identity of the paper, or an a-priori bound the paper states.
"""

import json
import math
import os

import numpy as np
import pytest
import scipy.special as sp

import oracle as O

pytestmark = pytest.mark.usefixtures("oracle_lib")
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
RNG = np.random.default_rng(12345)


def G(a, b):
    return 1.0 / (4.0 * math.pi * np.linalg.norm(np.asarray(a) - np.asarray(b)))


def _unit(v):
    v = np.asarray(v, dtype=float)
    return v / np.linalg.norm(v)


# --- Y_n^m --------------------------------------------------------------------------------

@pytest.mark.parametrize("v", [RNG.standard_normal(3) for _ in range(4)] + [np.array([0.0, 0.0, 2.0]),
                                                                          np.array([0.0, 0.0, -0.5])])
def test_ylm_matches_scipy(v):
    """Section 2.1's Y_n^m vs scipy (which carries the Condon-Shortley phase (-1)^m, m>0)."""
    p = 12
    Y = O.ylm(p, v)
    r = np.linalg.norm(v)
    th, ph = np.arccos(v[2] / r), np.arctan2(v[1], v[0])
    for n in range(p + 1):
        for m in range(-n, n + 1):
            ref = sp.sph_harm_y(n, m, th, ph) * ((-1) ** m if m > 0 else 1)
            assert abs(Y[O.cidx(n, m)] - ref) < 1e-13


def test_ylm_conjugate_symmetry():
    Y = O.ylm(10, RNG.standard_normal(3))
    for n in range(11):
        for m in range(1, n + 1):
            assert abs(Y[O.cidx(n, -m)] - np.conj(Y[O.cidx(n, m)])) < 1e-15


def test_addition_identity_for_G():
    """Section 2.1, spherical-harmonic expansion of G(a, b) for |a| < |b|, summed to n=40."""
    a = 0.4 * _unit(RNG.standard_normal(3))
    b = 1.0 * _unit(RNG.standard_normal(3))
    p = 40
    Ya, Yb = O.ylm(p, a), O.ylm(p, b)
    ra, rb = np.linalg.norm(a), np.linalg.norm(b)
    s = 0.0
    for n in range(p + 1):
        inner = sum(Ya[O.cidx(n, m)] * Yb[O.cidx(n, -m)] for m in range(-n, n + 1))
        s += inner * ra ** n / rb ** (n + 1) / (2 * n + 1)
    assert abs(s.imag) < 1e-15
    assert abs(s.real - G(a, b)) < 1e-15


# --- expansions vs Proposition 1 ---------------------------------------------------------

@pytest.mark.parametrize("p", [3, 6, 10, 15, 20])
def test_local_expansion_prop1(p):
    """Proposition 1(a): |G - L_p| <= (1/4pi) (rho - r)^-1 (r/rho)^(p+1)."""
    c = RNG.standard_normal(3) * 0.1
    for _ in range(20):
        s = c + 1.0 * _unit(RNG.standard_normal(3))
        t = c + 0.6 * RNG.uniform() * _unit(RNG.standard_normal(3))
        L = O.p2l("S", p, s, [1.0], c)
        rho, r = np.linalg.norm(s - c), np.linalg.norm(t - c)
        bound = (1.0 / (4 * math.pi)) / (rho - r) * (r / rho) ** (p + 1)
        assert abs(O.eval_local(p, L, c, t) - G(s, t)) <= bound * 1.0000001 + 4e-15 * G(s, t)


@pytest.mark.parametrize("p", [3, 6, 10, 15, 20])
def test_multipole_expansion_prop1(p):
    """Proposition 1(b) for the multipole expansion of Section 4.2."""
    c = RNG.standard_normal(3) * 0.1
    for _ in range(20):
        s = c + 0.6 * RNG.uniform() * _unit(RNG.standard_normal(3))
        t = c + 1.0 * _unit(RNG.standard_normal(3))
        M = O.p2m("S", p, s, [1.0], c)
        r, rho = np.linalg.norm(s - c), np.linalg.norm(t - c)
        bound = (1.0 / (4 * math.pi)) / (rho - r) * (r / rho) ** (p + 1)
        assert abs(O.eval_mpole(p, M, c, t) - G(s, t)) <= bound * 1.0000001 + 4e-15 * G(s, t)


def test_double_layer_coefficients_are_normal_derivatives():
    """D coefficients = n_s . grad_s of S coefficients: check by 4th-order central
    differences of the S-coefficient function, and against dG/dn_y at a target."""
    p = 8
    c = np.zeros(3)
    s = np.array([0.7, -0.4, 0.5])
    n = _unit([0.3, 0.8, -0.2])
    h = 1e-3
    fd = (-O.p2l("S", p, s + 2 * h * n, [1.0], c) + 8 * O.p2l("S", p, s + h * n, [1.0], c)
          - 8 * O.p2l("S", p, s - h * n, [1.0], c) + O.p2l("S", p, s - 2 * h * n, [1.0], c)) / (12 * h)
    D = O.p2l("D", p, s, [1.0], c, nrm=n)
    assert np.max(np.abs(D - fd)) < 1e-8 * np.max(np.abs(D))
    fdm = (-O.p2m("S", p, s + 2 * h * n, [1.0], c) + 8 * O.p2m("S", p, s + h * n, [1.0], c)
           - 8 * O.p2m("S", p, s - h * n, [1.0], c) + O.p2m("S", p, s - 2 * h * n, [1.0], c)) / (12 * h)
    Dm = O.p2m("D", p, s, [1.0], c, nrm=n)
    assert np.max(np.abs(Dm - fdm)) < 1e-8 * np.max(np.abs(Dm))
    # full expansion converges to the double-layer kernel dG/dn_y = n.(x - y)/(4 pi |x-y|^3)
    t = np.array([0.05, 0.02, -0.04])
    dG = np.dot(n, t - s) / (4 * math.pi * np.linalg.norm(t - s) ** 3)
    L = O.p2l("D", 25, s, [1.0], c, nrm=n)
    assert abs(O.eval_local(25, L, c, t) - dG) < 1e-14


def test_double_layer_at_pole():
    """Gradient formula stays finite on the polar axis (sin(theta) = 0)."""
    c = np.zeros(3)
    s = np.array([0.0, 0.0, 0.8])
    n = _unit([1.0, 0.5, 0.2])
    t = np.array([0.02, -0.03, 0.01])
    dG = np.dot(n, t - s) / (4 * math.pi * np.linalg.norm(t - s) ** 3)
    L = O.p2l("D", 30, s, [1.0], c, nrm=n)
    assert np.all(np.isfinite(L))
    assert abs(O.eval_local(30, L, c, t) - dG) < 1e-13


def test_local_real_symmetry():
    """Real sources give L_n^-m = conj(L_n^m)."""
    L = O.p2l("S", 7, RNG.standard_normal((5, 3)) + 3, RNG.standard_normal(5), np.zeros(3))
    for n in range(8):
        for m in range(1, n + 1):
            assert abs(L[O.cidx(n, -m)] - np.conj(L[O.cidx(n, m)])) < 1e-14 * np.abs(L).max()


# --- translations -----------------------------------------------------------------------

@pytest.mark.parametrize("kernel", ["S", "D"])
def test_m2m_exact(kernel):
    """Shifting an order-p multipole keeps its degrees <= p exactly: equals direct P2M."""
    p = 10
    src = RNG.standard_normal((6, 3)) * 0.2
    nrm = np.array([_unit(x) for x in RNG.standard_normal((6, 3))])
    q = RNG.standard_normal(6)
    c1, c2 = np.array([0.05, 0.02, -0.03]), np.array([0.4, -0.3, 0.2])
    M1 = O.p2m(kernel, p, src, q, c1, nrm=nrm)
    M2 = O.p2m(kernel, p, src, q, c2, nrm=nrm)
    assert np.max(np.abs(O.m2m(p, M1, c1, c2) - M2)) < 1e-13 * np.max(np.abs(M2))


def test_l2l_exact_and_truncation_consistent():
    """An order-p local is a degree-p harmonic polynomial: p->p L2L is exact; p->q keeps the
    first (q+1)^2 coefficients of p->p."""
    p, q = 9, 4
    src = np.array([[2.0, 1.0, -1.5], [-1.8, 2.2, 0.7]])
    c0 = np.zeros(3)
    L = O.p2l("S", p, src, [1.0, -0.7], c0)
    c1 = np.array([0.2, -0.1, 0.15])
    L1 = O.l2l(p, p, L, c0, c1)
    for _ in range(10):
        t = RNG.standard_normal(3) * 0.3
        assert abs(O.eval_local(p, L1, c1, t) - O.eval_local(p, L, c0, t)) < 1e-15
    Lq = O.l2l(p, q, L, c0, c1)
    assert np.max(np.abs(Lq - L1[:O.ncoef(q)])) < 1e-16 * 10 * np.max(np.abs(L1))


def test_l2l_projection_on_sphere():
    """L2L coefficients equal the projection of the polynomial onto Y_n^m on a sphere around
    the new center (an exact Gauss-Legendre x trapezoid rule), computed with scipy."""
    p = 6
    c0 = np.zeros(3)
    L = O.p2l("S", p, np.array([[1.5, -0.7, 0.9]]), [1.0], c0)
    c1 = np.array([0.1, 0.2, -0.1])
    L1 = O.l2l(p, p, L, c0, c1)
    rad = 0.3
    nt, nph = p + 2, 2 * p + 3
    x, wx = np.polynomial.legendre.leggauss(nt)
    ph = 2 * np.pi * np.arange(nph) / nph
    TH, PH = np.meshgrid(np.arccos(x), ph, indexing="ij")
    W = np.repeat(wx[:, None], nph, axis=1) * (2 * np.pi / nph)
    pts = c1 + rad * np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1)
    vals = np.vectorize(lambda i, j: O.eval_local(p, L, c0, pts[i, j]))(*np.indices(TH.shape))
    for n in range(p + 1):
        for m in range(-n, n + 1):
            Y = sp.sph_harm_y(n, abs(m), TH, PH)
            Y = (np.conj(Y) if m < 0 else Y) * ((-1) ** abs(m))  # remove CS phase
            coef = np.sum(W * vals * np.conj(Y)) / rad ** n
            assert abs(coef - L1[O.cidx(n, m)]) < 1e-12 * max(1.0, abs(L1[O.cidx(n, m)]))


@pytest.mark.parametrize("p", [4, 8, 16])
def test_m2l_converges_to_direct_local(p):
    """M2L of an order-p multipole tends to the direct local expansion (Section 4.3.1's
    limit), at the rate of Proposition 1."""
    q = 5
    s = np.array([0.1, -0.05, 0.08])
    c = np.zeros(3)
    c2 = np.array([2.0, 0.5, -0.3])
    Ld = O.p2l("S", q, s, [1.0], c2)
    Lt = O.m2l(p, q, O.p2m("S", p, s, [1.0], c), c, c2)
    t = c2 + np.array([0.05, 0.1, -0.02])
    r = np.linalg.norm(s - c)
    rho = np.linalg.norm(t - c)
    bound = (1.0 / (4 * math.pi)) / (rho - r) * (r / rho) ** (p + 1)
    assert abs(O.eval_local(q, Lt, c2, t) - O.eval_local(q, Ld, c2, t)) <= 1.01 * bound + 1e-16


def test_addition_theorems_RI():
    """R(x+y) = sum R_j^k(x) R_{n-j}^{m-k}(y) and I(X-y) = sum conj(R_j^k(y)) I_{n+j}^{m+k}(X)."""
    p = 8
    x, y = RNG.standard_normal(3) * 0.3, RNG.standard_normal(3) * 0.3
    Rx, Ry, Rxy = O.regular_RI(p, x), O.regular_RI(p, y), O.regular_RI(p, x + y)

    def g(a, n, m, pp):
        return a[O.cidx(n, m)] if 0 <= n <= pp and abs(m) <= n else 0.0

    for n in range(p + 1):
        for m in range(-n, n + 1):
            s = sum(g(Rx, j, k, p) * g(Ry, n - j, m - k, p) for j in range(n + 1) for k in range(-j, j + 1))
            assert abs(s - Rxy[O.cidx(n, m)]) < 1e-14
    X = np.array([1.2, -0.8, 0.9])
    y = RNG.standard_normal(3) * 0.1
    K = 40
    IX, Ry, IXy = O.irregular_RI(K + 3, X), O.regular_RI(K, y), O.irregular_RI(3, X - y)
    for n in range(4):
        for m in range(-n, n + 1):
            s = sum(np.conj(g(Ry, j, k, K)) * g(IX, n + j, m + k, K + 3)
                    for j in range(K - 3) for k in range(-j, j + 1))
            assert abs(s - IXy[O.cidx(n, m)]) < 1e-12 * abs(IXy[O.cidx(n, m)]) + 1e-14


# --- Section 4.3 hypotheses on a sample of Appendix B's grid -------------------------------

def _sphere_pts(k, seed):
    r = np.random.default_rng(seed)
    v = r.standard_normal((k, 3))
    v = np.concatenate([v / np.linalg.norm(v, axis=1)[:, None], [[0, 0, 1.0], [0, 0, -1.0]]])
    return v


@pytest.mark.parametrize("R,rho,rr", [(1.0, 1.0, 0.5), (0.1, 10.0, 0.75), (10.0, 1.0, 0.25)])
def test_hypothesis1_m2qbxl(R, rho, rr):
    """Hypothesis 1 (source -> multipole(p) -> local(q)) with the paper's constant 1.002:
    max over samples of E_M(q) / bound <= C."""
    C = GOLD["hypothesis_constants"]["m2qbxl"]
    r = rr * rho
    c = np.array([0.0, 0.0, R + rho])
    worst = 0.0
    for p in (3, 5, 10):
        for q in (3, 5, 10):
            bound = (1 / (4 * math.pi)) / (rho - r) * (r / rho) ** (p + 1)
            for s in c + r * _sphere_pts(4, 1):
                M = O.p2m("S", p, s, [1.0], c)
                for cp in _sphere_pts(3, 2) * R * 0.5:
                    Lt = O.m2l(p, q, M, c, cp)
                    Ld = O.p2l("S", q, s, [1.0], cp)
                    for t in cp + (R - np.linalg.norm(cp)) * _sphere_pts(3, 3):
                        e = abs(O.eval_local(q, Lt, cp, t) - O.eval_local(q, Ld, cp, t))
                        worst = max(worst, e / bound)
    assert worst <= C


@pytest.mark.parametrize("rho,rr", [(1.0, 0.5), (10.0, 0.75), (0.1, 0.25)])
def test_hypothesis2_l2qbxl(rho, rr):
    """Hypothesis 2 (source -> local(p) -> local(q)) with the paper's constant 1.001."""
    C = GOLD["hypothesis_constants"]["l2qbxl"]
    r = rr * rho
    s = np.array([0.0, 0.0, rho])
    worst = 0.0
    for p in (3, 5, 10):
        L0 = O.p2l("S", p, s, [1.0], np.zeros(3))
        for q in (3, 5, 10):
            bound = (1 / (4 * math.pi)) / (rho - r) * (r / rho) ** (p + 1)
            for cc in _sphere_pts(3, 4) * r * 0.5:
                Lt = O.l2l(p, q, L0, np.zeros(3), cc)
                Ld = O.p2l("S", q, s, [1.0], cc)
                for t in cc + (r - np.linalg.norm(cc)) * _sphere_pts(4, 5):
                    e = abs(O.eval_local(q, Lt, cc, t) - O.eval_local(q, Ld, cc, t))
                    worst = max(worst, e / bound)
    assert worst <= C


def test_hypothesis3_m2l2qbxl():
    """Hypothesis 3 (source -> multipole(p) -> local(p) -> local(q)), constant 1.001."""
    C = GOLD["hypothesis_constants"]["m2l2qbxl"]
    R, rho, rr = 1.0, 1.0, 0.5
    r = rr * rho
    c = np.array([0.0, 0.0, R + rho])
    worst = 0.0
    for p in (3, 5, 10):
        for q in (3, 5):
            bound = (1 / (4 * math.pi)) * ((1 / (rho - r)) * (R / (R + rho - r)) ** (p + 1)
                                           + (1 / (rho - r)) * (r / rho) ** (p + 1))
            for s in c + r * _sphere_pts(3, 6):
                L0 = O.m2l(p, p, O.p2m("S", p, s, [1.0], c), c, np.zeros(3))
                for cp in _sphere_pts(3, 7) * R * 0.5:
                    Lt = O.l2l(p, q, L0, np.zeros(3), cp)
                    Ld = O.p2l("S", q, s, [1.0], cp)
                    for t in cp + (R - np.linalg.norm(cp)) * _sphere_pts(3, 8):
                        e = abs(O.eval_local(q, Lt, cp, t) - O.eval_local(q, Ld, cp, t))
                        worst = max(worst, e / bound)
    assert worst <= C


def test_theorem1_factor_constants():
    """Theorem 1's convergence factor: 3/4 for t_f <= (6 sqrt3 - 7)/4 and 0.771 at 0.9."""
    g = GOLD["theorem1"]

    def factor(tf):
        return max(math.sqrt(3) * (1 + tf) / (6 - math.sqrt(3)), math.sqrt(3) / 3)

    assert abs((6 * math.sqrt(3) - 7) / 4 - g["tf_threshold"]) < 1e-4
    assert abs(factor((6 * math.sqrt(3) - 7) / 4) - 0.75) < 1e-12
    assert abs(factor(0.9) - g["factor_at_tf_0.9"]) < 1e-4
    col = GOLD["table3_bound_column"]
    for p, b in zip(col["p_fmm"], col["bound"]):
        assert abs(0.75 ** (p + 1) - b) / b < 5e-3
