"""CPU tests of the iterative solver and of the oversampled (stage-2 quadrature)
discretization used for boundary value problems.

* GMRES and GMRES with two-precision iterative refinement on dense systems, against
  numpy's direct solve.
* The oversampled input set: the node lattice is unisolvent and the interpolation exact on
  polynomials, the subdivided rule integrates monomials exactly, and through the oracle's
  direct QBX the interior double layer of the unit density reproduces Gauss's law far
  better with the oversampled quadrature than without (the reason the paper evaluates
  layer potentials on the stage-2 quadrature discretization, Section 3).
"""

import numpy as np
import pytest
import torch

import oracle as O
from paper_1805_06106_amd.solve import gmres, gmres_ir
from workloads import make_workload, oversampled_workload
from workloads.geometry import (SurfaceSpec, interior_lattice, lattice_interpolation,
                                subdivided_rule)


def _system(n=120, seed=0):
    rng = np.random.default_rng(seed)
    K = rng.standard_normal((n, n)) * (0.35 / np.sqrt(n))
    A = -0.5 * np.eye(n) + K  # second-kind: spectrum clustered around -1/2
    b = rng.standard_normal(n)
    return torch.from_numpy(A), torch.from_numpy(b)


def test_gmres_matches_direct_solve():
    A, b = _system()
    x, k, hist = gmres(lambda v: A @ v, b, tol=1e-13, maxiter=200, restart=200)
    ref = np.linalg.solve(A.numpy(), b.numpy())
    assert np.max(np.abs(x.numpy() - ref)) / np.max(np.abs(ref)) < 1e-11
    assert k < 100 and hist[-1] <= 1e-13
    assert all(h2 <= h1 * (1 + 1e-12) for h1, h2 in zip(hist, hist[1:]))  # GMRES is monotone


def test_gmres_restarted_and_budget():
    A, b = _system(seed=1)
    x, k, _ = gmres(lambda v: A @ v, b, tol=1e-12, maxiter=300, restart=7)
    assert float(torch.linalg.vector_norm(b - A @ x) / torch.linalg.vector_norm(b)) < 1e-11
    x, k, hist = gmres(lambda v: A @ v, b, tol=1e-14, maxiter=5, restart=50)
    assert k == 5 and hist[-1] > 1e-14
    x, k, hist = gmres(lambda v: A @ v, torch.zeros_like(b), tol=1e-10)
    assert k == 0 and float(x.abs().max()) == 0.0


def test_gmres_ir_reaches_the_accurate_residual():
    """Inner applies in FP32 (relative error ~1e-7) cannot alone reach 1e-12; refinement
    with FP64 residuals does, in a few outer steps."""
    A, b = _system(seed=2)
    A32 = A.float()
    lo = lambda v: (A32 @ v.float()).double()  # noqa: E731
    hi = lambda v: A @ v  # noqa: E731
    _, _, hist = gmres(lo, b, tol=1e-13, maxiter=100)
    x, info = gmres_ir(lo, hi, b, tol=1e-12, inner_tol=1e-5, max_applies=200)
    res = float(torch.linalg.vector_norm(b - A @ x) / torch.linalg.vector_norm(b))
    assert info["converged"] and res <= 1e-12
    assert res == pytest.approx(info["outer_residuals"][-1], rel=1e-6)
    assert 2 <= info["applies_hi"] <= 4
    assert info["applies_lo"] > 3 * info["applies_hi"]
    x, info = gmres_ir(lo, hi, b, tol=1e-14, inner_tol=1e-5, max_applies=12)
    assert not info["converged"] and info["applies_lo"] + info["applies_hi"] <= 12


@pytest.mark.parametrize("order", [2, 4, 6])
def test_lattice_unisolvent_and_interpolation_exact(order):
    xn, yn = interior_lattice(order)
    assert len(xn) == (order + 1) * (order + 2) // 2
    assert np.all(yn > 0) and np.all(xn - yn > 0) and np.all(xn < 1)  # strictly inside
    xq, yq, _ = subdivided_rule(4, 3)
    M = lattice_interpolation(order, xq, yq)
    rng = np.random.default_rng(order)
    for _ in range(3):  # a random polynomial of total degree `order`
        c = rng.standard_normal((order + 1, order + 1))
        f = lambda x, y: sum(c[i, j] * x ** i * y ** j  # noqa: E731
                             for i in range(order + 1) for j in range(order + 1 - i))
        assert np.max(np.abs(M @ f(xn, yn) - f(xq, yq))) < 1e-11
    assert np.allclose(M.sum(axis=1), 1.0, atol=1e-12)  # constants are reproduced


@pytest.mark.parametrize("order,sub", [(2, 1), (4, 2), (4, 4)])
def test_subdivided_rule_exact_on_monomials(order, sub):
    """Integral of x^i y^j over {0 <= y <= x <= 1} is 1 / ((j+1)(i+j+2))."""
    x, y, w = subdivided_rule(order, sub)
    assert len(w) == sub * sub * (order + 1) * ((order + 2) // 2)
    assert np.all(w > 0) and np.all(y >= 0) and np.all(y <= x) and np.all(x <= 1)
    for i in range(order + 2):
        for j in range(order + 2 - i):
            exact = 1.0 / ((j + 1) * (i + j + 2))
            assert abs(np.sum(w * x ** i * y ** j) - exact) < 1e-14, (i, j)


def test_oversampling_sharpens_gauss_law():
    """D[1] = -1 at interior targets (Gauss's law).  Through interior QBX centers with
    p_qbx = 5, the unit density on a curved sphere (80 elements) misses it by about 0.1 with
    one 15-node rule per element, and by about 2e-5 with the 16x subdivided rule."""
    spec = SurfaceSpec(curved=True)
    w0 = make_workload("plain", level=1, order=4, spec=spec, kernel="D", p_qbx=5, p_fmm=10,
                       density="ones")
    ws = oversampled_workload("over", level=1, spec=spec, kernel="D", p_qbx=5, p_fmm=10,
                              sides="interior", node_order=4, quad_order=4, sub=4)
    ws.density = np.ones_like(ws.density)
    inner = np.arange(1, w0.n_ctr, 2)
    pot0, _ = O.direct_qbx("D", 5, w0.src_xyz, O.strengths(w0)[0], w0.ctr_xyz, w0.tgt_xyz[inner],
                           inner, nrm=w0.src_normal)
    pots, _ = O.direct_qbx("D", 5, ws.src_xyz, O.strengths(ws)[0], ws.ctr_xyz, ws.tgt_xyz,
                           ws.tgt_center, nrm=ws.src_normal)
    e0 = np.max(np.abs(pot0 + 1.0))
    es = np.max(np.abs(pots + 1.0))
    print(f"Gauss's law error: single rule {e0:.2e}, oversampled {es:.2e}")
    assert e0 > 1e-2
    assert es < 1e-4 and es < e0 / 1000
