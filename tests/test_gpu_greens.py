"""Green's formula through the library (the accuracy experiment of Section 6.1, at small
size): for u the potential of a unit charge outside the surface, S(du/dn) - D(u) = u at the
interior-side limit.  The residual must fall as p_fmm grows and stay under the a-priori
acceleration factor (3/4)^(p_fmm+1) once p_fmm exceeds p_qbx; with a single box (no
acceleration) it is the plain QBX error."""

import numpy as np
import pytest

from workloads import workload_tiny

pytestmark = pytest.mark.gpu


def _residual(w, p_fmm, p_qbx, nmax):
    import torch

    import paper_1805_06106_amd  # noqa: F401
    from paper_1805_06106_amd import Plan

    x0 = np.array([3.0, 1.0, 2.0])
    d = w.src_xyz - x0
    r = np.linalg.norm(d, axis=1)
    u = 1.0 / r
    dudn = -np.sum(d * w.src_normal, axis=1) / r ** 3
    pots = {}
    for kern, dens in (("S", dudn), ("D", u)):
        P = Plan.from_workload(w, kernel=kern, p_fmm=p_fmm, p_qbx=p_qbx, nmax=nmax)
        pots[kern] = P.apply(torch.tensor(dens[None, :], device="cuda:0"))[0].cpu().numpy()
    inner = np.arange(1, w.n_tgt, 2)
    E = pots["S"][inner] - pots["D"][inner] - u[inner // 2]
    return float(np.max(np.abs(E)) / np.max(np.abs(u)))


def test_greens_formula_residual_pattern():
    w = workload_tiny(level=3, order=4, kernel="S", p_qbx=3, p_fmm=10, nmax=64)
    print(f"[gpu] greens n_src={w.n_src}", flush=True)
    plain = _residual(w, 10, 3, nmax=10 ** 7)  # one box: unaccelerated QBX
    errs = {p: _residual(w, p, 3, nmax=64) for p in (3, 5, 10, 15)}
    print(f"[gpu] greens plain {plain:.3e} accelerated {errs}", flush=True)
    for p, e in errs.items():
        assert abs(e - plain) <= 0.75 ** (p + 1)
    assert abs(errs[15] - plain) <= 1e-3 * plain + 1e-12
    assert errs[3] >= errs[15]
