"""Several densities per apply: the double layer's near field takes them two at a time.

For the double layer up to p_qbx = 5 the two-density near-field kernel shares each
(source, center) pair's solid harmonics between two densities; every other stage, and the
other kernels and orders, run once per density.  Three densities exercise a pair and a
single.  Checks, on deterministic plans so that the far field adds in a fixed order:
* the multi-density apply equals one-density applies bit for bit (the two-density kernel's
  per-density arithmetic is the one-density kernel's);
* every density against the step-by-step oracle (Tier B) at the parity bar 1e-10;
* the QBX locals exported after the apply are the last density's.
"""

import numpy as np
import pytest

import oracle as O  # noqa: F401  (builds the oracle library for the fixture)
from oracle.gigaqbx import OracleFMM
from workloads import workload_tiny

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

CASES = {
    "D-l1-n32": dict(level=1, order=2, kernel="D", p_qbx=3, p_fmm=6, nmax=32),
    "D-l2-q5p15": dict(level=2, order=2, kernel="D", p_qbx=5, p_fmm=15, nmax=48),
    "S-l2-q8p20": dict(level=2, order=2, kernel="S", p_qbx=8, p_fmm=20, nmax=48),
    # one density per pass: the single layer, and the double layer beyond q = 5
    "S-l1-q9p12": dict(level=1, order=2, kernel="S", p_qbx=9, p_fmm=12, nmax=32),
    "D-l1-q6p10": dict(level=1, order=2, kernel="D", p_qbx=6, p_fmm=10, nmax=32),
}


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU test without a GPU"
    import paper_1805_06106_amd  # noqa: F401  (fails loudly if the library is missing)

    return torch.device("cuda:0")


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("case", sorted(CASES))
def test_densities_in_pairs(dev, case):
    import torch

    from paper_1805_06106_amd import Plan

    w = workload_tiny(n_densities=3, **CASES[case])
    nd = w.density.shape[0]
    print(f"[gpu] densities case={case} n_densities={nd} n_src={w.n_src}", flush=True)
    P = Plan.from_workload(w, n_densities=nd, deterministic=True)
    many = P.apply(torch.tensor(w.density, device=dev)).cpu().numpy()
    last_locals = P.qbx_locals()
    one = Plan.from_workload(w, n_densities=1, deterministic=True)
    F = OracleFMM(w)
    for d in range(nd):
        single = one.apply(torch.tensor(w.density[d:d + 1], device=dev)).cpu().numpy()[0]
        assert np.array_equal(many[d], single), f"density {d} differs from its own apply"
        tids, ref, _ = F.evaluate(density_index=d)
        assert rel(many[d][tids], ref) < 1e-10
    # after the loop, `one` holds the last density's locals
    assert np.array_equal(last_locals, one.qbx_locals())
    P.close()
    one.close()
