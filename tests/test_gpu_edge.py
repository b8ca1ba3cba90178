"""Edge cases through the C ABI on the GPU: the largest orders the build supports, order-0
expansions, a single source, no QBX targets, all-point targets, one center per box, and
strongly ragged boxes; each against the oracle."""

import numpy as np
import pytest

import oracle as O
from oracle.gigaqbx import OracleFMM
from workloads import add_point_targets, workload_tiny

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _run(w, **kw):
    import torch

    import paper_1805_06106_amd  # noqa: F401
    from paper_1805_06106_amd import Plan

    P = Plan.from_workload(w, n_densities=w.density.shape[0], **kw)
    pot = P.apply(torch.tensor(w.density, dtype=torch.float64, device="cuda:0"))
    torch.cuda.synchronize()
    return pot.cpu().numpy()


@pytest.mark.parametrize("kernel", ["S", "D"])
def test_max_orders(kernel):
    w = workload_tiny(level=1, order=2, kernel=kernel, p_qbx=10, p_fmm=20, nmax=32)
    print(f"[gpu] max orders {kernel}", flush=True)
    pot = _run(w)
    tids, ref, _ = OracleFMM(w).evaluate()
    assert rel(pot[0][tids], ref) < 1e-10


@pytest.mark.parametrize("p_qbx,p_fmm", [(0, 0), (0, 3), (3, 3)])
def test_low_orders(p_qbx, p_fmm):
    w = workload_tiny(level=1, order=2, kernel="D", p_qbx=p_qbx, p_fmm=p_fmm, nmax=32)
    print(f"[gpu] orders {p_qbx}/{p_fmm}", flush=True)
    pot = _run(w)
    tids, ref, _ = OracleFMM(w).evaluate()
    assert rel(pot[0][tids], ref) < 1e-10


def test_single_source():
    import dataclasses

    w = workload_tiny(level=1, order=2, kernel="S", p_qbx=3, p_fmm=6, nmax=32)
    w = dataclasses.replace(w, src_xyz=w.src_xyz[:1], src_w=w.src_w[:1],
                            src_normal=w.src_normal[:1], src_dir=w.src_dir[:1],
                            density=w.density[:, :1])
    print("[gpu] single source", flush=True)
    pot = _run(w)
    ref, _ = O.direct_qbx("S", w.p_qbx, w.src_xyz, O.strengths(w)[0], w.ctr_xyz, w.tgt_xyz,
                          w.tgt_center)
    tids, refb, _ = OracleFMM(w).evaluate()
    assert rel(pot[0][tids], refb) < 1e-10
    assert rel(pot[0], ref) <= 0.75 ** (w.p_fmm + 1)  # acceleration error (Theorem 1)


def test_only_point_targets_and_no_targets():
    import dataclasses

    base = workload_tiny(level=2, order=1, kernel="S", p_qbx=2, p_fmm=6, nmax=24)
    w = add_point_targets(base, n_out=60, n_in=30)
    w = dataclasses.replace(w, tgt_xyz=w.tgt_xyz[base.n_tgt:], tgt_center=w.tgt_center[base.n_tgt:])
    print("[gpu] only point targets", flush=True)
    pot = _run(w)
    tids, ref = OracleFMM(w).evaluate_points()
    assert len(tids) == 90
    assert rel(pot[0][tids], ref) < 1e-10
    w0 = dataclasses.replace(base, tgt_xyz=np.zeros((0, 3)),
                             tgt_center=np.zeros(0, dtype=np.int64))
    print("[gpu] no targets", flush=True)
    assert _run(w0).shape == (1, 0)


def test_one_center_per_leaf_and_deep_ragged_tree():
    """nmax = 1 forces the deepest tree the particles allow (ragged, many suspended
    centers); t_f = 0 makes centers descend only when their ball fits the child's own
    sphere."""
    for tcf in (0.0, 0.9):
        w = workload_tiny(level=1, order=1, kernel="D", p_qbx=2, p_fmm=5, nmax=1, tcf=tcf)
        print(f"[gpu] nmax=1 tcf={tcf}", flush=True)
        pot = _run(w)
        tids, ref, _ = OracleFMM(w).evaluate()
        assert rel(pot[0][tids], ref) < 1e-10


def test_device_memory_cap():
    """A plan over its device-memory cap is refused with GQ_ENOMEM and nothing else happens;
    at a cap equal to what the plan holds it is created and evaluates as without a cap."""
    import torch

    import paper_1805_06106_amd as G
    from paper_1805_06106_amd import Plan

    w = workload_tiny(level=2, order=2, kernel="D", p_qbx=3, p_fmm=8, nmax=32)
    print("[gpu] device memory cap", flush=True)
    P0 = Plan.from_workload(w)
    need = P0.stats()["device_bytes"]
    assert need > 0
    for cap in (1, need // 2, need - 1):
        with pytest.raises(G.GQError) as e:
            Plan.from_workload(w, max_device_bytes=cap)
        assert e.value.status == 2 and "cap" in str(e.value)
    P1 = Plan.from_workload(w, max_device_bytes=need)
    assert P1.stats()["device_bytes"] == need
    d = torch.tensor(w.density, dtype=torch.float64, device="cuda:0")
    p0, p1 = P0.apply(d), P1.apply(d)
    torch.cuda.synchronize()
    # equal up to the order of the translations' atomic additions
    assert rel(p1.cpu().numpy(), p0.cpu().numpy()) < 1e-14
    # the refused creations left the device usable and the existing plans intact
    assert rel(P0.apply(d).cpu().numpy(), p0.cpu().numpy()) < 1e-14


def test_autotuned_tree():
    """GQ_FLAG_AUTOTUNE_TREE builds and times candidate trees and keeps one of them; the
    plan it returns evaluates like any plan with the kept parameters (against Tier B built
    with them)."""
    import torch

    from paper_1805_06106_amd import Plan

    w = workload_tiny(level=2, order=2, kernel="D", p_qbx=5, p_fmm=15, nmax=48)
    print("[gpu] autotuned tree", flush=True)
    P = Plan.from_workload(w, autotune_tree=True, wfar_direct_max=16, level_restrict=True)
    st = P.stats()
    assert st["nmax"] in (24, 36, 48, 72), st["nmax"]
    assert st["wfar_direct_max"] in (8, 16, 32), st["wfar_direct_max"]
    pot = P.apply(torch.tensor(w.density, dtype=torch.float64, device="cuda:0")).cpu().numpy()
    F = OracleFMM(w, nmax=st["nmax"], wfar_direct_max=st["wfar_direct_max"], level_restrict=True)
    tids, ref, _ = F.evaluate()
    assert rel(pot[0][tids], ref) < 1e-10
    P.close()
