"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerance: the stated bar for the FP64 path is 1e-8 relative (l-inf error over l-inf norm of
the oracle's result, per density); the tests assert 1e-10, which the two FP64
implementations (different formula routes, same arithmetic precision) meet with margin.
"""

import math

import numpy as np
import pytest

import oracle as O
from oracle.gigaqbx import OracleFMM
from workloads import workload_c1, workload_tiny

import gq_convert as CV

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]
TOL = 1e-10

CASES = {
    "S-l1-n32": dict(level=1, order=2, kernel="S", p_qbx=3, p_fmm=6, nmax=32),
    "D-l1-n32": dict(level=1, order=2, kernel="D", p_qbx=3, p_fmm=6, nmax=32),
    "S-l2-tf05": dict(level=2, order=1, kernel="S", p_qbx=2, p_fmm=5, nmax=24, tcf=0.5),
    "D-l2-flat": dict(level=2, order=1, kernel="D", p_qbx=2, p_fmm=5, nmax=40, curved=False),
    "D-l2-q5p15": dict(level=2, order=2, kernel="D", p_qbx=5, p_fmm=15, nmax=48),
    # smallest M2QBXL table (p <= 8) at q = 5: the waves' sums are combined in two rounds
    "D-l2-q5p8": dict(level=2, order=2, kernel="D", p_qbx=5, p_fmm=8, nmax=32),
    "S-l2-q8p20": dict(level=2, order=2, kernel="S", p_qbx=8, p_fmm=20, nmax=48),
}


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU test without a GPU"
    import paper_1805_06106_amd  # noqa: F401  (fails loudly if the library is missing)

    return torch.device("cuda:0")


def run_gpu(w, dev, **kw):
    import torch

    from paper_1805_06106_amd import Plan

    P = Plan.from_workload(w, n_densities=w.density.shape[0], **kw)
    dens = torch.tensor(w.density, dtype=torch.float64, device=dev)
    pot = P.apply(dens)
    torch.cuda.synchronize()
    return P, pot.cpu().numpy()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("case", sorted(CASES))
def test_gpu_vs_tier_b(dev, case):
    w = workload_tiny(**CASES[case])
    print(f"[gpu] case={case} n_src={w.n_src} n_ctr={w.n_ctr}", flush=True)
    P, pot = run_gpu(w, dev)
    F = OracleFMM(w)
    tids, ref, qloc = F.evaluate()
    assert rel(pot[0][tids], ref) < TOL
    # QBX locals (after Stage 8) against the oracle's, mapped to the internal form
    Lq = P.qbx_locals()
    for c in range(0, w.n_ctr, max(1, w.n_ctr // 97)):
        want = CV.paper_local_to_packed(qloc[c], w.p_qbx)
        assert np.max(np.abs(Lq[c] - want)) <= TOL * np.max(np.abs(want)) * 10


@pytest.mark.parametrize("case", ["S-l1-n32", "D-l1-n32", "D-l2-q5p15"])
@pytest.mark.parametrize("lst", ["U", "V", "Wclose", "Wfar", "Xclose", "Xfar"])
def test_gpu_per_list_vs_tier_b(dev, case, lst):
    w = workload_tiny(**CASES[case])
    print(f"[gpu] case={case} list={lst}", flush=True)
    _, pot = run_gpu(w, dev, lists=(lst,))
    F = OracleFMM(w)
    tids, ref, _ = F.evaluate(lists=(lst,))
    _, full, _ = F.evaluate()
    err = np.max(np.abs(pot[0][tids] - ref)) / np.max(np.abs(full))
    assert err < TOL


@pytest.mark.parametrize("case,thr", [("D-l1-n32", 24), ("D-l2-q5p15", 64), ("S-l2-q8p20", 10 ** 6)])
def test_gpu_remark4_vs_tier_b(dev, case, thr):
    w = workload_tiny(**CASES[case])
    print(f"[gpu] case={case} wfar_direct_max={thr}", flush=True)
    _, pot = run_gpu(w, dev, wfar_direct_max=thr)
    tids, ref, _ = OracleFMM(w, wfar_direct_max=thr).evaluate()
    assert rel(pot[0][tids], ref) < TOL


@pytest.mark.parametrize("kernel", ["S", "D"])
def test_single_box_equals_direct(dev, kernel):
    w = workload_tiny(level=1, order=2, kernel=kernel, p_qbx=4, p_fmm=4, nmax=10 ** 7)
    print(f"[gpu] single box {kernel}", flush=True)
    _, pot = run_gpu(w, dev)
    ref, _ = O.direct_qbx(kernel, w.p_qbx, w.src_xyz, O.strengths(w)[0], w.ctr_xyz, w.tgt_xyz,
                          w.tgt_center, nrm=w.src_normal)
    assert rel(pot[0], ref) < 1e-12


def test_c1_vs_tier_b_and_tier_a(dev):
    w = workload_c1()
    print("[gpu] C1 sphere320 S 3/10", flush=True)
    _, pot = run_gpu(w, dev)
    F = OracleFMM(w)
    tids, ref, _ = F.evaluate()
    assert rel(pot[0][tids], ref) < TOL
    refA, _ = O.direct_qbx("S", w.p_qbx, w.src_xyz, O.strengths(w)[0], w.ctr_xyz, w.tgt_xyz,
                           w.tgt_center)
    assert rel(pot[0], refA) <= 0.75 ** (w.p_fmm + 1)


def test_c1_small_boxes_vs_tier_b(dev):
    w = workload_c1(nmax=32)
    print("[gpu] C1 nmax=32", flush=True)
    _, pot = run_gpu(w, dev)
    F = OracleFMM(w)
    rng = np.random.default_rng(0)
    cs = np.sort(rng.choice(w.n_ctr, 300, replace=False))
    tids, ref, _ = F.evaluate(centers=cs)
    assert rel(pot[0][tids], ref) < TOL


def test_multiple_densities(dev):
    w = workload_tiny(level=1, order=2, kernel="D", p_qbx=3, p_fmm=6, nmax=32, n_densities=3)
    print("[gpu] 3 densities", flush=True)
    _, pot = run_gpu(w, dev)
    F = OracleFMM(w)
    for d in range(3):
        tids, ref, _ = F.evaluate(density_index=d)
        assert rel(pot[d][tids], ref) < TOL


def test_repeat_apply_stable(dev):
    import torch

    from paper_1805_06106_amd import Plan

    w = workload_tiny(**CASES["D-l1-n32"])
    P = Plan.from_workload(w)
    dens = torch.tensor(w.density, device=dev)
    a = P.apply(dens).cpu().numpy()
    b = P.apply(dens).cpu().numpy()
    assert rel(a, b) < 1e-14


def test_zero_density_and_linearity(dev):
    import torch

    from paper_1805_06106_amd import Plan

    w = workload_tiny(**CASES["S-l1-n32"])
    P = Plan.from_workload(w)
    z = torch.zeros((1, w.n_src), dtype=torch.float64, device=dev)
    assert float(P.apply(z).abs().max()) == 0.0
    d1 = torch.tensor(w.density, device=dev)
    d2 = torch.tensor(np.random.default_rng(5).standard_normal((1, w.n_src)), device=dev)
    p1, p2, p12 = P.apply(d1).cpu().numpy(), P.apply(d2).cpu().numpy(), P.apply(2 * d1 - d2).cpu().numpy()
    assert rel(p12, 2 * p1 - p2) < 1e-12


# --- FP32 matrix-core translations ------------------------------------------------------
# Bar for the FP32 matrix-core translations: 1e-6 relative against the FP64 oracle.  The
# split form (leading degrees in FP64, hi/lo correction products, FP64 accumulation per
# K-step) must also not be less accurate than the uncorrected FP32 form.

@pytest.mark.parametrize("case", ["D-l1-n32", "D-l2-q5p15", "S-l2-q8p20"])
def test_fp32_split_translations_vs_tier_b(dev, case):
    w = workload_tiny(**CASES[case])
    F = OracleFMM(w)
    tids, ref, _ = F.evaluate()
    errs = {}
    for prec in ("fp32_split", "fp32_lead", "fp32"):
        print(f"[gpu] case={case} precision={prec}", flush=True)
        _, pot = run_gpu(w, dev, precision=prec)
        errs[prec] = rel(pot[0][tids], ref)
    print(f"[gpu] {case}: " + ", ".join(f"{k} {v:.3e}" for k, v in errs.items()), flush=True)
    for prec in errs:
        assert errs[prec] < 1e-6, prec
    assert errs["fp32_split"] <= errs["fp32"]


def test_fp32_split_c1_vs_tier_b(dev):
    w = workload_c1()
    print("[gpu] C1 fp32_split", flush=True)
    _, pot = run_gpu(w, dev, precision="fp32_split")
    tids, ref, _ = OracleFMM(w).evaluate()
    assert rel(pot[0][tids], ref) < 1e-6


@pytest.mark.parametrize("case", ["S-l1-n32", "D-l2-flat", "S-l2-tf05"])
def test_gpu_linf_tcr_vs_tier_b(dev, case):
    """The box-shaped TCR of the cost comparison: same kernels, other lists."""
    w = workload_tiny(**CASES[case])
    print(f"[gpu] case={case} tcr=linf", flush=True)
    _, pot = run_gpu(w, dev, tcr_norm="linf")
    tids, ref, _ = OracleFMM(w, tcr_norm="linf").evaluate()
    assert rel(pot[0][tids], ref) < TOL


@pytest.mark.parametrize("case", ["S-l1-n32", "D-l2-flat", "S-l2-tf05"])
def test_gpu_level_restricted_vs_tier_b(dev, case):
    """A level-restricted tree (the remark on List 3 complexity): same kernels, a refined
    tree, and the oracle's own level-restricted tree and lists."""
    w = workload_tiny(**CASES[case])
    print(f"[gpu] case={case} level-restricted", flush=True)
    _, pot = run_gpu(w, dev, level_restrict=True)
    tids, ref, _ = OracleFMM(w, level_restrict=True).evaluate()
    assert rel(pot[0][tids], ref) < TOL


@pytest.mark.parametrize("case", ["S-l1-n32", "D-l2-flat"])
@pytest.mark.parametrize("p_fmm", [2, 3, 5, 10, 15])
def test_gpu_m2l_rotation_vs_tier_b(dev, case, p_fmm):
    """M2L by rotation (T = B Z A on the matrix cores) against the oracle, whose M2L is the
    plain translation formula, and against the dense-matrix M2L of the library.  The kernel
    is compiled per order: p_fmm 2 and 3 fit one row tile (9 and 16 rows), 5 and 10 end in
    a ragged one, 15 fills 16."""
    kw = dict(CASES[case])
    if p_fmm < kw["p_qbx"]:
        pytest.skip("p_fmm below the case's p_qbx")
    kw["p_fmm"] = p_fmm
    w = workload_tiny(**kw)
    print(f"[gpu] case={case} p_fmm={p_fmm} m2l rotation", flush=True)
    _, pot = run_gpu(w, dev, m2l_rotation=True)
    _, dense = run_gpu(w, dev)
    tids, ref, _ = OracleFMM(w).evaluate()
    assert rel(pot[0][tids], ref) < TOL
    assert rel(pot[0], dense[0]) < 1e-11


@pytest.mark.parametrize("kernel", ["S", "D"])
def test_gpu_point_targets_vs_tier_b(dev, kernel):
    """Conventional targets (tgt_center = -1) beside the QBX targets: both against the
    oracle, and the QBX results unchanged by the extra points' presence in the lists."""
    from workloads import add_point_targets

    w = add_point_targets(workload_tiny(level=2, order=2, kernel=kernel, p_qbx=3, p_fmm=8,
                                        nmax=24), n_out=150, n_in=70)
    print(f"[gpu] point targets {kernel} n_tgt={w.n_tgt}", flush=True)
    _, pot = run_gpu(w, dev)
    F = OracleFMM(w)
    tids, ref = F.evaluate_points()
    assert rel(pot[0][tids], ref) < TOL
    qt, qref, _ = F.evaluate()
    assert rel(pot[0][qt], qref) < TOL
    # a single box: point targets are plain direct sums
    w1 = add_point_targets(workload_tiny(level=1, order=2, kernel=kernel, p_qbx=3, p_fmm=8,
                                         nmax=10 ** 9), n_out=30, n_in=10)
    _, pot1 = run_gpu(w1, dev)
    t1, r1 = OracleFMM(w1).evaluate_points()
    assert rel(pot1[0][t1], r1) < 1e-12


@pytest.mark.parametrize("case", ["S-l1-n32", "S-l2-tf05", "S-l2-q8p20"])
def test_gpu_sprime_vs_tier_b(dev, case):
    """Adjoint double layer: the single-layer QBX locals of the oracle differentiated along
    each target's normal (the base node's normal)."""
    import torch

    from paper_1805_06106_amd import Plan

    w = workload_tiny(**CASES[case])
    print(f"[gpu] S' case={case}", flush=True)
    tn = w.src_normal[np.arange(w.n_tgt) // 2]
    P = Plan.from_workload(w, kernel="SP")
    P.set_target_normals(tn)
    pot = P.apply(torch.tensor(w.density, device=dev)).cpu().numpy()[0]
    F = OracleFMM(w)
    tids, _, qloc = F.evaluate()
    ref = np.array([O.local_normal_derivative(w.p_qbx, qloc[int(w.tgt_center[t])],
                                              w.ctr_xyz[w.tgt_center[t]], w.tgt_xyz[t], tn[t])
                    for t in tids])
    assert rel(pot[tids], ref) < TOL
    # without normals the apply is refused
    from paper_1805_06106_amd import GQError

    Q = Plan.from_workload(w, kernel="SP")
    with pytest.raises(GQError):
        Q.apply(torch.tensor(w.density, device=dev))
