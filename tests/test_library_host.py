"""CPU tests of the library's host side: exported symbols, planner vs the oracle's
definition-based tree and lists, translation matrices vs the oracle's translations,
argument validation.  No GPU call is made (plans are created host-only)."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from oracle.gigaqbx import OracleFMM
from workloads import workload_c1, workload_tiny

import gq_convert as CV

pytestmark = pytest.mark.usefixtures("oracle_lib")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gq():
    import paper_1805_06106_amd as G

    G._capi.lib()
    return G


def test_library_exports_every_declared_symbol(gq):
    hdr = open(os.path.join(ROOT, "include", "gigaqbx.h")).read()
    names = set(re.findall(r"\b(gq_[a-z_]+)\s*\(", hdr))
    assert {"gq_plan_create", "gq_apply", "gq_stats", "gq_plan_destroy"} <= names
    L = ctypes.CDLL(gq._capi.LIB_PATH)
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(gq._capi.EXPORTED) == names


CASES = {
    "S-l1-n32": dict(level=1, order=2, kernel="S", p_qbx=3, p_fmm=6, nmax=32),
    "D-l1-n32": dict(level=1, order=2, kernel="D", p_qbx=3, p_fmm=6, nmax=32),
    "S-l2-tf05": dict(level=2, order=1, kernel="S", p_qbx=2, p_fmm=5, nmax=24, tcf=0.5),
    "D-l2-flat": dict(level=2, order=1, kernel="D", p_qbx=2, p_fmm=5, nmax=40, curved=False),
    "S-l2-tf0": dict(level=2, order=2, kernel="S", p_qbx=2, p_fmm=4, nmax=64, tcf=0.0),
}


@pytest.mark.parametrize("case", sorted(CASES) + ["D-l1-n32-r4", "S-l1-n32-linf",
                                                   "S-l2-tf05-linf", "D-l2-flat-linf",
                                                   "S-l1-n32-lr", "D-l2-flat-lr",
                                                   "S-l2-tf05-lr"])
def test_planner_matches_oracle_lists(gq, case):
    thr = 24 if case.endswith("-r4") else 0
    tcr = "linf" if case.endswith("-linf") else "l2"
    lr = case.endswith("-lr")
    w = workload_tiny(**CASES[case.replace("-r4", "").replace("-linf", "").replace("-lr", "")])
    P = gq.Plan.from_workload(w, host_only=True, wfar_direct_max=thr, tcr_norm=tcr,
                              level_restrict=lr)
    F = OracleFMM(w, wfar_direct_max=thr, tcr_norm=tcr, level_restrict=lr)
    c, h, lev, par, own = P.tree()
    t = F.tree
    assert len(h) == t.nboxes
    assert np.array_equal(c, t.center) and np.array_equal(h, t.h)
    assert np.array_equal(par, t.parent) and np.array_equal(own, t.ctr_owner)
    owners, targets = F.list_owner_boxes(), F.target_boxes()
    for nm in ("U", "V", "Wclose", "Wfar", "Xclose", "Xfar"):
        ptr, items = P.list(nm)
        for b in (targets if nm in ("U", "Wclose", "Wfar") else owners):
            assert set(items[ptr[b]:ptr[b + 1]].tolist()) == F.lists.get(nm, b), (nm, b)


@pytest.mark.parametrize("kernel", ["S", "D"])
def test_planner_lists_with_point_targets(gq, kernel):
    """Boxes that own conventional targets are target boxes: their lists equal the
    oracle's, and the plan counts the targets."""
    from workloads import add_point_targets

    w = add_point_targets(workload_tiny(level=2, order=1, kernel=kernel, p_qbx=2, p_fmm=5,
                                        nmax=24), n_out=80, n_in=40)
    P = gq.Plan.from_workload(w, host_only=True)
    F = OracleFMM(w)
    assert P.stats()["n_point_targets"] == 120
    owners = F.list_owner_boxes()
    targets = F.target_boxes()
    for nm in ("U", "V", "Wclose", "Wfar", "Xclose", "Xfar"):
        ptr, items = P.list(nm)
        for b in (targets if nm in ("U", "Wclose", "Wfar") else owners):
            assert set(items[ptr[b]:ptr[b + 1]].tolist()) == F.lists.get(nm, b), (nm, b)


def test_planner_c1_matches_oracle(gq):
    w = workload_c1()
    P = gq.Plan.from_workload(w, host_only=True)
    F = OracleFMM(w)
    _, h, _, par, own = P.tree()
    assert np.array_equal(par, F.tree.parent) and np.array_equal(own, F.tree.ctr_owner)
    for nm in ("U", "V", "Wclose", "Wfar", "Xclose", "Xfar"):
        ptr, items = P.list(nm)
        for b in F.list_owner_boxes():
            if nm in ("U", "Wclose", "Wfar") and b not in F.target_boxes():
                continue
            assert set(items[ptr[b]:ptr[b + 1]].tolist()) == F.lists.get(nm, b), (nm, b)


def test_stats_pair_counts(gq):
    w = workload_tiny(**CASES["S-l1-n32"])
    P = gq.Plan.from_workload(w, host_only=True)
    F = OracleFMM(w)
    s = P.stats()
    t, L = F.tree, F.lists
    for nm in ("U", "Wclose", "Xclose"):
        ref = sum(sum(len(t.own_src[d]) for d in L.get(nm, b)) * len(t.own_ctr[b])
                  for b in F.target_boxes())
        assert s["pairs"][nm] == ref
    assert s["pairs"]["V"] == sum(len(L.V(b)) for b in F.list_owner_boxes())
    assert s["pairs"]["Wfar"] == sum(len(L.Wfar(b)) * len(t.own_ctr[b]) for b in F.target_boxes())
    assert s["n_boxes"] == t.nboxes and s["n_levels"] == t.nlevels


def test_stats_modeled_flops_table7(gq):
    """gq_stats' modeled flops are Table 7's counts over the plan's lists, checked against
    the per-entry sum written out from the oracle's own lists."""
    from paper_1805_06106_amd import costmodel as CM

    w = workload_tiny(**CASES["D-l1-n32"])
    P = gq.Plan.from_workload(w, host_only=True)
    F = OracleFMM(w)
    s = P.stats()
    t, L = F.tree, F.lists
    p, q = w.p_fmm, w.p_qbx
    ref = {nm: 0.0 for nm in ("U", "V", "Wclose", "Wfar", "Xclose", "Xfar")}
    for b in F.target_boxes():
        nt = len(t.own_ctr[b])
        for nm in ("U", "Wclose", "Xclose"):
            ref[nm] += q * q * sum(len(t.own_src[d]) for d in L.get(nm, b)) * nt
        ref["Wfar"] += p ** 3 * len(L.Wfar(b)) * nt
    for b in F.list_owner_boxes():
        ref["V"] += p ** 3 * len(L.V(b))
    model = s["modeled_flops"]
    for nm in ("U", "V", "Wclose", "Wfar", "Xclose"):
        assert model[nm] == ref[nm], nm
    assert model["Xfar"] == p * p * s["pairs"]["Xfar"]
    assert model["total_lists"] == sum(model[nm] for nm in ref)
    py = CM.paper_list_model(s, p, q)
    for nm in ref:
        assert model[nm] == py[nm]


# --- translation matrices ----------------------------------------------------------------

def _octant_vec(o):
    return np.array([1.0 if o & 1 else -1.0, 1.0 if o & 2 else -1.0, 1.0 if o & 4 else -1.0])


@pytest.mark.parametrize("p", [4, 10, 15])
@pytest.mark.parametrize("kernel", ["S", "D"])
def test_m2m_matrix_vs_oracle(gq, p, kernel):
    rng = np.random.default_rng(p)
    a = 0.25
    xp = np.array([0.1, -0.3, 0.2])
    for o in range(8):
        xc = xp + (a / 2) * _octant_vec(o)
        src = xc + rng.uniform(-a / 2, a / 2, (7, 3))
        nrm = rng.standard_normal((7, 3))
        nrm /= np.linalg.norm(nrm, axis=1)[:, None]
        q = rng.standard_normal(7)
        Mc = CV.paper_mpole_to_packed(O.p2m(kernel, p, src, q, xc, nrm=nrm), p, a / 2)
        Mp = CV.paper_mpole_to_packed(O.p2m(kernel, p, src, q, xp, nrm=nrm), p, a)
        T = gq.gq_translation_matrix(0, p, o)
        assert np.max(np.abs(T @ Mc - Mp)) < 1e-12 * np.max(np.abs(Mp))


@pytest.mark.parametrize("p", [4, 10, 15])
def test_l2l_matrix_vs_oracle(gq, p):
    rng = np.random.default_rng(p + 1)
    a = 0.5
    xp = np.array([-0.2, 0.1, 0.4])
    src = xp + np.array([[3.0, 1.0, -2.0], [-2.5, 2.2, 1.7]])
    Lp = O.p2l("S", p, src, [1.0, -0.4], xp)
    for o in range(8):
        xc = xp + (a / 2) * _octant_vec(o)
        Lc = O.l2l(p, p, Lp, xp, xc)
        T = gq.gq_translation_matrix(1, p, o)
        got = T @ CV.paper_local_to_packed(Lp, p, a)
        ref = CV.paper_local_to_packed(Lc, p, a / 2)
        assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("p", [4, 10, 15])
def test_m2l_matrix_vs_oracle(gq, p):
    rng = np.random.default_rng(p + 2)
    a = 0.125
    xs = np.array([0.3, 0.1, -0.2])
    src = xs + rng.uniform(-a, a, (6, 3))
    q = rng.standard_normal(6)
    M = O.p2m("S", p, src, q, xs)
    for off in [(3, 0, 0), (-5, 4, 2), (0, -3, 5), (4, 4, -4), (-3, -3, -3), (5, 5, 5)]:
        xt = xs + 2 * a * np.array(off, dtype=float)
        Lt = O.m2l(p, p, M, xs, xt)
        T = gq.gq_translation_matrix(2, p, *off)
        got = T @ CV.paper_mpole_to_packed(M, p, a)
        ref = CV.paper_local_to_packed(Lt, p, a)
        assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))


# --- validation ---------------------------------------------------------------------------

def _args(w, **over):
    d = dict(src_xyz=w.src_xyz, src_w=w.src_w, src_normal=w.src_normal, ctr_xyz=w.ctr_xyz,
             ctr_radius=w.ctr_radius, tgt_xyz=w.tgt_xyz, tgt_center=w.tgt_center,
             p_qbx=w.p_qbx, p_fmm=w.p_fmm, kernel=w.kernel, nmax=w.nmax, tcf=w.tcf,
             host_only=True)
    d.update(over)
    return d


def test_invalid_arguments(gq):
    w = workload_tiny(level=0, order=2, kernel="D", p_qbx=2, p_fmm=4, nmax=16)
    G = gq
    with pytest.raises(G.GQError) as e:
        G.Plan(**_args(w, p_qbx=5, p_fmm=4))
    assert e.value.status == 1 and "p_qbx" in str(e.value)
    with pytest.raises(G.GQError) as e:
        G.Plan(**_args(w, p_fmm=21, p_qbx=3))
    assert e.value.status == 4
    with pytest.raises(G.GQError):
        G.Plan(**_args(w, tcf=1.5))
    with pytest.raises(G.GQError) as e:
        G.Plan(**_args(w, max_device_bytes=-1))
    assert e.value.status == 1 and "max_device_bytes" in str(e.value)
    # the tree search times applies, so it needs a device plan
    with pytest.raises(G.GQError) as e:
        G.Plan(**_args(w, autotune_tree=True))
    assert e.value.status == 1 and "AUTOTUNE_TREE" in str(e.value)
    with pytest.raises(G.GQError):
        G.Plan(**_args(w, src_normal=None))
    bad = w.src_normal.copy()
    bad[3] *= 1.01
    with pytest.raises(G.GQError):
        G.Plan(**_args(w, src_normal=bad))
    r = w.ctr_radius.copy()
    r[0] = 0.0
    with pytest.raises(G.GQError):
        G.Plan(**_args(w, ctr_radius=r))
    tc = w.tgt_center.copy()
    tc[0] = w.n_ctr
    with pytest.raises(G.GQError):
        G.Plan(**_args(w, tgt_center=tc))
    x = w.src_xyz.copy()
    x[2, 1] = np.nan
    with pytest.raises(G.GQError):
        G.Plan(**_args(w, src_xyz=x))
    with pytest.raises(G.GQError):
        G.Plan(**_args(w, nmax=0))
    # a valid host-only plan cannot be applied
    P = G.Plan(**_args(w))
    with pytest.raises(G.GQError):
        G.gq_apply(P.handle, 1, 1)


def test_single_box_plan(gq):
    w = workload_tiny(level=0, order=2, kernel="S", p_qbx=2, p_fmm=4, nmax=10 ** 6)
    P = gq.Plan.from_workload(w, host_only=True)
    s = P.stats()
    assert s["n_boxes"] == 1
    assert s["pairs"]["U"] == w.n_src * w.n_ctr
    assert all(s["pairs"][k] == 0 for k in ("V", "Wclose", "Wfar", "Xclose", "Xfar"))


def test_batch_and_graph_validation(gq):
    w = workload_tiny(level=0, order=2, kernel="D", p_qbx=2, p_fmm=4, nmax=16)
    G = gq
    P = G.Plan(**_args(w))  # host-only
    with pytest.raises(G.GQError) as e:
        G.Plan.batch([P])
    assert e.value.status == 1 and "host-only" in str(e.value)
    with pytest.raises(G.GQError):
        G.Plan.batch([])
    with pytest.raises(G.GQError) as e:
        G.Plan(**_args(w, timing=True, graph=True))
    assert "exclusive" in str(e.value)


def test_default_translation_tile_widths(gq):
    """Without autotuning: 32-pair M2L tiles in every precision mode (the split kernel keeps
    FP64 accumulators in registers); 64-pair tiles for the rotation M2L (four waves of 16
    pairs); XCD-aware tile order."""
    w = workload_tiny(level=1, order=2, kernel="D", p_qbx=3, p_fmm=6, nmax=32)
    G = gq
    for prec, cols in (("fp64", 32), ("fp32", 32), ("fp32_split", 32), ("fp32_lead", 32)):
        st = G.Plan(**_args(w, precision=prec)).stats()
        assert (st["m2l_tile_cols"], st["m2l_xcd_order"]) == (cols, True), prec
    st = G.Plan(**_args(w, m2l_rotation=True)).stats()
    assert st["m2l_tile_cols"] == 64


def test_overlap_setting_validation(gq):
    w = workload_tiny(level=0, order=2, kernel="D", p_qbx=2, p_fmm=4, nmax=16)
    G = gq
    P = G.Plan(**_args(w))  # host-only: the setting is stored, nothing is launched
    P.set_overlap(False)
    P.set_overlap(True)
    from paper_1805_06106_amd import _capi as C

    for bad in (2, -1):
        with pytest.raises(G.GQError) as e:
            C.gq_set_overlap(P.handle, bad)
        assert e.value.status == 1
    with pytest.raises(G.GQError):
        C.gq_set_overlap(None, 1)


def test_sprime_validation(gq):
    w = workload_tiny(level=1, order=2, kernel="S", p_qbx=2, p_fmm=4, nmax=16)
    G = gq
    P = G.Plan(**_args(w, kernel="SP"))  # host-only S' plan is valid
    with pytest.raises(G.GQError):
        P.set_target_normals(np.repeat(w.src_normal, 2, axis=0))  # host-only: no device
    from workloads import add_point_targets

    wp = add_point_targets(w, n_out=5, n_in=0)
    with pytest.raises(G.GQError) as e:
        G.Plan(**_args(wp, kernel="SP", host_only=False))
    assert e.value.status == 4


def test_source_interp_validation(gq):
    """gq_set_source_interp checks its sizes against the plan's sources before anything
    touches the device; a host-only plan is then refused."""
    from workloads import oversampled_workload
    from workloads.geometry import SurfaceSpec

    w = oversampled_workload("os", level=0, spec=SurfaceSpec(curved=True), kernel="S",
                             p_qbx=2, p_fmm=4, node_order=2, quad_order=2, sub=2, nmax=32)
    G = gq
    P = G.Plan.from_workload(w, host_only=True)
    nq, nn = w.interp.shape
    assert w.n_src == w.n_elem * nq
    bad = [(w.n_elem + 1, w.interp, "n_elem"), (w.n_elem, np.zeros((nq, 65)), "size"),
           (w.n_elem, np.zeros((nq + 1, nn)), "n_elem"), (0, w.interp, "n_elem")]
    for ne, m, what in bad:
        with pytest.raises(G.GQError) as e:
            P.set_source_interp(ne, m)
        assert e.value.status == 1 and what in str(e.value), (ne, m.shape, str(e.value))
    nan = w.interp.copy()
    nan[0, 0] = np.nan
    with pytest.raises(G.GQError) as e:
        P.set_source_interp(w.n_elem, nan)
    assert "non-finite" in str(e.value)
    with pytest.raises(G.GQError) as e:
        P.set_source_interp(w.n_elem, w.interp)
    assert "host-only" in str(e.value)


def test_associate_targets_validation(gq):
    """Argument errors of gq_associate_targets are found on the host, before any device
    work."""
    G = gq
    s3, c3, t3 = np.zeros((2, 3)), np.ones((1, 3)), np.zeros((3, 3))
    bad = [dict(src_danger=[1.0, -1.0]), dict(src_danger=[1.0, np.nan]), dict(ctr_radius=[0.0]),
           dict(tol=-0.1), dict(tol=np.inf), dict(tgt_side=[0, 1, 0]),
           dict(ctr_side=[2], tgt_side=[0, 0, 0]), dict(ctr_side=[1], tgt_side=[0, 3, 0]),
           dict(tgt_xyz=np.array([[0, 0, np.nan]]))]
    for over in bad:
        a = dict(src_xyz=s3, src_danger=[1.0, 1.0], ctr_xyz=c3, ctr_radius=[1.0], tgt_xyz=t3)
        a.update(over)
        with pytest.raises(G.GQError) as e:
            G.associate_targets(**a)
        assert e.value.status == 1, over
    assert G.associate_targets(s3, [1.0, 1.0], c3, [1.0], np.zeros((0, 3))).shape == (0,)
    got = G.associate_targets(np.zeros((0, 3)), [], c3, [1.0], t3)  # no sources: no danger
    assert got.tolist() == [G.GQ_TARGET_FAR] * 3


@pytest.mark.parametrize("p", [2, 5, 10, 15])
def test_rotation_m2l_work_model(gq, p):
    """The executed work of the rotation-form M2L that the benchmark's matrix-core fraction
    uses: the nonzero 16 x 16 tiles of the factors A and B, counted from the factors the
    library builds, and the k-steps of Z's order blocks (p + 1 - m rows each, rounded up to
    4), each k-step 16 x 16 x 4 multiply-adds per 16 pairs."""
    from paper_1805_06106_amd import costmodel as CM

    npc = (p + 1) ** 2
    ntr = -(-npc // 16)
    A = np.zeros((16 * ntr, 16 * ntr))
    A[:npc, :npc] = gq.gq_translation_matrix(3, p, 1, 2, 3)  # a generic direction
    B = np.zeros_like(A)
    B[:npc, :npc] = gq.gq_translation_matrix(5, p, 1, 2, 3)
    tiles = [int(np.count_nonzero(np.abs(M.reshape(ntr, 16, ntr, 16)).sum(axis=(1, 3))))
             for M in (A, B)]
    assert tiles[0] == tiles[1]
    zsteps = sum(-(-(p + 1 - m) // 4) * (1 if m == 0 else 2) for m in range(p + 1))
    assert CM.rotation_m2l_pair(p) == (4 * sum(tiles) + zsteps) * 2 * 16 * 16 * 4 / 16
    if p == 15:
        assert tiles[0] == 44 and zsteps == 76  # 428 k-steps per 16 pairs
        assert CM.rotation_m2l_pair(p) == 54784


@pytest.mark.parametrize("p", [4, 10, 15])
def test_m2l_rotation_factors(gq, p):
    """The rotated form of M2L: T = B Z A to rounding, A and B block diagonal by degree
    (rotations keep the degree), and Z couples only equal orders, real with real and
    imaginary with imaginary parts (a translation along z)."""
    np_ = (p + 1) ** 2
    deg = np.repeat(np.arange(p + 1), 2 * np.arange(p + 1) + 1)
    off = np.arange(np_) - deg ** 2
    order = (off + 1) // 2
    part = np.where(off == 0, 0, 2 - off % 2)  # 0: m = 0, 1: real, 2: imaginary
    for o in [(2, 0, 0), (0, 0, -2), (1, 2, 3), (-3, 3, -2), (0, 2, -2)]:
        T = gq.gq_translation_matrix(2, p, *o)
        A, Z, B = (gq.gq_translation_matrix(k, p, *o) for k in (3, 4, 5))
        BZA = B @ Z @ A
        rowmax = np.max(np.abs(T), axis=1)
        assert np.max(np.max(np.abs(BZA - T), axis=1) / rowmax) < 1e-11, o
        for M in (A, B):
            assert np.all(M[deg[:, None] != deg[None, :]] == 0.0)
        same = (order[:, None] == order[None, :]) & (part[:, None] == part[None, :])
        assert np.max(np.abs(Z[~same])) == 0.0


def test_m2l_rotation_validation(gq):
    w = workload_tiny(level=0, order=2, kernel="D", p_qbx=2, p_fmm=4, nmax=16)
    G = gq
    G.Plan(**_args(w, m2l_rotation=True))  # host-only FP64 plan: accepted
    for over in (dict(precision="fp32_split"), dict(p_fmm=16)):
        with pytest.raises(G.GQError) as e:
            G.Plan(**_args(w, m2l_rotation=True, **over))
        assert e.value.status == 4


def test_points_near_validation(gq):
    """gq_points_near rejects bad arguments on the host and needs no device for empty
    inputs."""
    G = gq
    q, p = np.zeros((2, 3)), np.ones((3, 3))
    for r in ([1.0, -1.0], [np.nan, 1.0], [np.inf, 1.0]):
        with pytest.raises(G.GQError) as e:
            G.points_near(q, r, p)
        assert e.value.status == 1
    with pytest.raises(G.GQError):
        G.points_near(np.array([[0.0, np.nan, 0.0]]), [1.0], p)
    assert G.points_near(np.zeros((0, 3)), [], p).shape == (0,)
    assert not G.points_near(q, [1.0, 1.0], np.zeros((0, 3))).any()
