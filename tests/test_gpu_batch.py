"""Batched plans (several surfaces in one set of launches) and HIP-graph applies, through
the C ABI, against single-plan applies and the FP64 oracle."""

import numpy as np
import pytest

from oracle.gigaqbx import OracleFMM
from workloads import workload_tiny

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

MEMBERS = [
    dict(level=1, order=2, kernel="D", p_qbx=3, p_fmm=6, nmax=32, seed=11, n_densities=2),
    dict(level=2, order=1, kernel="D", p_qbx=3, p_fmm=6, nmax=40, seed=12, n_densities=2,
         bump=(5, 2, 0.2)),
    dict(level=1, order=2, kernel="D", p_qbx=3, p_fmm=6, nmax=24, seed=13, n_densities=2,
         curved=False),
]


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def members():
    import torch

    import paper_1805_06106_amd  # noqa: F401

    assert torch.cuda.is_available()
    return [workload_tiny(**m) for m in MEMBERS]


def test_batch_equals_members_and_oracle(members):
    import torch

    from paper_1805_06106_amd import Plan

    dev = torch.device("cuda:0")
    plans = [Plan.from_workload(w, n_densities=2) for w in members]
    singles = [p.apply(torch.tensor(w.density, device=dev)).cpu().numpy()
               for p, w in zip(plans, members)]
    for graph in (False, True):
        print(f"[gpu] batch of {len(members)} surfaces, graph={graph}", flush=True)
        B = Plan.batch(plans, graph=graph)
        dens = torch.tensor(np.concatenate([w.density for w in members], axis=1), device=dev)
        for rep in range(3):  # graph replays with eager work in between
            pot = B.apply(dens).cpu().numpy()
            torch.cuda.synchronize()
            off = 0
            for w, ref in zip(members, singles):
                got = pot[:, off:off + w.n_tgt]
                assert rel(got, ref) < 1e-12, (graph, rep)
                off += w.n_tgt
            dens.mul_(1.0)  # eager work between replays
        B.close()
    for w, ref in zip(members, singles):
        F = OracleFMM(w)
        for d in range(2):
            tids, o, _ = F.evaluate(density_index=d)
            assert rel(ref[d][tids], o) < 1e-10
    # members stay usable after the batch is gone
    again = plans[0].apply(torch.tensor(members[0].density, device=dev)).cpu().numpy()
    assert rel(again, singles[0]) < 1e-14


def test_batch_rotation_m2l(members):
    """A batch of plans with the rotation-factored M2L: its factors are built for the union
    of the members' offset classes; eager and graph applies against the members' own
    applies, and against the dense-M2L batch to the factors' accuracy."""
    import torch

    from paper_1805_06106_amd import Plan

    dev = torch.device("cuda:0")
    print(f"[gpu] batch of {len(members)} surfaces, rotation M2L", flush=True)
    plans = [Plan.from_workload(w, n_densities=2, m2l_rotation=True) for w in members]
    singles = np.concatenate([p.apply(torch.tensor(w.density, device=dev)).cpu().numpy()
                              for p, w in zip(plans, members)], axis=1)
    dens = torch.tensor(np.concatenate([w.density for w in members], axis=1), device=dev)
    dense = Plan.batch([Plan.from_workload(w, n_densities=2) for w in members])
    ref = dense.apply(dens).cpu().numpy()
    for graph in (False, True):
        B = Plan.batch(plans, graph=graph)
        for _ in range(2):
            pot = B.apply(dens).cpu().numpy()
            assert rel(pot, singles) < 1e-13, graph
            assert rel(pot, ref) < 1e-11, graph
            dens.mul_(1.0)  # eager work between replays
        B.close()
    dense.close()
    for p in plans:
        p.close()


def test_graph_apply_replays_and_recaptures(members):
    import torch

    from paper_1805_06106_amd import Plan

    dev = torch.device("cuda:0")
    w = members[0]
    eager = Plan.from_workload(w, n_densities=2)
    G = Plan.from_workload(w, n_densities=2, graph=True)
    rng = np.random.default_rng(3)
    d1 = torch.tensor(w.density, device=dev)
    out = torch.empty((2, w.n_tgt), dtype=torch.float64, device=dev)
    for rep in range(4):
        print(f"[gpu] graph replay {rep}", flush=True)
        # same buffers, new contents: the captured graph reads them at replay time
        d1.copy_(torch.tensor(rng.standard_normal((2, w.n_src)), device=dev))
        G.apply(d1, out)
        ref = eager.apply(d1)
        torch.cuda.synchronize()
        assert rel(out.cpu().numpy(), ref.cpu().numpy()) < 1e-14
    # a different output buffer triggers a new capture
    out2 = G.apply(d1)
    torch.cuda.synchronize()
    assert rel(out2.cpu().numpy(), eager.apply(d1).cpu().numpy()) < 1e-14


def test_overlapped_far_field_equals_serial(members):
    """The far-field chain on the plan's own stream against every stage in order on one
    stream (the default): eager, timed and graph applies, single and batch plans."""
    import torch

    from paper_1805_06106_amd import Plan

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(17)
    for w in members[:2]:
        serial = Plan.from_workload(w, n_densities=2)
        d = torch.tensor(rng.standard_normal((2, w.n_src)), device=dev)
        ref = serial.apply(d).cpu().numpy()
        for kw in (dict(), dict(timing=True), dict(graph=True)):
            print(f"[gpu] overlap vs serial {kw}", flush=True)
            P = Plan.from_workload(w, n_densities=2, overlap=True, **kw)
            out = torch.empty((2, w.n_tgt), dtype=torch.float64, device=dev)
            for rep in range(3):
                P.apply(d, out)
                torch.cuda.synchronize()
                assert rel(out.cpu().numpy(), ref) < 1e-14, (kw, rep)
                d.mul_(1.0)  # eager work between replays
            if kw.get("timing"):
                st = P.stats()
                assert st["timed_applies"] == 3
                assert all(v >= 0 for v in st["stage_ms"].values())
                assert st["stage_ms"]["total"] >= st["stage_ms"]["p2qbxl"]
            # switching to serial recaptures the graph and gives the same result
            P.set_overlap(False)
            P.apply(d, out)
            torch.cuda.synchronize()
            assert rel(out.cpu().numpy(), ref) < 1e-14, kw
            P.close()
    plans = [Plan.from_workload(w, n_densities=2) for w in members]
    dens = torch.tensor(np.concatenate([w.density for w in members], axis=1), device=dev)
    a = Plan.batch(plans, graph=True, overlap=True).apply(dens).cpu().numpy()
    b = Plan.batch(plans).apply(dens).cpu().numpy()
    assert rel(a, b) < 1e-14


def test_batch_rejects_mismatched_members(members):
    from paper_1805_06106_amd import GQError, Plan

    a = Plan.from_workload(members[0], n_densities=2)
    b = Plan.from_workload(members[1], n_densities=1)
    with pytest.raises(GQError):
        Plan.batch([a, b])
    with pytest.raises(GQError):
        Plan.batch([a, a])
    c = Plan.from_workload(members[1], n_densities=2, p_fmm=7)
    with pytest.raises(GQError):
        Plan.batch([a, c])


def test_batch_fp32_split(members):
    import torch

    from paper_1805_06106_amd import Plan

    dev = torch.device("cuda:0")
    plans = [Plan.from_workload(w, n_densities=2, precision="fp32_split") for w in members]
    B = Plan.batch(plans, graph=True)
    dens = torch.tensor(np.concatenate([w.density for w in members], axis=1), device=dev)
    pot = B.apply(dens).cpu().numpy()
    off = 0
    for w in members:
        tids, o, _ = OracleFMM(w).evaluate(density_index=1)
        assert rel(pot[1, off:off + w.n_tgt][tids], o) < 1e-6
        off += w.n_tgt


def test_autotuned_plan_matches_default(members):
    import torch

    from paper_1805_06106_amd import Plan

    dev = torch.device("cuda:0")
    w = members[1]
    d = torch.tensor(w.density, device=dev)
    ref = Plan.from_workload(w, n_densities=2).apply(d).cpu().numpy()
    for prec in ("fp64", "fp32_split"):
        print(f"[gpu] autotune {prec}", flush=True)
        P = Plan.from_workload(w, n_densities=2, autotune=True, precision=prec)
        st = P.stats()
        assert st["m2l_tile_cols"] in (32, 64)
        got = P.apply(d).cpu().numpy()
        assert rel(got, ref) < (1e-13 if prec == "fp64" else 1e-6)


def test_batch_with_point_targets(members):
    import torch

    from paper_1805_06106_amd import Plan
    from workloads import add_point_targets

    dev = torch.device("cuda:0")
    ws = [add_point_targets(members[0], n_out=50, n_in=20, seed=1), members[1],
          add_point_targets(members[2], n_out=30, n_in=10, seed=2)]
    plans = [Plan.from_workload(w, n_densities=2) for w in ws]
    singles = [p.apply(torch.tensor(w.density, device=dev)).cpu().numpy()
               for p, w in zip(plans, ws)]
    print("[gpu] batch with point targets", flush=True)
    B = Plan.batch(plans, graph=True)
    dens = torch.tensor(np.concatenate([w.density for w in ws], axis=1), device=dev)
    pot = B.apply(dens).cpu().numpy()
    off = 0
    for w, ref in zip(ws, singles):
        assert rel(pot[:, off:off + w.n_tgt], ref) < 1e-12
        off += w.n_tgt
    assert B.stats()["n_point_targets"] == 110


def test_c3_members_full_size_vs_tier_b():
    """Three surfaces of the 64-urchin batch at full size (surfaces 2, 0 and 14: 20 * 4^l
    triangles at l = 3, 4, 5; 28 nodes each; D, 5/15; 8 densities), merged into one batch
    plan with split-precision translations and a HIP graph, on a level-restricted tree with
    Remark 4 at 64 (the workloads' own nmax, 512); every member against Tier B on sampled
    centers for the first and the last density, at the 1e-8 bar."""
    import torch

    from paper_1805_06106_amd import Plan
    from workloads import workload_c3

    dev = torch.device("cuda:0")
    tree = dict(wfar_direct_max=64, level_restrict=True)
    ws = [workload_c3(i) for i in (2, 0, 14)]
    nd = ws[0].density.shape[0]
    print(f"[gpu] C3 members {[w.n_src for w in ws]} sources, {nd} densities", flush=True)
    members = [Plan.from_workload(w, n_densities=nd, precision="fp32_split", **tree)
               for w in ws]
    B = Plan.batch(members, graph=True)
    for P in members:
        P.close()
    dens = torch.tensor(np.concatenate([w.density for w in ws], axis=1), device=dev)
    pot = B.apply(dens)
    pot2 = B.apply(dens)  # a replay of the captured graph
    torch.cuda.synchronize()
    pot, pot2 = pot.cpu().numpy(), pot2.cpu().numpy()
    B.close()
    assert np.array_equal(pot, pot2) or rel(pot2, pot) < 1e-14
    rng = np.random.default_rng(91)
    off = 0
    for w in ws:
        F = OracleFMM(w, **tree)
        owner = np.asarray(F.tree.ctr_owner)
        seeds = rng.choice(w.n_ctr, 3, replace=False)
        cs = np.unique(np.concatenate([np.nonzero(owner == owner[c])[0][:8] for c in seeds]))
        for d in (0, nd - 1):
            tids, ref, _ = F.evaluate(density_index=d, centers=cs)
            err = rel(pot[d, off + tids], ref)
            print(f"[gpu] C3 member n_src={w.n_src} density {d}: {err:.3e}", flush=True)
            assert err < 1e-8
        off += w.n_tgt
