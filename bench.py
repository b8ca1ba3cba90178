#!/usr/bin/env python3
"""Benchmark: QBX-FMM target evaluations per second on one MI355X.

Workload (default): the 'urchin' surface rho = 1 + 0.2 Re Y_8^4 on 20,480 curved triangles,
28 nodes per triangle (573,440 sources), two QBX centers per node (1,146,880 centers, one
target each), double-layer potential, p_qbx = 5, p_fmm = 15, nmax = 160, t_f = 0.9, FP64;
level-restricted tree, Remark 4 at 128 sources (both paper options, measured fastest here),
rotation-form M2L.
One step = one full evaluation (Algorithm 5 Stages 2-9) of one density with the plan cached
and all inputs resident in HBM.

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU_TFLOPS = 78.6  # MI355X: 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3  # MI355X dense FP32 matrix

# HBM bytes per launch (read + write) of the main kernels on the default workload, from two
# rocprofv3 counter passes (FETCH_SIZE, WRITE_SIZE) scaled by a 1 GiB copy measured in the
# same process (profiles/hbm_traffic_urchin20480_D_q5p15.md).  Valid only for the kernel
# sources (sha256 over csrc/kernels*.hip in name order) and tree options they were measured
# on: reported while they match, else null.
COUNTER_TRAFFIC = {
    "kernels_sha256": "9dcc72e4476c9b470801527bc0ac54b7b336be3e1ac37f59c32d8a2d910fab11",
    "workload": "urchin8-20480", "wfar_direct_max": 128, "level_restrict": True, "nmax": 160,
    "precision": "fp64", "m2l_rotation": True,
    "bytes_per_launch": {"p2qbxl": 6.38616e+09, "m2l": 2.51890e+10, "l2qbxl": 1.003443e+09},
}


def tree_opts(args):
    """Plan options that shape the tree and lists: Remark 4's threshold, level restriction
    and (when given) nmax, the most particles a box holds before it is split."""
    opts = {"wfar_direct_max": args.wfar_direct_max, "level_restrict": bool(args.level_restrict)}
    if getattr(args, "nmax", None):
        opts["nmax"] = args.nmax
    if getattr(args, "autotune_tree", 0):
        opts["autotune_tree"] = True
    return opts


def counter_traffic(kernel, workload, wfar_direct_max, level_restrict, nmax, m2l_rotation):
    import hashlib

    csrc = os.path.join(ROOT, "paper_1805_06106_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.startswith("kernels") and name.endswith(".hip"):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(f.read())
    h = h.hexdigest()
    c = COUNTER_TRAFFIC
    if (h != c["kernels_sha256"] or workload != c["workload"]
            or wfar_direct_max != c["wfar_direct_max"]
            or level_restrict != c.get("level_restrict", False) or nmax != c.get("nmax")
            or m2l_rotation != c.get("m2l_rotation", False)):
        return None
    return c["bytes_per_launch"].get(kernel)


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def make_workload(name):
    from workloads import workload_c1, workload_c2, workload_c4

    return {"c1": workload_c1, "c2": workload_c2, "c4": workload_c4}[name]()


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 10; 200 for --workload c5)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c4", "c3", "c5"],
                    help="c2: the urchin (default); c3: the many-urchin batch (see --surfaces); "
                         "c5: the urchin with its plan cached, one fresh density per step, "
                         "split-precision translations")
    ap.add_argument("--study", choices=["greens", "tcr", "scaling", "solve"], default=None,
                    help="greens: Green's-formula accuracy sweep over p_fmm x p_qbx on the "
                         "urchin; tcr: modeled cost and time of the ball-shaped vs the "
                         "box-shaped target confinement region, and of a level-restricted "
                         "tree; scaling: modeled cost (and "
                         "time, with a GPU) over urchins of growing size; solve: the interior "
                         "Dirichlet problem on an oversampled urchin by GMRES with "
                         "split-precision applies and FP64 refinement; instead of the timing "
                         "run")
    ap.add_argument("--level", type=int, default=4,
                    help="--study solve: icosphere level of the urchin's elements")
    ap.add_argument("--surfaces", type=int, default=8,
                    help="c3 only: how many of the 64 batch surfaces to evaluate")
    ap.add_argument("--nmax", type=int, default=None,
                    help="most particles (sources + centers + targets) of a box before it is "
                         "split; default: the measured optimum, 160 for the urchin workloads "
                         "with the rotation-form M2L (c2, c3), 192 with the dense one (and "
                         "c5), 256 for the ellipsoid (c4); the workload's own (512, the "
                         "paper's choice) for c1")
    ap.add_argument("--c3-modes", default="fp64,fp32_split,fp32_lead",
                    help="c3 only: precision modes of the batch plan, comma-separated (fp64 "
                         "first: its member plans are the plain FP64 ones)")
    ap.add_argument("--c3-direct", type=int, default=0,
                    help="c3 only: random centers per surface checked against the direct QBX "
                         "oracle, every density (0: none)")
    ap.add_argument("--cpu-sample", type=int, default=768,
                    help="centers evaluated by the CPU oracle (direct QBX) for the baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-c1", type=int, choices=[0, 1], default=1,
                    help="1 (default): also time the CPU oracles on the small sphere (4,800 "
                         "sources, S 3/10) in full: direct QBX on one core and on all cores, "
                         "and the step-by-step GIGAQBX oracle, beside this GPU on the same "
                         "workload (about 40 s of CPU)")
    ap.add_argument("--cpu-tier-b", type=int, default=0,
                    help="centers of the main workload evaluated by the step-by-step GIGAQBX "
                         "oracle (the algorithmic CPU baseline; 0: none; 64 take about 40 s "
                         "on 8 cores, tree and lists included)")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the split-precision (FP32 matrix-core) translation runs")
    ap.add_argument("--no-det", action="store_true",
                    help="skip the run of the deterministic plan (GQ_FLAG_DETERMINISTIC: "
                         "bitwise-reproducible applies)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain elementwise copy (y = -x) over 1 GiB, so that a "
                         "hardware-counter pass can scale its byte counters by a kernel of "
                         "known traffic")
    ap.add_argument("--wfar-direct-max", type=int, default=None,
                    help="Remark 4: List 3 far boxes with at most this many sources are "
                         "evaluated directly (0 disables). Default: for the urchin workloads "
                         "128 with the rotation-form M2L (c2, c3) and 64 with the dense one "
                         "(and c5), the measured optima for D 5/15 on the level-restricted "
                         "tree; for c1 and c4 the cost-model crossover, the "
                         "flops of one M2QBXL pair over those of one direct pair (89 at S "
                         "3/10, 335 at S 8/20)")
    ap.add_argument("--level-restrict", type=int, choices=[0, 1], default=1,
                    help="1 (default): level-restricted tree, adjacent leaves differ by at most "
                         "one level (the remark on List 3 complexity); 0: the adaptive tree as "
                         "built")
    ap.add_argument("--overlap", type=int, choices=[0, 1], default=0,
                    help="1: the far-field chain (P2M, M2M, M2L, P2L, L2L) runs on a second "
                         "stream beside the near field, and a few extra applies with every "
                         "stage in order on one stream report each kernel's time alone; "
                         "0 (default): every stage in order on one stream (no gain was "
                         "measured from the second stream)")
    ap.add_argument("--autotune", type=int, choices=[0, 1], default=0,
                    help="1: time the M2L launch at plan creation over tile widths 64 and 32, "
                         "with and without the XCD-aware order, and keep the fastest (outside "
                         "the timed region); 0 (default): the library's default tiles (width "
                         "64 for split FP32, 32 otherwise; XCD-aware order)")
    ap.add_argument("--autotune-tree", type=int, choices=[0, 1], default=0,
                    help="1: every plan chooses its nmax and Remark 4 threshold at creation "
                         "by timing candidate trees around the given values "
                         "(GQ_FLAG_AUTOTUNE_TREE; outside the timed region), and the values "
                         "kept are reported")
    ap.add_argument("--m2l-rotation", type=int, choices=[-1, 0, 1], default=-1,
                    help="1: FP64 M2L as rotate, translate along z, rotate back (three sparse "
                         "tile products) instead of one dense matrix per offset class; 0: "
                         "dense; -1 (default): rotation where it is built (FP64, p_fmm <= 15)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 200 if args.workload == "c5" else 10
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures a single GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1805_06106_amd import Plan
    from paper_1805_06106_amd import costmodel as CM

    if args.wfar_direct_max is None:
        # Remark 4's crossover: a W-far box of n sources is cheaper to evaluate directly
        # than through its multipole while n is below the flops of one (box, center) M2QBXL
        # pair over those of one direct (source, center) pair (72 at D 5/15, where 64 was
        # measured best on the urchin)
        orders = {"c1": (10, 3, "S"), "c4": (20, 8, "S")}
        if args.workload in orders and args.study is None:
            p, q, k = orders[args.workload]
            args.wfar_direct_max = round(CM.m2qbxl_pair(p, q) / CM.p2qbxl_pair(q, k))
        elif args.workload in ("c2", "c3") and args.m2l_rotation != 0 and args.study is None:
            # with the rotation-form M2L (28.6 ms per apply at 64 and nmax 192, 27.6 at 128
            # and nmax 160, same box)
            args.wfar_direct_max = 128
        else:
            args.wfar_direct_max = 64
    if args.nmax is None and args.study is None:
        # nmax measured on one MI355X (smaller leaves move work from the near field to M2L,
        # which the matrix cores run at a higher fraction of their peak): the urchin
        # workloads (D, 5/15) with the dense M2L 192 (32.3-32.5 ms per apply against 43.3 ms
        # at the paper's 512; 33.5 at 128, 36.6 at 256, 39.1 at 384), with the rotation-form
        # M2L 160 (27.8 ms against 28.6 at 192 and 27.8 at 176); the ellipsoid (S, 8/20) 256
        # (242.8 ms against 262.7 at 512 and 244.0 at 384)
        rot = args.m2l_rotation != 0
        args.nmax = {"c2": 160 if rot else 192, "c3": 160 if rot else 192, "c5": 192,
                     "c4": 256}.get(args.workload)

    if args.study == "scaling":
        return study_scaling(args)
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.study == "greens":
        return study_greens(args, dev)
    if args.study == "tcr":
        return study_tcr(args, dev)
    if args.study == "solve":
        return study_solve(args, dev)
    if args.workload == "c3":
        return bench_batch(args, dev)
    if args.workload == "c5":
        return bench_fresh_densities(args, dev)
    if args.calibrate_copy:
        n = 1 << 27
        x = torch.ones(n, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        log(f"calibration copy: read {n * 8} B, wrote {n * 8} B")
        del x, y
    t0 = time.time()
    w = make_workload(args.workload)
    log(f"workload {w.name}: {w.n_src} sources, {w.n_ctr} centers, {w.n_tgt} targets, "
        f"kernel {w.kernel}, p_qbx={w.p_qbx}, p_fmm={w.p_fmm} ({time.time() - t0:.1f}s)")
    dens = torch.tensor(w.density[:1], dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    # the FP64 M2L form: the rotation-factored kernel covers p_fmm <= 15
    rotation = args.m2l_rotation == 1 or (args.m2l_rotation == -1 and w.p_fmm <= 15)

    def run(precision, deterministic=False):
        t0 = time.time()
        plan = Plan.from_workload(w, timing=True, precision=precision,
                                  m2l_rotation=rotation and precision == "fp64",
                                  overlap=bool(args.overlap), autotune=bool(args.autotune),
                                  deterministic=deterministic, **tree_opts(args))
        plan_wall = time.time() - t0
        st = plan.stats()
        log(f"[{precision}] plan: {st['n_boxes']} boxes, {st['n_levels']} levels, pairs "
            f"{st['pairs']} ({plan_wall:.2f}s)")
        pot = torch.empty((1, w.n_tgt), dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            plan.apply(dens, pot, stream=stream)
        torch.cuda.synchronize()
        plan.stats()  # closes the warmup timing window
        log(f"[{precision}] warmup {args.warmup} done; timing {args.steps} steps")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.apply(dens, pot, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms_per_step = (t1 - t0) * 1e3 / args.steps
        st = plan.stats()
        k = max(st["timed_applies"], 1)
        stage_ms = {s: v / k for s, v in st["stage_ms"].items()}
        if deterministic:
            # outside the timed region: one more apply must reproduce the last bit for bit
            last = pot.clone()
            plan.apply(dens, pot, stream=stream)
            torch.cuda.synchronize()
            st["repeat_bitwise_equal"] = bool(torch.equal(last, pot))
        log(f"[{precision}] {ms_per_step:.2f} ms/step, {w.n_tgt / (ms_per_step * 1e-3):.4g} "
            f"target evals/s; stage ms {stage_ms}")
        alone = None
        if args.overlap:
            # outside the timed region: every stage in order on one stream, so that each
            # stage time is its kernel's alone
            plan.set_overlap(False)
            n_alone = min(args.steps, 5)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(n_alone):
                plan.apply(dens, pot, stream=stream)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st_a = plan.stats()
            ka = max(st_a["timed_applies"], 1)
            alone = {"ms_per_step": (t1 - t0) * 1e3 / n_alone, "steps": n_alone,
                     "stage_ms": {s: v / ka for s, v in st_a["stage_ms"].items()}}
            log(f"[{precision}] one stream: {alone['ms_per_step']:.2f} ms/step; stage ms "
                f"{alone['stage_ms']}")
        if precision == "fp64" and not deterministic:
            # outside the timed region: the density copied in from pinned host memory and
            # the potentials copied back over PCIe around each apply, as a caller holding
            # host arrays sees it
            hd = torch.empty(tuple(dens.shape), dtype=torch.float64, pin_memory=True)
            hd.copy_(dens.cpu())
            hp = torch.empty(tuple(pot.shape), dtype=torch.float64, pin_memory=True)
            n_e2e = min(args.steps, 5)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(n_e2e):
                dens.copy_(hd, non_blocking=True)
                plan.apply(dens, pot, stream=stream)
                hp.copy_(pot, non_blocking=True)
            torch.cuda.synchronize()
            st["end_to_end_ms"] = (time.perf_counter() - t0) * 1e3 / n_e2e
            log(f"[{precision}] with host transfers: {st['end_to_end_ms']:.2f} ms per apply")
        plan.close()
        return ms_per_step, stage_ms, st, plan_wall, pot, alone

    ms_per_step, stage_ms, st, plan_wall, pot, alone = run("fp64")
    value = w.n_tgt / (ms_per_step * 1e-3)

    flops = CM.apply_flops(st, w.p_fmm, w.p_qbx, w.kernel)
    kern_stage = {"p2qbxl": "p2qbxl", "m2qbxl": "m2qbxl", "m2l": "m2l", "l2qbxl": "l2qbxl"}
    dominant = max(kern_stage, key=lambda s: stage_ms[kern_stage[s]])
    dom_ms = stage_ms[kern_stage[dominant]]
    achieved = flops[dominant] / (dom_ms * 1e-3) / 1e12
    roofline = {"kernel": dominant, "bound": "mfma" if dominant == "m2l" else "alu",
                "achieved": round(achieved, 3),
                "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_VALU_TFLOPS, 4),
                "traffic": counter_traffic(dominant, w.name, args.wfar_direct_max,
                                           bool(args.level_restrict), args.nmax or w.nmax,
                                           rotation),
                "flops_per_launch": flops[dominant], "ms_per_launch": round(dom_ms, 4)}
    if alone:
        # the same kernel with the far field not running beside it
        a_ms = alone["stage_ms"][kern_stage[dominant]]
        roofline["ms_per_launch_alone"] = round(a_ms, 4)
        roofline["frac_alone"] = round(flops[dominant] / (a_ms * 1e-3) / 1e12
                                       / PEAK_FP64_VALU_TFLOPS, 4)
    per_stage = {}
    for s, f in flops.items():
        ms = stage_ms[kern_stage.get(s, s)]
        per_stage[s] = {"ms": round(ms, 4), "tflops": round(f / (ms * 1e-3) / 1e12, 3) if ms > 0 else None}
    # matrix-core use: the executed flops (the dense product's, or the rotation's three
    # sparse products) over the time and the FP64 MFMA peak
    m2l_exec = (st["pairs"]["V"] * CM.rotation_m2l_pair(w.p_fmm) if rotation
                else flops["m2l"])
    m2l = {"engine": "fp64 mfma (v_mfma_f64_16x16x4f64)"
                     + (", rotation-factored" if rotation else ", dense"),
           "ms": round(stage_ms["m2l"], 4),
           "dense_equivalent_tflops": per_stage["m2l"]["tflops"],
           "executed_flops": m2l_exec,
           "frac_of_fp64_mfma_peak": round(m2l_exec / (stage_ms["m2l"] * 1e-3) / 1e12
                                           / PEAK_FP64_VALU_TFLOPS, 4)
           if stage_ms["m2l"] > 0 else None}
    if alone:
        m2l["ms_alone"] = round(alone["stage_ms"]["m2l"], 4)
        m2l["frac_of_fp64_mfma_peak_alone"] = round(
            m2l_exec / (alone["stage_ms"]["m2l"] * 1e-3) / 1e12 / PEAK_FP64_VALU_TFLOPS, 4)

    # FP32 matrix-core translations: split (leading degrees in FP64, hi/lo correction
    # products with FP64 accumulation per K-step), leading degrees only, and uncorrected
    m2l_gemm_flops = flops["m2l"]
    split = {}
    if not args.no_fp32:
        p64 = pot[0].clone()
        npc = (w.p_fmm + 1) ** 2
        lead = min(16, npc)
        for prec in ("fp32_split", "fp32_lead", "fp32"):
            ms_p, sm_p, _, _, pot_p, alone_p = run(prec)
            if alone_p:
                sm_p = alone_p["stage_ms"]  # the M2L kernel's own time
            err = float((pot_p[0] - p64).abs().max() / p64.abs().max())
            m2l_ms = sm_p["m2l"]
            eff = m2l_gemm_flops / (m2l_ms * 1e-3) / 1e12
            # executed matrix-core work: FP32 products over the trailing columns, FP64 over
            # the leading ones
            tail = (npc - lead) / npc if prec != "fp32" else 1.0
            products = 3 if prec == "fp32_split" else 1
            f32_tf = eff * tail * products
            f64_tf = eff * (1.0 - tail)
            split[prec] = {
                "value": round(w.n_tgt / (ms_p * 1e-3), 1), "ms_per_step": round(ms_p, 4),
                "rel_err_vs_fp64_path": err,
                "ms_per_step_one_stream": round(alone_p["ms_per_step"], 4) if alone_p else None,
                "m2l": {"ms": round(m2l_ms, 4), "fp32_products_per_trailing_column": products,
                        "leading_fp64_columns": lead if prec != "fp32" else 0,
                        "executed_fp32_tflops": round(f32_tf, 3),
                        "executed_fp64_tflops": round(f64_tf, 3),
                        "effective_tflops": round(eff, 3),
                        "frac_of_mfma_peak": round(f32_tf / PEAK_FP32_MFMA_TFLOPS
                                                   + f64_tf / PEAK_FP64_VALU_TFLOPS, 4)},
                ("stage_ms_one_stream" if alone_p else "stage_ms"):
                    {s: round(v, 4) for s, v in sm_p.items()},
            }
            log(f"[{prec}] rel err vs fp64 path {err:.3e}")

    # reproducible applies (GQ_FLAG_DETERMINISTIC): per-pair slots and ordered sums
    det = None
    if not args.no_det:
        ms_d, sm_d, st_d, _, pot_d, _ = run("fp64", deterministic=True)
        det = {"value": round(w.n_tgt / (ms_d * 1e-3), 1), "ms_per_step": round(ms_d, 4),
               "repeat_bitwise_equal": st_d["repeat_bitwise_equal"],
               "rel_diff_vs_atomic_path": float((pot_d[0] - pot[0]).abs().max()
                                                / pot[0].abs().max()),
               "device_bytes": st_d.get("device_bytes"),
               "stage_ms": {s: round(v, 4) for s, v in sm_d.items()}}
        log(f"[deterministic] {ms_d:.2f} ms/step; repeat bitwise equal "
            f"{det['repeat_bitwise_equal']}; vs atomic {det['rel_diff_vs_atomic_path']:.2e}")

    cpu = None
    err_direct = None
    if not args.no_cpu_baseline:
        import oracle as O

        rng = np.random.default_rng(12345)
        cids = np.sort(rng.choice(w.n_ctr, args.cpu_sample, replace=False))
        log(f"cpu baseline: direct QBX oracle on {len(cids)} centers")
        t0 = time.perf_counter()
        tids, ref, used = O.direct_qbx_sampled(w, cids, density_index=0,
                                               nthreads=int(os.environ.get("OMP_NUM_THREADS", "0")))
        dt = time.perf_counter() - t0
        got = pot[0].cpu().numpy()[tids]
        err_direct = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        model = next((ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo")
                      if ln.startswith("model name")), "unknown")
        cpu = {"value": round(len(tids) / dt, 3), "unit": "target evals/s", "cores": int(used),
               "kind": "oracle", "cpu_model": model,
               "sample": f"direct (unaccelerated) FP64 QBX on {len(cids)} random centers of "
                         f"{w.n_ctr}, each from all {w.n_src} sources; {dt:.1f}s"}
        log(f"cpu baseline {cpu['value']} evals/s on {used} threads; rel err vs direct {err_direct:.3e}")
        if args.cpu_tier_b > 0:
            cpu["tier_b"] = cpu_tier_b_sample(args, w, pot[0].cpu().numpy(), int(used))
        if args.cpu_c1:
            cpu["c1"] = cpu_c1(args, dev)

    out = {
        "metric": "QBX-FMM target evals/sec at stated rel. error; M2L MFMA util (FP32 vs FP64)",
        "value": round(value, 1),
        "unit": "target evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "kernel": w.kernel, "p_qbx": w.p_qbx, "p_fmm": w.p_fmm,
                   "n_sources": w.n_src, "n_centers": w.n_ctr, "n_targets": w.n_tgt,
                   "nmax": args.nmax or w.nmax, "tcf": w.tcf, "n_densities": 1, "precision": "fp64",
                   "wfar_direct_max": args.wfar_direct_max,
                   "level_restrict": bool(args.level_restrict),
                   "m2l_rotation": rotation,
                   "m2l_autotune": bool(args.autotune),
                   "m2l_tile": [st.get("m2l_tile_cols"), st.get("m2l_xcd_order")],
                   "tree_autotuned": ({"nmax": st.get("nmax"),
                                       "wfar_direct_max": st.get("wfar_direct_max")}
                                      if args.autotune_tree else None),
                   "schedule": ("near and far field on two streams" if args.overlap
                                else "one stream")},
        "rel_err_vs_direct_qbx": err_direct,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "m2l": m2l,
        "split_precision": split,
        "deterministic": det,
        "stages": per_stage,
        "stage_ms": {s: round(v, 4) for s, v in stage_ms.items()},
        "one_stream": ({"ms_per_step": round(alone["ms_per_step"], 4), "steps": alone["steps"],
                        "stage_ms": {s: round(v, 4) for s, v in alone["stage_ms"].items()}}
                       if alone else None),
        "plan_seconds": round(plan_wall, 3),
        # not `value`: the same apply with the density in and the potentials out over PCIe
        "end_to_end": {"ms_per_apply": round(st["end_to_end_ms"], 4),
                       "value": round(w.n_tgt / (st["end_to_end_ms"] * 1e-3), 1),
                       "unit": "target evals/s",
                       "includes": "density host-to-device and potentials device-to-host "
                                   "copies (pinned host buffers) around each apply; the "
                                   "plan (plan_seconds) is built once and cached"},
        "tree": {"boxes": st["n_boxes"], "levels": st["n_levels"], "pairs": st["pairs"]},
    }
    print(json.dumps(out), flush=True)


def cpu_tier_b_sample(args, w, got, cores):
    """The step-by-step GIGAQBX oracle on a random sample of centers of the main workload,
    with the plan's tree options, on all host cores: the algorithmic CPU baseline."""
    import numpy as np

    from oracle.gigaqbx import OracleFMM

    rng = np.random.default_rng(54321)
    cids = np.sort(rng.choice(w.n_ctr, args.cpu_tier_b, replace=False))
    log(f"cpu tier b: step-by-step oracle on {len(cids)} centers")
    t0 = time.perf_counter()
    F = OracleFMM(w, nmax=args.nmax or w.nmax, wfar_direct_max=args.wfar_direct_max,
                  level_restrict=bool(args.level_restrict))
    t1 = time.perf_counter()
    tids, ref, _ = F.evaluate(0, centers=cids)
    dt = time.perf_counter() - t0
    err = float(np.max(np.abs(got[tids] - ref)) / np.max(np.abs(ref)))
    out = {"value": round(len(tids) / dt, 4), "unit": "target evals/s",
           "cores": cores, "kind": "oracle (step-by-step GIGAQBX)",
           "sample": f"{len(cids)} random centers of {w.n_ctr}; tree and lists "
                     f"{t1 - t0:.1f}s, evaluation {dt - (t1 - t0):.1f}s",
           "gpu_rel_err_vs_it": err}
    log(f"cpu tier b {out['value']} evals/s ({dt:.1f}s); GPU vs it {err:.3e}")
    return out


def cpu_c1(args, dev):
    """The small sphere (4,800 sources, 9,600 targets, single layer, 3/10) in full: direct
    QBX on one core and on all cores, the step-by-step GIGAQBX oracle on one thread, and the
    GPU apply on the same inputs."""
    import numpy as np
    import torch

    import oracle as O
    from oracle.gigaqbx import OracleFMM
    from paper_1805_06106_amd import Plan

    w = make_workload("c1")
    cids = np.arange(w.n_ctr)
    # all cores first: a one-thread request stays in force for the process's later calls
    t0 = time.perf_counter()
    tids, ref, used_n = O.direct_qbx_sampled(
        w, cids, density_index=0,
        nthreads=int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count())
    dn = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, ref_1, used1 = O.direct_qbx_sampled(w, cids, density_index=0, nthreads=1)
    d1 = time.perf_counter() - t0
    assert np.array_equal(tids, np.arange(w.n_tgt))
    scale = np.max(np.abs(ref))
    res = {"workload": w.name, "n_sources": w.n_src, "n_targets": w.n_tgt,
           "direct_1core_vs_all_cores": float(np.max(np.abs(ref_1 - ref)) / scale)}
    t0 = time.perf_counter()
    F = OracleFMM(w, nthreads=1)
    tb_ids, tb, _ = F.evaluate(0)
    db = time.perf_counter() - t0
    tb_full = np.empty(w.n_tgt)
    tb_full[tb_ids] = tb
    plan = Plan.from_workload(w, timing=False)
    dens = torch.tensor(w.density[:1], dtype=torch.float64, device=dev)
    pot = torch.empty((1, w.n_tgt), dtype=torch.float64, device=dev)
    for _ in range(3):
        plan.apply(dens, pot)
    torch.cuda.synchronize()
    n = 50
    t0 = time.perf_counter()
    for _ in range(n):
        plan.apply(dens, pot)
    torch.cuda.synchronize()
    dg = (time.perf_counter() - t0) / n
    got = pot[0].cpu().numpy()
    plan.close()
    res.update({
        "direct_1core": {"value": round(w.n_tgt / d1, 1), "cores": int(used1), "seconds": round(d1, 2)},
        "direct_all_cores": {"value": round(w.n_tgt / dn, 1), "cores": int(used_n),
                             "seconds": round(dn, 2)},
        "tier_b_1thread": {"value": round(w.n_tgt / db, 1), "cores": 1, "seconds": round(db, 2),
                           "rel_err_vs_direct": float(np.max(np.abs(tb_full - ref)) / scale)},
        "gpu": {"value": round(w.n_tgt / dg, 1), "ms_per_apply": round(dg * 1e3, 4),
                "rel_err_vs_direct": float(np.max(np.abs(got - ref)) / scale)},
        "unit": "target evals/s",
    })
    log(f"c1 in full: direct {res['direct_1core']['value']} evals/s on 1 core, "
        f"{res['direct_all_cores']['value']} on {used_n}; tier b {res['tier_b_1thread']['value']} "
        f"on 1 thread; GPU {res['gpu']['value']} ({dg * 1e3:.3f} ms)")
    return res


def study_greens(args, dev):
    """Green's formula on the urchin (the accuracy experiment of Section 6.1): for u the
    potential of a unit charge at (3, 1, 2), outside the surface, u = S(du/dn) - D(u) holds
    inside, so at every density node x, evaluated through its interior center,
        E(x) = S(du/dn)(x) - D(u)(x) - u(x)
    vanishes up to the discretization, truncation and acceleration errors.  The surface is
    discretized as the paper's stage-2 pair: u and du/dn live on 45 nodes per element
    (degree 8) and the layer potentials use an oversampled quadrature on the same elements
    (the degree-8 collapsed rule on each of 64 sub-triangles).  Reported: max |E| / max |u|
    for each p_fmm x p_qbx (p_qbx <= p_fmm), beside the a-priori factor (3/4)^(p_fmm + 1)
    of the acceleration error."""
    import numpy as np
    import torch

    from paper_1805_06106_amd import Plan
    from workloads import oversampled_workload
    from workloads.geometry import SurfaceSpec

    spec = SurfaceSpec(curved=True, bump_k=8, bump_m=4, bump_a=0.2)
    x0 = np.array([3.0, 1.0, 2.0])
    t0 = time.time()
    w = oversampled_workload(f"urchin8-{20 * 4 ** args.level}-stage2", level=args.level,
                             spec=spec, kernel="S", p_qbx=3, p_fmm=3, node_order=8,
                             quad_order=8, sub=8, sides="interior")
    d = w.node_xyz - x0
    r = np.linalg.norm(d, axis=1)
    u = 1.0 / r
    dens = {"D": u, "S": -np.sum(d * w.node_normal, axis=1) / r ** 3}
    log(f"{w.name}: {w.n_src} sources, {w.n_ctr} nodes ({time.time() - t0:.1f}s)")
    rows = []
    for p_fmm in (3, 5, 10, 15, 20):
        for p_qbx in (3, 5, 7, 9):
            if p_qbx > p_fmm:
                continue
            t0 = time.time()
            pots = {}
            for kern in ("S", "D"):
                P = Plan.from_workload(w, kernel=kern, p_qbx=p_qbx, p_fmm=p_fmm,
                                       **tree_opts(args))
                pots[kern] = P.apply(torch.tensor(dens[kern][None, :],
                                                  device=dev))[0].cpu().numpy()
                P.close()
            meta = (w.name, w.n_src, w.n_ctr)
            E = pots["S"] - pots["D"] - u
            err = float(np.max(np.abs(E)) / np.max(np.abs(u)))
            rows.append({"p_fmm": p_fmm, "p_qbx": p_qbx, "rel_err": err,
                         "bound_factor": 0.75 ** (p_fmm + 1)})
            log(f"p_fmm={p_fmm:2d} p_qbx={p_qbx}: {err:.3e}  ({time.time() - t0:.1f}s)")
    print(json.dumps({"study": "greens_formula", "workload": meta[0], "n_sources": meta[1],
                      "n_targets": meta[2], "charge": x0.tolist(), "nmax": args.nmax or 512,
                      "tcf": 0.9, "wfar_direct_max": args.wfar_direct_max,
                      "level_restrict": bool(args.level_restrict), "rows": rows}), flush=True)


def study_scaling(args):
    """Cost scaling over the urchin family (Section 6, modeled operation counts over
    gamma_2 ... gamma_10): bump orders k = 2..10, icosphere levels growing with k, single
    layer, p_qbx = 5, p_fmm = 15, nmax 512, t_f 0.9, Remark 4 off.  Reports the Table 7
    model per list and per source (host plans); with a GPU also the measured apply time."""
    import torch

    from paper_1805_06106_amd import Plan
    from paper_1805_06106_amd import costmodel as CM
    from workloads.geometry import SurfaceSpec, make_workload

    gpu = torch.cuda.is_available()
    rows = []
    for k, level in ((2, 3), (4, 4), (6, 4), (8, 5), (10, 5), (10, 6)):
        w = make_workload(f"urchin{k}-L{level}", level=level, order=6,
                          spec=SurfaceSpec(curved=True, bump_k=k, bump_m=k // 2, bump_a=0.2),
                          kernel="S", p_qbx=5, p_fmm=15, seed=100 + k, density="ones")
        t0 = time.time()
        P = Plan.from_workload(w, host_only=not gpu, timing=gpu)
        plan_s = time.time() - t0
        st = P.stats()
        model = CM.paper_list_model(st, w.p_fmm, w.p_qbx)
        # the lists do not depend on the orders: the same plan gives the (9, 20) model
        model_hi = CM.paper_list_model(st, 20, 9)
        row = {"k": k, "level": level, "n_sources": w.n_src, "n_boxes": st["n_boxes"],
               "model": model, "model_per_source": model["total_lists"] / w.n_src,
               "model_q9_p20": model_hi,
               "model_q9_p20_per_source": model_hi["total_lists"] / w.n_src,
               "plan_seconds": round(plan_s, 2)}
        if gpu:
            d = torch.ones((1, w.n_src), dtype=torch.float64, device="cuda:0")
            pot = torch.empty((1, w.n_tgt), dtype=torch.float64, device="cuda:0")
            P.apply(d, pot)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                P.apply(d, pot)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / args.steps
            row["ms_per_apply"] = round(ms, 3)
            row["ns_per_target"] = round(ms * 1e6 / w.n_tgt, 3)
        P.close()
        rows.append(row)
        log(f"k={k} level={level}: N_S={w.n_src}, modeled {model['total_lists']:.3e} "
            f"({row['model_per_source']:.3e}/source)" + (f", {row['ms_per_apply']} ms" if gpu else ""))
    print(json.dumps({"study": "cost_scaling", "orders": [[5, 15], [9, 20]], "kernel": "S",
                      "rows": rows}), flush=True)


def study_tcr(args, dev):
    """The cost comparison of Section 6 (Table 8) on the urchin: modeled operation counts
    per interaction list (Table 7 model) and measured apply time, for the ball-shaped TCR
    of this method and the box-shaped TCR of the earlier algorithm, and for the ball with a
    level-restricted tree (the remark on List 3 complexity).  Remark 4 is off for all, so
    the lists are the plain ones."""
    import numpy as np
    import torch

    from paper_1805_06106_amd import Plan
    from paper_1805_06106_amd import costmodel as CM
    from workloads import workload_c2

    w = workload_c2()
    dens = torch.tensor(w.density[:1], device=dev)
    out = {"study": "tcr_shape", "workload": w.name, "p_fmm": w.p_fmm, "p_qbx": w.p_qbx,
           "nmax": w.nmax, "tcf": w.tcf, "rows": {}}
    pots = {}
    variants = {"linf": dict(tcr_norm="linf"), "l2": dict(tcr_norm="l2"),
                "l2_level_restricted": dict(tcr_norm="l2", level_restrict=True)}
    for tcr, kw in variants.items():
        P = Plan.from_workload(w, timing=True, overlap=False, **kw)  # stage times alone
        st = P.stats()
        model = CM.paper_list_model(st, w.p_fmm, w.p_qbx)
        pot = torch.empty((1, w.n_tgt), dtype=torch.float64, device=dev)
        P.apply(dens, pot)
        torch.cuda.synchronize()
        P.stats()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            P.apply(dens, pot)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        st2 = P.stats()
        k = max(st2["timed_applies"], 1)
        pots[tcr] = pot[0].cpu().numpy()
        out["rows"][tcr] = {"model": model, "ms_per_apply": round(ms, 3),
                            "stage_ms": {s: round(v / k, 3) for s, v in st2["stage_ms"].items()},
                            "n_boxes": st["n_boxes"], "n_suspended_centers":
                            st["n_suspended_centers"], "pairs": st["pairs"]}
        log(f"{tcr}: modeled {model['total_lists']:.3e}, {ms:.2f} ms/apply")
        P.close()
    out["model_ratio_l2_over_linf"] = (out["rows"]["l2"]["model"]["total_lists"]
                                       / out["rows"]["linf"]["model"]["total_lists"])
    out["time_ratio_l2_over_linf"] = (out["rows"]["l2"]["ms_per_apply"]
                                      / out["rows"]["linf"]["ms_per_apply"])
    out["rel_diff_potentials"] = float(np.max(np.abs(pots["l2"] - pots["linf"]))
                                       / np.max(np.abs(pots["l2"])))
    out["rel_diff_level_restricted"] = float(np.max(np.abs(pots["l2"] - pots["l2_level_restricted"]))
                                             / np.max(np.abs(pots["l2"])))
    print(json.dumps(out), flush=True)


def bench_fresh_densities(args, dev):
    """The urchin with its plan cached and a fresh density for every apply (split-precision
    translations, translation matrices resident in HBM): all densities are uploaded before
    the timed region, and step i applies density i."""
    import numpy as np
    import torch

    from paper_1805_06106_amd import Plan
    from workloads import fresh_densities, workload_c2

    t0 = time.time()
    w = workload_c2()
    n = args.warmup + args.steps
    dens = torch.tensor(fresh_densities(w, n), device=dev)
    log(f"workload {w.name}: {w.n_src} sources, {w.n_tgt} targets, {n} fresh densities "
        f"({time.time() - t0:.1f}s)")
    t0 = time.time()
    plan = Plan.from_workload(w, **tree_opts(args), precision="fp32_split",
                              autotune=bool(args.autotune))
    plan_s = time.time() - t0
    out = torch.empty((n, w.n_tgt), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    for i in range(args.warmup):
        plan.apply(dens[i:i + 1], out[i:i + 1], stream=stream)
    torch.cuda.synchronize()
    log(f"plan {plan_s:.2f}s; warmup {args.warmup} done; timing {args.steps} steps")
    t = time.perf_counter()
    for i in range(args.warmup, n):
        plan.apply(dens[i:i + 1], out[i:i + 1], stream=stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / args.steps
    plan.close()
    # accuracy: the last density through the FP64 path, and through direct QBX on a sample
    ref64 = Plan.from_workload(w, **tree_opts(args))
    last = ref64.apply(dens[n - 1:n])[0]
    err64 = float((out[n - 1] - last).abs().max() / last.abs().max())
    ref64.close()
    err_direct = None
    if not args.no_cpu_baseline:
        import dataclasses

        import oracle as O

        rng = np.random.default_rng(12345)
        cids = np.sort(rng.choice(w.n_ctr, 128, replace=False))
        wl = dataclasses.replace(w, density=dens[n - 1:n].cpu().numpy())
        tids, ref, _ = O.direct_qbx_sampled(wl, cids, density_index=0)
        got = out[n - 1].cpu().numpy()[tids]
        err_direct = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    log(f"{ms:.2f} ms per apply, {w.n_tgt / (ms * 1e-3):.4g} target evals/s; rel err vs FP64 "
        f"path {err64:.3e}, vs direct QBX {err_direct}")
    print(json.dumps({
        "metric": "QBX-FMM target evals/sec at stated rel. error; M2L MFMA util (FP32 vs FP64)",
        "value": round(w.n_tgt / (ms * 1e-3), 1), "unit": "target evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}, plan cached, fresh density per apply",
                   "kernel": w.kernel, "p_qbx": w.p_qbx, "p_fmm": w.p_fmm,
                   "n_sources": w.n_src, "n_targets": w.n_tgt, "precision": "fp32_split",
                   "densities": n, "wfar_direct_max": args.wfar_direct_max,
                   "level_restrict": bool(args.level_restrict),
                   "m2l_autotune": bool(args.autotune)},
        "rel_err_vs_fp64_path": err64, "rel_err_vs_direct_qbx": err_direct,
        "plan_seconds": round(plan_s, 3)}), flush=True)


def study_solve(args, dev):
    """The interior Dirichlet problem on an oversampled urchin (rho = 1 + 0.2 Re Y_8^4):
    boundary values of u = 1 / (4 pi |x - x0|), x0 = (3, 1, 2); u = D[mu] with the interior
    limit taken through the interior QBX centers; GMRES on split-precision applies, residuals
    refined with the FP64 path, to a relative residual of 1e-10 within 200 applies.  D[mu] is
    then compared with u at points inside."""
    import dataclasses

    import numpy as np
    import torch

    from paper_1805_06106_amd import Plan
    from paper_1805_06106_amd.solve import gmres_ir, plan_operator
    from workloads import oversampled_workload
    from workloads.geometry import SurfaceSpec

    t0 = time.time()
    spec = SurfaceSpec(curved=True, bump_k=8, bump_m=4, bump_a=0.2)
    w = oversampled_workload(f"urchin8-{20 * 4 ** args.level}-oversampled", level=args.level,
                             spec=spec, kernel="D", p_qbx=5, p_fmm=15, node_order=4,
                             quad_order=4, sub=4, sides="interior")
    log(f"{w.name}: {w.n_tgt} density nodes, {w.n_src} quadrature sources "
        f"({time.time() - t0:.1f}s)")
    x0 = np.array([3.0, 1.0, 2.0])
    g_np = 1.0 / (4 * np.pi * np.linalg.norm(w.node_xyz - x0, axis=1))
    g = torch.tensor(g_np, device=dev)
    t0 = time.time()
    hi = Plan.from_workload(w, **tree_opts(args))
    lo = Plan.from_workload(w, **tree_opts(args), precision="fp32_split")
    plan_s = time.time() - t0
    A_hi, A_lo = plan_operator(hi), plan_operator(lo)
    for A in (A_hi, A_lo):  # warm
        A(g)
    torch.cuda.synchronize()
    t = time.perf_counter()
    mu, info = gmres_ir(A_lo, A_hi, g, tol=1e-10, inner_tol=1e-6, max_applies=200)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - t
    ms = {}
    for name, A in (("fp64", A_hi), ("fp32_split", A_lo)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            A(g)
        torch.cuda.synchronize()
        ms[name] = round((time.perf_counter() - t) * 200, 3)
    rng = np.random.default_rng(8)
    v = rng.standard_normal((256, 3))
    pts = v / np.linalg.norm(v, axis=1)[:, None] * rng.uniform(0.1, 0.6, 256)[:, None]
    wp = dataclasses.replace(w, tgt_xyz=pts, tgt_center=np.full(len(pts), -1, dtype=np.int64))
    u = Plan.from_workload(wp).apply(mu.reshape(1, -1)).cpu().numpy()[0]
    exact = 1.0 / (4 * np.pi * np.linalg.norm(pts - x0, axis=1))
    err = float(np.max(np.abs(u - exact)) / np.max(np.abs(exact)))
    log(f"solve {solve_s:.2f}s, residuals {info['outer_residuals']}, inner "
        f"{info['inner_iterations']}; interior error {err:.3e}")
    print(json.dumps({"study": "interior_dirichlet_gmres_ir", "workload": w.name,
                      "n_nodes": w.n_tgt, "n_sources": w.n_src, "p_qbx": 5, "p_fmm": 15,
                      "oversampling": "15-node interior lattice -> 16 x 15-node rule",
                      "charge": x0.tolist(), "tol": 1e-10, "converged": info["converged"],
                      "outer_residuals": info["outer_residuals"],
                      "inner_iterations": info["inner_iterations"],
                      "applies_fp32_split": info["applies_lo"], "applies_fp64": info["applies_hi"],
                      "ms_per_apply": ms, "solve_seconds": round(solve_s, 3),
                      "plan_seconds": round(plan_s, 3), "interior_rel_err": err}), flush=True)


def c3_workloads(count):
    """The first `count` surfaces of the 64-urchin batch, generated by up to 16 worker
    processes (spawned, so that none inherits the parent's GPU state)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    from workloads import workload_c3

    if count <= 2:
        return [workload_c3(i) for i in range(count)]
    # largest surfaces first, so that the pool ends evenly
    from workloads.geometry import c3_surface_params
    order = sorted(range(count), key=lambda i: -c3_surface_params(i)[3])
    with ProcessPoolExecutor(max_workers=min(16, count),
                             mp_context=mp.get_context("spawn")) as ex:
        made = dict(zip(order, ex.map(workload_c3, order)))
    return [made[i] for i in range(count)]


def bench_batch(args, dev):
    """Many surfaces with 8 densities each: plain FP64 (one plan per surface, applied one
    after another) against one batch plan per precision mode (HIP graph, autotuned M2L).
    Member plans are released once their batch exists, so at most one precision's members
    and batch are held at a time.  The stated error is measured against the plain FP64
    potentials on every target and against the direct (unaccelerated) QBX oracle on a
    sample of targets of every surface and every density."""
    import numpy as np
    import torch

    from paper_1805_06106_amd import Plan

    t0 = time.time()
    ws = c3_workloads(args.surfaces)
    nd = ws[0].density.shape[0]
    n_tgt = sum(w.n_tgt for w in ws)
    n_src = sum(w.n_src for w in ws)
    log(f"batch workload: {len(ws)} surfaces, {n_src} sources, {n_tgt} targets, {nd} densities "
        f"({time.time() - t0:.1f}s)")
    dall = torch.cat([torch.tensor(w.density) for w in ws], dim=1).to(dev).contiguous()
    offs_s = np.cumsum([0] + [w.n_src for w in ws])
    offs_t = np.cumsum([0] + [w.n_tgt for w in ws])

    def timed(fn, k):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / k

    from concurrent.futures import ThreadPoolExecutor

    # the FP64 M2L form, as for the single surface
    rotation = args.m2l_rotation == 1 or (args.m2l_rotation == -1 and ws[0].p_fmm <= 15)

    def make_plans(prec):
        # host planning runs in the library without the GIL: 8 plans at a time
        out = [None] * len(ws)

        def one(k):
            out[k] = Plan.from_workload(ws[k], n_densities=nd, precision=prec,
                                        m2l_rotation=rotation and prec == "fp64",
                                        **tree_opts(args))
            return k

        with ThreadPoolExecutor(max_workers=8) as ex:
            for i, _ in enumerate(ex.map(one, range(len(ws)))):
                if i % 8 == 7:
                    log(f"[{prec}] {i + 1} of {len(ws)} plans")
        return out

    # plain FP64: one plan per surface, applied one after another
    t0 = time.time()
    plans = make_plans("fp64")
    plan64_s = time.time() - t0
    ref = torch.empty((nd, n_tgt), dtype=torch.float64, device=dev)
    dsl = [dall[:, offs_s[k]:offs_s[k + 1]].contiguous() for k in range(len(ws))]
    osl = [torch.empty((nd, w.n_tgt), dtype=torch.float64, device=dev) for w in ws]

    def plain():
        for P, d, o in zip(plans, dsl, osl):
            P.apply(d, o)

    ms_plain = timed(plain, args.steps)
    for k, o in enumerate(osl):
        ref[:, offs_t[k]:offs_t[k + 1]] = o
    del dsl, osl
    log(f"plain fp64: {ms_plain:.2f} ms per batch apply ({plan64_s:.1f}s of plans)")
    res = {}
    pots = {}
    for prec in args.c3_modes.split(","):
        t0 = time.time()
        members = plans if prec == "fp64" else make_plans(prec)
        log(f"[{prec}] merging {len(members)} plans into one batch plan")
        B = Plan.batch(members, graph=True, autotune=True)
        for P in members:
            P.close()
        plans = []
        plan_s = time.time() - t0
        st = B.stats()
        out = torch.empty((nd, n_tgt), dtype=torch.float64, device=dev)
        ms = timed(lambda: B.apply(dall, out), args.steps)
        err = float((out - ref).abs().max() / ref.abs().max())
        res[prec] = {"value": round(nd * n_tgt / (ms * 1e-3), 1), "ms_per_apply": round(ms, 3),
                     "rel_err_vs_plain_fp64": err, "plan_seconds": round(plan_s, 2),
                     "device_bytes": st["device_bytes"],
                     "m2l_tile_cols": st["m2l_tile_cols"], "m2l_xcd_order": st["m2l_xcd_order"],
                     "m2l_classes": st["m2l_classes"]}
        log(f"batched {prec} + graph: {ms:.2f} ms per apply, rel err vs plain fp64 {err:.3e}")
        pots[prec] = out.cpu().numpy() if args.c3_direct > 0 else None
        B.close()
        del out
    for P in plans:  # the plain plans, if no FP64 batch took them over
        P.close()
    direct = None
    if args.c3_direct > 0:
        import oracle as O

        # Tier A: args.c3_direct random centers per surface, every density
        t0 = time.time()
        worst = {p: 0.0 for p in pots}
        worst_plain = 0.0
        refc = ref.cpu().numpy()
        rng = np.random.default_rng(777)
        for k, w in enumerate(ws):
            cids = np.sort(rng.choice(w.n_ctr, args.c3_direct, replace=False))
            for d in range(nd):
                tids, dref, _ = O.direct_qbx_sampled(w, cids, density_index=d)
                scale = np.max(np.abs(dref))
                worst_plain = max(worst_plain, float(np.max(np.abs(
                    refc[d, offs_t[k] + tids] - dref)) / scale))
                for p, pot in pots.items():
                    worst[p] = max(worst[p], float(np.max(np.abs(
                        pot[d, offs_t[k] + tids] - dref)) / scale))
            if k % 8 == 7:
                log(f"direct QBX sample: {k + 1} of {len(ws)} surfaces ({time.time() - t0:.0f}s)")
        direct = {"centers_per_surface": args.c3_direct, "densities": nd,
                  "max_rel_err_plain_fp64": worst_plain,
                  **{f"max_rel_err_batched_{p}": v for p, v in worst.items()},
                  "seconds": round(time.time() - t0, 1)}
        log(f"vs direct QBX (worst surface and density): {direct}")
    # the headline form is the batched FP32 split; with --c3-modes without it, the first mode
    head = "fp32_split" if "fp32_split" in res else next(iter(res))
    out = {
        "metric": f"QBX-FMM target evals/sec, batched {head} translations (hipGraph) vs "
                  "plain FP64",
        "value": res[head]["value"],
        "unit": "target evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res[head]["ms_per_apply"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"urchin-batch-{len(ws)}-of-64", "kernel": "D", "p_qbx": 5,
                   "p_fmm": 15, "n_surfaces": len(ws), "n_densities": nd,
                   "n_sources": n_src, "n_targets": n_tgt,
                   "levels": [w.meta["level"] for w in ws],
                   "wfar_direct_max": args.wfar_direct_max,
                   "level_restrict": bool(args.level_restrict),
                   "fp64_m2l_rotation": rotation},
        "plain_fp64": {"value": round(nd * n_tgt / (ms_plain * 1e-3), 1),
                       "ms_per_apply": round(ms_plain, 3), "plan_seconds": round(plan64_s, 2)},
        "batched_fp64_graph": res["fp64"],
        **{f"batched_{p}_graph": r for p, r in res.items()},
        "vs_direct_qbx": direct,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
