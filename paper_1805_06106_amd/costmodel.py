"""Floating-point operation counts per interaction for each stage of the evaluation.

Counts follow the arithmetic each kernel performs for one unit of work (a fused
multiply-add counts 2, a division or square root counts 1).  They are used to turn
measured kernel times into achieved FLOP/s; they are not used by the compute path.

Units:
  p2qbxl  one (source, center) pair of Lists 1, 3-close, 4-close (Stages 3, 5a, 6a)
  m2qbxl  one (List 3-far box, center) pair (Stage 5b)
  l2qbxl  one center (Stage 8)
  translate  one dense (p+1)^2 x (p+1)^2 matrix-vector product (M2M, M2L, L2L)
  qbxl2p  one target (Stage 9)
"""

from __future__ import annotations


def p2qbxl_pair(q: int, kernel: str) -> int:
    f = 3 + 5 + 1 + 1 + 1 + (1 if kernel == "S" else 0)  # d, |d|^2, 1/|d|^2, z/|d|^2, sqrt(, *q)
    top = q if kernel == "S" else q + 1
    for m in range(0, top + 1):
        if m > 0:
            f += 10  # diagonal: factor (4) and complex product (6)
        for n in range(m, top + 1):
            if n > m:
                f += 5 if m == 0 else 8  # recurrence: c1, c2 and the 2-term update
            if kernel == "S":
                f += 1 if m == 0 else 2  # accumulate
            else:
                if n == 0:
                    continue
                nn = n - 1
                if m <= nn:
                    f += 2 if m == 0 else 4  # -n_z J -> l^m
                if m == 1:
                    f += 5  # 2 Re(qa J^1) -> l^0
                elif m >= 2 and m - 1 <= nn:
                    f += 8  # qa J -> l^(m-1)
                if m + 1 <= nn:
                    f += 4 if m == 0 else 8  # -conj(qa) J -> l^(m+1)
    return f


def _stream_macs(p: int, q: int, irregular: bool) -> int:
    """Complex MAC flops of the order-q outputs fed by a streamed order-(p+q) (M2QBXL) or
    order-p (L2QBXL) solid-harmonic table."""
    f = 0
    nt = p + q if irregular else p
    for mo in range(0, nt + 1):
        for N in range(mo, nt + 1):
            for j in range(q + 1):
                n = N - j if irregular else N + j
                if n < 0 or n > p:
                    continue
                for k in range(j + 1):
                    m1 = mo - k if irregular else mo + k
                    if -n <= m1 <= n:
                        f += 8 if k else 4
                    if mo > 0:
                        m2 = -mo - k if irregular else k - mo
                        if -n <= m2 <= n:
                            f += 8 if k else 4
    return f


def m2qbxl_pair(p: int, q: int) -> int:
    nt = p + q
    gen = 14 + 10 * nt + 8 * (nt * (nt + 1) // 2)
    return gen + _stream_macs(p, q, True) + 2 * (q + 1) ** 2


def l2qbxl_center(p: int, q: int) -> int:
    gen = 14 + 10 * p + 9 * (p * (p + 1) // 2)
    return gen + _stream_macs(p, q, False) + 2 * (q + 1) ** 2


def translate(p: int) -> int:
    n = (p + 1) ** 2
    return 2 * n * n


def rotation_m2l_pair(p: int) -> float:
    """Executed flops per pair of the rotation-factored M2L (T = B Z A): per 16 pairs, the
    nonzero 16 x 16 tiles of A and B (block diagonal by degree), 4 matrix-core k-steps
    each, and the order blocks of Z (p + 1 - m rows each, k-steps of 4 past its padding),
    every k-step 16 x 16 x 4 multiply-adds."""
    npc = (p + 1) ** 2
    ntr = (npc + 15) // 16

    def touches(r, n):
        return n * n <= 16 * r + 15 and (n + 1) ** 2 - 1 >= 16 * r

    ntile = sum(1 for r in range(ntr) for c in range(ntr)
                if any(touches(r, n) and touches(c, n) for n in range(p + 1)))
    zsteps = sum(-(-(p + 1 - (b + 1) // 2) // 4) for b in range(2 * p + 1))
    return (2 * 4 * ntile + zsteps) * 2 * 16 * 16 * 4 / 16


def qbxl2p_target(q: int) -> int:
    return 8 + 10 * q + 9 * (q * (q + 1) // 2) + 4 * (q + 1) ** 2 + 1


# FP64 flops per unit that the kernels execute, counted on the GPU with rocprofv3
# (64 lanes x (2 SQ_INSTS_VALU_FMA_F64 + SQ_INSTS_VALU_MUL_F64 + SQ_INSTS_VALU_ADD_F64) over
# one launch, divided by the launch's units) on the urchin (double layer, p_qbx = 5,
# p_fmm = 15, nmax 192, level-restricted tree, Remark 4 at 64; the near field counted 526.4
# per pair at nmax 512, where its items are larger).  Where a configuration has no count,
# the written models above are used.
COUNTED_P2QBXL_PAIR = {(5, "D"): 532.9}      # near field, per (source, center) pair
COUNTED_P2M_SOURCE = {(15, "D"): 9327.0}     # P2M, per source
COUNTED_P2L_PAIR = {(15, "D"): 9565.0}       # P2L, per (source, List 4 far box) pair


def p2qbxl_pair_counted(q: int, kernel: str) -> float:
    return COUNTED_P2QBXL_PAIR.get((q, kernel), float(p2qbxl_pair(q, kernel)))


def apply_flops(stats: dict, p: int, q: int, kernel: str) -> dict:
    """Work of one apply, per stage, from the plan's interaction counts: the near field by
    its counted flops per pair where counted; the M2QBXL, L2QBXL and QBXL2P models; the
    dense translations at 2 (p+1)^4 per product (M2M and L2L: one product per box below
    the root); P2M per source and P2L per (source, box) pair by their counted flops where
    counted (else omitted)."""
    pr = stats["pairs"]
    near = pr["U"] + pr["Wclose"] + pr["Xclose"]
    out = {
        "p2qbxl": near * p2qbxl_pair_counted(q, kernel),
        "m2qbxl": pr["Wfar"] * m2qbxl_pair(p, q),
        "m2l": pr["V"] * translate(p),
        "l2qbxl": stats["n_centers"] * l2qbxl_center(p, q),
        "qbxl2p": stats["n_targets"] * qbxl2p_target(q),
        "m2m": (stats["n_boxes"] - 1) * translate(p),
        "l2l": (stats["n_boxes"] - 1) * translate(p),
    }
    if (p, kernel) in COUNTED_P2M_SOURCE:
        out["p2m"] = stats["n_sources"] * COUNTED_P2M_SOURCE[(p, kernel)]
    if (p, kernel) in COUNTED_P2L_PAIR:
        out["p2l"] = pr["Xfar"] * COUNTED_P2L_PAIR[(p, kernel)]
    return out


def paper_list_model(stats: dict, p: int, q: int) -> dict:
    """The per-list cost model of Section 6 (Table 7): for one (source box, target box)
    entry, q^2 n_s n_t for Lists 1, 3-close and 4-close, p^3 for List 2, p^3 n_t for
    List 3-far and p^2 n_s for List 4-far, summed over the plan's lists."""
    pr = stats["pairs"]
    out = {
        "U": q * q * pr["U"],
        "V": p ** 3 * pr["V"],
        "Wclose": q * q * pr["Wclose"],
        "Wfar": p ** 3 * pr["Wfar"],
        "Xclose": q * q * pr["Xclose"],
        "Xfar": p * p * pr["Xfar"],
    }
    out["total_lists"] = sum(out.values())
    return out
