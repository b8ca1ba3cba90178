"""ctypes binding of libgigaqbx.so (include/gigaqbx.h).  Argument marshalling only.

Every function keeps the C name.  Host arrays are numpy arrays; device buffers are torch
CUDA (HIP) tensors or raw integer device pointers; streams are torch streams, raw
integers or None (the current torch stream when a tensor is given, else the default).
Failures raise GQError carrying the status and gq_last_error().
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GQ_LIBRARY selects another build of the same library (the host-sanitized one)
LIB_PATH = os.environ.get("GQ_LIBRARY") or os.path.join(_HERE, "libgigaqbx.so")

GQ_OK, GQ_EINVAL, GQ_ENOMEM, GQ_EDEVICE, GQ_EUNSUPPORTED = 0, 1, 2, 3, 4
GQ_KERNEL_S, GQ_KERNEL_D, GQ_KERNEL_SP = 0, 1, 2
GQ_FP64 = 0
GQ_FP32_SPLIT = 1
GQ_FP32 = 2
GQ_FP32_LEAD = 3
PRECISIONS = {"fp64": GQ_FP64, "fp32_split": GQ_FP32_SPLIT, "fp32": GQ_FP32,
              "fp32_lead": GQ_FP32_LEAD}
GQ_FLAG_HOST_ONLY = 1 << 0
GQ_FLAG_TIMING = 1 << 1
GQ_FLAG_GRAPH = 1 << 2
GQ_FLAG_AUTOTUNE = 1 << 3
GQ_FLAG_DETERMINISTIC = 1 << 4
GQ_FLAG_AUTOTUNE_TREE = 1 << 5
GQ_LIST_U = 1 << 8
GQ_LIST_V = 1 << 9
GQ_LIST_WCLOSE = 1 << 10
GQ_LIST_WFAR = 1 << 11
GQ_LIST_XCLOSE = 1 << 12
GQ_LIST_XFAR = 1 << 13
LIST_BITS = {"U": GQ_LIST_U, "V": GQ_LIST_V, "Wclose": GQ_LIST_WCLOSE, "Wfar": GQ_LIST_WFAR,
             "Xclose": GQ_LIST_XCLOSE, "Xfar": GQ_LIST_XFAR}
LIST_INDEX = {"U": 0, "V": 1, "Wclose": 2, "Wfar": 3, "Xclose": 4, "Xfar": 5}
STAGES = ("strength", "p2m", "m2m", "m2l", "p2l", "l2l", "p2qbxl", "m2qbxl", "l2qbxl",
          "qbxl2p", "fill", "total")

EXPORTED = ("gq_plan_create", "gq_apply", "gq_stats", "gq_plan_destroy", "gq_last_error",
            "gq_tree_export", "gq_list_export", "gq_qbx_locals", "gq_translation_matrix",
            "gq_batch_create", "gq_set_target_normals", "gq_set_source_interp",
            "gq_associate_targets", "gq_points_near", "gq_set_overlap",
            "gq_points_near_noalloc")
GQ_TARGET_FAR = -1
GQ_TARGET_UNMATCHED = -2


class gq_params(ctypes.Structure):
    _fields_ = [("p_qbx", ctypes.c_int), ("p_fmm", ctypes.c_int), ("nmax", ctypes.c_int),
                ("tcf", ctypes.c_double), ("kernel", ctypes.c_int), ("precision", ctypes.c_int),
                ("n_densities", ctypes.c_int), ("flags", ctypes.c_uint),
                ("wfar_direct_max", ctypes.c_int), ("tcr_norm", ctypes.c_int),
                ("level_restrict", ctypes.c_int), ("m2l_rotation", ctypes.c_int),
                ("max_device_bytes", ctypes.c_int64)]


class gq_stats_t(ctypes.Structure):
    _fields_ = [("n_sources", ctypes.c_int64), ("n_centers", ctypes.c_int64),
                ("n_targets", ctypes.c_int64), ("n_boxes", ctypes.c_int64),
                ("n_levels", ctypes.c_int64), ("n_target_boxes", ctypes.c_int64),
                ("n_suspended_centers", ctypes.c_int64),
                ("list_entries", ctypes.c_int64 * 6), ("pairs", ctypes.c_int64 * 6),
                ("m2l_classes", ctypes.c_int64), ("plan_seconds", ctypes.c_double),
                ("stage_ms", ctypes.c_double * 12), ("timed_applies", ctypes.c_int64),
                ("m2l_tile_cols", ctypes.c_int32), ("m2l_xcd_order", ctypes.c_int32),
                ("n_point_targets", ctypes.c_int64), ("modeled_flops", ctypes.c_double * 7),
                ("device_bytes", ctypes.c_int64), ("nmax", ctypes.c_int32),
                ("wfar_direct_max", ctypes.c_int32)]


class GQError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gigaqbx status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load the HIP library; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1805_06106_amd.build` (hipcc, gfx950)")
        # torch carries its own HIP runtime; loading it first makes this library bind to
        # that same runtime instead of initializing a second one in the process (torch then
        # finds no device if the library's runtime claimed it first)
        import torch  # noqa: F401

        L = ctypes.CDLL(LIB_PATH)
        P, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.gq_plan_create.restype = i32
        L.gq_plan_create.argtypes = [ctypes.POINTER(gq_params), i64, P, P, P, i64, P, P, i64, P, P,
                                     P, ctypes.POINTER(ctypes.c_void_p)]
        L.gq_apply.restype = i32
        L.gq_apply.argtypes = [P, P, P, P]
        L.gq_stats.restype = i32
        L.gq_stats.argtypes = [P, ctypes.POINTER(gq_stats_t)]
        L.gq_plan_destroy.restype = None
        L.gq_plan_destroy.argtypes = [P]
        L.gq_last_error.restype = ctypes.c_char_p
        L.gq_last_error.argtypes = []
        L.gq_tree_export.restype = i32
        L.gq_tree_export.argtypes = [P, P, P, P, P, P]
        L.gq_list_export.restype = i32
        L.gq_list_export.argtypes = [P, i32, P, P, ctypes.POINTER(ctypes.c_int64)]
        L.gq_qbx_locals.restype = i32
        L.gq_qbx_locals.argtypes = [P, P]
        L.gq_set_target_normals.restype = i32
        L.gq_set_target_normals.argtypes = [P, P]
        L.gq_set_overlap.restype = i32
        L.gq_set_overlap.argtypes = [P, i32]
        L.gq_set_source_interp.restype = i32
        L.gq_points_near.restype = i32
        L.gq_points_near.argtypes = [ctypes.c_int64, P, P, i32, ctypes.c_int64, P, P, P]
        L.gq_points_near_noalloc.restype = i32
        L.gq_points_near_noalloc.argtypes = [ctypes.c_int64, P, P, i32, ctypes.c_int64, P, P, P]
        L.gq_associate_targets.restype = i32
        L.gq_associate_targets.argtypes = [ctypes.c_int64, P, P, ctypes.c_int64, P, P, P,
                                           ctypes.c_int64, P, P, ctypes.c_double, P, P]
        L.gq_set_source_interp.argtypes = [P, ctypes.c_int64, i32, i32, P]
        L.gq_batch_create.restype = i32
        L.gq_batch_create.argtypes = [i32, P, ctypes.c_uint, P, ctypes.POINTER(ctypes.c_void_p)]
        L.gq_translation_matrix.restype = i32
        L.gq_translation_matrix.argtypes = [i32, i32, i32, i32, i32, P]
        _lib = L
    return _lib


def _check(st):
    if st != GQ_OK:
        raise GQError(st, gq_last_error())


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _dptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream, tensor=None):
    if stream is None:
        if tensor is not None and not isinstance(tensor, int):
            import torch

            return ctypes.c_void_p(torch.cuda.current_stream(tensor.device).cuda_stream)
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def gq_last_error():
    return lib().gq_last_error().decode()


def make_params(p_qbx, p_fmm, nmax=512, tcf=0.9, kernel="S", n_densities=1, flags=0,
                lists=None, wfar_direct_max=0, precision="fp64", tcr_norm="l2",
                level_restrict=False, m2l_rotation=False, max_device_bytes=0):
    k = {"S": GQ_KERNEL_S, "D": GQ_KERNEL_D, "SP": GQ_KERNEL_SP}.get(kernel, kernel)
    prec = PRECISIONS.get(precision, precision)
    if lists is not None:
        for nm in lists:
            flags |= LIST_BITS[nm]
    return gq_params(int(p_qbx), int(p_fmm), int(nmax), float(tcf), int(k), int(prec),
                     int(n_densities), int(flags), int(wfar_direct_max),
                     {"l2": 0, "linf": 1}.get(tcr_norm, tcr_norm), int(level_restrict),
                     int(m2l_rotation), int(max_device_bytes))


def gq_plan_create(params, src_xyz, src_w, src_normal, ctr_xyz, ctr_radius, tgt_xyz,
                   tgt_center, stream=None):
    """Returns an opaque plan handle (int).  Arrays: numpy, shapes (N,3)/(N,)."""
    f64 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    src_xyz, src_w, src_normal = f64(src_xyz), f64(src_w), f64(src_normal)
    ctr_xyz, ctr_radius, tgt_xyz = f64(ctr_xyz), f64(ctr_radius), f64(tgt_xyz)
    tgt_center = np.ascontiguousarray(tgt_center, dtype=np.int64)
    out = ctypes.c_void_p()
    st = lib().gq_plan_create(ctypes.byref(params), src_xyz.shape[0], _ptr(src_xyz), _ptr(src_w),
                              _ptr(src_normal), ctr_xyz.shape[0], _ptr(ctr_xyz),
                              _ptr(ctr_radius), tgt_xyz.shape[0], _ptr(tgt_xyz),
                              _ptr(tgt_center), _stream(stream), ctypes.byref(out))
    _check(st)
    return out.value


def gq_set_overlap(plan, on):
    """1: far-field chain on the plan's own stream beside the near field; 0: all in order."""
    _check(lib().gq_set_overlap(ctypes.c_void_p(plan), int(on)))


def gq_set_target_normals(plan, normals):
    """normals: host (n_tgt, 3) float64 unit vectors in input target order."""
    normals = np.ascontiguousarray(normals, dtype=np.float64)
    _check(lib().gq_set_target_normals(ctypes.c_void_p(plan), _ptr(normals)))


def gq_set_source_interp(plan, n_elem, interp):
    """interp: host (n_quad, n_node) float64 matrix from an element's node values to its
    quadrature nodes; the plan's sources are the n_elem * n_quad quadrature nodes."""
    interp = np.ascontiguousarray(interp, dtype=np.float64)
    n_quad, n_node = interp.shape
    _check(lib().gq_set_source_interp(ctypes.c_void_p(plan), int(n_elem), int(n_node),
                                      int(n_quad), _ptr(interp)))


def gq_points_near(q_xyz, radius, p_xyz, strict=False, stream=None, noalloc=False):
    """Host bool array: is some point of p_xyz within radius[i] of q_xyz[i] (< if strict)?
    noalloc=True calls gq_points_near_noalloc (device buffers in the library's fixed
    scratch, no device allocation)."""
    q_xyz = np.ascontiguousarray(np.asarray(q_xyz, dtype=np.float64).reshape(-1, 3))
    p_xyz = np.ascontiguousarray(np.asarray(p_xyz, dtype=np.float64).reshape(-1, 3))
    radius = np.ascontiguousarray(np.broadcast_to(np.asarray(radius, dtype=np.float64),
                                                  (q_xyz.shape[0],)))
    hit = np.empty(q_xyz.shape[0], dtype=np.uint8)
    fn = lib().gq_points_near_noalloc if noalloc else lib().gq_points_near
    _check(fn(q_xyz.shape[0], _ptr(q_xyz), _ptr(radius), int(bool(strict)),
              p_xyz.shape[0], _ptr(p_xyz), _ptr(hit), _stream(stream)))
    return hit.astype(bool)


def gq_associate_targets(src_xyz, src_danger, ctr_xyz, ctr_radius, tgt_xyz, tol=0.0,
                         ctr_side=None, tgt_side=None, stream=None):
    """Algorithm 3 on the device; host arrays in, host int64 array out (a center index per
    target, GQ_TARGET_FAR or GQ_TARGET_UNMATCHED)."""
    f64 = lambda a, shape: np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))  # noqa: E731
    src_xyz = f64(src_xyz, (-1, 3))
    ctr_xyz = f64(ctr_xyz, (-1, 3))
    tgt_xyz = f64(tgt_xyz, (-1, 3))
    src_danger = f64(src_danger, (-1,))
    ctr_radius = f64(ctr_radius, (-1,))
    i8 = lambda a: None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.int8))  # noqa: E731
    ctr_side, tgt_side = i8(ctr_side), i8(tgt_side)
    if src_danger.shape[0] != src_xyz.shape[0] or ctr_radius.shape[0] != ctr_xyz.shape[0]:
        raise ValueError("radius arrays must match their point arrays")
    for side, n in ((ctr_side, ctr_xyz.shape[0]), (tgt_side, tgt_xyz.shape[0])):
        if side is not None and side.shape != (n,):
            raise ValueError("side arrays must have one entry per point")
    out = np.empty(tgt_xyz.shape[0], dtype=np.int64)
    _check(lib().gq_associate_targets(
        src_xyz.shape[0], _ptr(src_xyz), _ptr(src_danger), ctr_xyz.shape[0], _ptr(ctr_xyz),
        _ptr(ctr_radius), _ptr(ctr_side), tgt_xyz.shape[0], _ptr(tgt_xyz), _ptr(tgt_side),
        float(tol), _ptr(out), _stream(stream)))
    return out


def gq_batch_create(plans, flags=0, stream=None):
    """Merge plan handles into one batch plan handle."""
    arr = (ctypes.c_void_p * len(plans))(*plans)
    out = ctypes.c_void_p()
    _check(lib().gq_batch_create(len(plans), ctypes.cast(arr, ctypes.c_void_p), int(flags),
                                 _stream(stream), ctypes.byref(out)))
    return out.value


def gq_apply(plan, density, potential, stream=None):
    """density: device [n_densities, n_src] float64; potential: device [n_densities, n_tgt]."""
    _check(lib().gq_apply(ctypes.c_void_p(plan), _dptr(density), _dptr(potential),
                          _stream(stream, density)))


def gq_stats(plan):
    s = gq_stats_t()
    _check(lib().gq_stats(ctypes.c_void_p(plan), ctypes.byref(s)))
    return {
        "n_sources": s.n_sources, "n_centers": s.n_centers, "n_targets": s.n_targets,
        "n_boxes": s.n_boxes, "n_levels": s.n_levels, "n_target_boxes": s.n_target_boxes,
        "n_suspended_centers": s.n_suspended_centers,
        "list_entries": dict(zip(LIST_INDEX, list(s.list_entries))),
        "pairs": dict(zip(LIST_INDEX, list(s.pairs))),
        "m2l_classes": s.m2l_classes, "plan_seconds": s.plan_seconds,
        "stage_ms": dict(zip(STAGES, list(s.stage_ms))),
        "timed_applies": s.timed_applies,
        "m2l_tile_cols": s.m2l_tile_cols, "m2l_xcd_order": bool(s.m2l_xcd_order),
        "n_point_targets": s.n_point_targets,
        "modeled_flops": dict(zip(list(LIST_INDEX) + ["total_lists"], list(s.modeled_flops))),
        "device_bytes": s.device_bytes,
        "nmax": s.nmax, "wfar_direct_max": s.wfar_direct_max,
    }


def gq_plan_destroy(plan):
    if plan:
        lib().gq_plan_destroy(ctypes.c_void_p(plan))


def gq_tree_export(plan, n_ctr):
    s = gq_stats(plan)
    nb = s["n_boxes"]
    c = np.empty((nb, 3))
    h = np.empty(nb)
    lev = np.empty(nb, dtype=np.int32)
    par = np.empty(nb, dtype=np.int32)
    own = np.empty(n_ctr, dtype=np.int64)
    _check(lib().gq_tree_export(ctypes.c_void_p(plan), _ptr(c), _ptr(h), _ptr(lev), _ptr(par),
                                _ptr(own)))
    return c, h, lev, par, own


def gq_list_export(plan, name):
    nb = gq_stats(plan)["n_boxes"]
    n = ctypes.c_int64()
    idx = LIST_INDEX[name]
    _check(lib().gq_list_export(ctypes.c_void_p(plan), idx, None, None, ctypes.byref(n)))
    ptr = np.empty(nb + 1, dtype=np.int64)
    items = np.empty(max(n.value, 1), dtype=np.int32)
    _check(lib().gq_list_export(ctypes.c_void_p(plan), idx, _ptr(ptr), _ptr(items),
                                ctypes.byref(n)))
    return ptr, items[:n.value]


def gq_qbx_locals(plan, n_ctr, p_qbx):
    out = np.empty((n_ctr, (p_qbx + 1) ** 2))
    _check(lib().gq_qbx_locals(ctypes.c_void_p(plan), _ptr(out)))
    return out


def gq_translation_matrix(kind, p, a, b=0, c=0):
    n = (p + 1) ** 2
    out = np.empty(n * n)
    _check(lib().gq_translation_matrix(int(kind), int(p), int(a), int(b), int(c), _ptr(out)))
    return out.reshape(n, n).T.copy()  # column-major storage -> row-major matrix
