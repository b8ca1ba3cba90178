"""FP64 CPU oracle for 3D Laplace QBX and the GIGAQBX FMM.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
baseline may import this package; the library never does.  It shares no code with the
HIP path (its numerics live in ``qbx_oracle.c``; its tree and interaction lists in
``gigaqbx.py`` are written straight from the paper's definitions).

Two tiers:
  * Tier A (``direct_qbx``): the plain definition of QBX discretized by the quadrature
    sum -- every source contributes to every center's order-p_qbx local expansion
    (Section 2.1, QBX coefficient integral and its quadrature), each target evaluated
    through its center.  Exact up to rounding; the accelerated method approximates it.
  * Tier B (``gigaqbx.OracleFMM``): the GIGAQBX algorithm (Algorithm 5, Stages 1-9) as
    plain steps in the paper's order, with its own octree and lists.

All coefficients are complex, in the paper's normalization, all m.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qbx_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

KERNELS = {"S": 0, "D": 1}


_SAN_LIB = os.path.join(_HERE, "liboracle_san.so")
if os.environ.get("ORACLE_SANITIZED"):
    # a process started with gcc's ASan runtime preloaded uses the sanitized build
    _LIB = _SAN_LIB


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C11 + OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        san = (["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g"]
               if _LIB == _SAN_LIB else [])
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", *san,
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
        P = ctypes.c_void_p
        sig = {
            "oq_ylm": (None, [i32, d, d, d, P, P]),
            "oq_p2l": (None, [i32, i32, i64, P, P, P, P, P]),
            "oq_p2m": (None, [i32, i32, i64, P, P, P, P, P]),
            "oq_eval_local": (d, [i32, P, P, P]),
            "oq_eval_mpole": (d, [i32, P, P, P]),
            "oq_m2m": (None, [i32, P, P, P, P]),
            "oq_m2l": (None, [i32, i32, P, P, P, P]),
            "oq_l2l": (None, [i32, i32, P, P, P, P]),
            "oq_regular_RI": (None, [i32, P, P]),
            "oq_irregular_RI": (None, [i32, P, P]),
            "oq_p2l_shared": (None, [i32, i32, i64, P, i64, P, P, P, P, P, i32]),
            "oq_p2m_csr": (None, [i32, i32, i64, P, P, P, P, P, P, P, i32]),
            "oq_m2l_csr": (None, [i32, i32, i64, P, P, P, P, P, P, i32]),
            "oq_l2l_csr": (None, [i32, i32, i64, P, P, P, P, P, P, i32]),
            "oq_eval_locals": (None, [i32, i64, P, P, P, P, P, i32]),
            "oq_direct_qbx": (i32, [i32, i32, i64, P, P, P, i64, P, i64, P, P, P, i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def ncoef(p):
    return (p + 1) * (p + 1)


def cidx(n, m):
    return n * n + n + m


# ---------------------------------------------------------------------------------------
# Single-expansion helpers (complex numpy vectors in the paper's normalization)
# ---------------------------------------------------------------------------------------


def ylm(p, v):
    v = _f64(v)
    re = np.empty(ncoef(p))
    im = np.empty(ncoef(p))
    lib().oq_ylm(p, float(v[0]), float(v[1]), float(v[2]), _p(re), _p(im))
    return re + 1j * im


def p2l(kernel, p, src, q, c, nrm=None):
    src, q, c = _f64(src).reshape(-1, 3), _f64(q).ravel(), _f64(c)
    nrm = None if nrm is None else _f64(nrm).reshape(-1, 3)
    out = np.zeros(ncoef(p), dtype=np.complex128)
    lib().oq_p2l(KERNELS[kernel], p, src.shape[0], _p(src), _p(nrm), _p(q), _p(c), _p(out))
    return out


def p2m(kernel, p, src, q, c, nrm=None):
    src, q, c = _f64(src).reshape(-1, 3), _f64(q).ravel(), _f64(c)
    nrm = None if nrm is None else _f64(nrm).reshape(-1, 3)
    out = np.zeros(ncoef(p), dtype=np.complex128)
    lib().oq_p2m(KERNELS[kernel], p, src.shape[0], _p(src), _p(nrm), _p(q), _p(c), _p(out))
    return out


def eval_local(p, L, c, t):
    L = np.ascontiguousarray(L, dtype=np.complex128)
    return lib().oq_eval_local(p, _p(L), _p(_f64(c)), _p(_f64(t)))


def eval_mpole(p, M, c, t):
    M = np.ascontiguousarray(M, dtype=np.complex128)
    return lib().oq_eval_mpole(p, _p(M), _p(_f64(c)), _p(_f64(t)))


def m2m(p, M, c_from, c_to):
    M = np.ascontiguousarray(M, dtype=np.complex128)
    out = np.zeros(ncoef(p), dtype=np.complex128)
    lib().oq_m2m(p, _p(M), _p(_f64(c_from)), _p(_f64(c_to)), _p(out))
    return out


def m2l(p, q, M, c_from, c_to):
    M = np.ascontiguousarray(M, dtype=np.complex128)
    out = np.zeros(ncoef(q), dtype=np.complex128)
    lib().oq_m2l(p, q, _p(M), _p(_f64(c_from)), _p(_f64(c_to)), _p(out))
    return out


def l2l(p, q, L, c_from, c_to):
    L = np.ascontiguousarray(L, dtype=np.complex128)
    out = np.zeros(ncoef(q), dtype=np.complex128)
    lib().oq_l2l(p, q, _p(L), _p(_f64(c_from)), _p(_f64(c_to)), _p(out))
    return out


def regular_RI(p, v):
    out = np.zeros(ncoef(p), dtype=np.complex128)
    lib().oq_regular_RI(p, _p(_f64(v)), _p(out))
    return out


def irregular_RI(p, v):
    out = np.zeros(ncoef(p), dtype=np.complex128)
    lib().oq_irregular_RI(p, _p(_f64(v)), _p(out))
    return out


# ---------------------------------------------------------------------------------------
# Tier A: direct QBX
# ---------------------------------------------------------------------------------------


def direct_qbx(kernel, p_qbx, src, strength, ctr, tgt, tgt_center, nrm=None, nthreads=0):
    """Potential at each target through its center, every source direct (Tier A).

    Returns (potential[n_tgt], threads_used).  ``strength`` = w * mu for one density.
    """
    src, strength, ctr, tgt = _f64(src), _f64(strength), _f64(ctr), _f64(tgt)
    tgt_center = _i64(tgt_center)
    nrm = None if nrm is None else _f64(nrm)
    if kernel == "D" and nrm is None:
        raise ValueError("double layer needs normals")
    out = np.empty(tgt.shape[0])
    used = lib().oq_direct_qbx(KERNELS[kernel], p_qbx, src.shape[0], _p(src), _p(nrm),
                               _p(strength), ctr.shape[0], _p(ctr), tgt.shape[0], _p(tgt),
                               _p(tgt_center), _p(out), int(nthreads))
    return out, used


def qbx_locals(kernel, p_qbx, src, strength, ctr, nrm=None, nthreads=0):
    """Tier A QBX coefficients (paper form, order p_qbx) at each center from every source."""
    src, strength, ctr = _f64(src), _f64(strength), _f64(ctr).reshape(-1, 3)
    nrm = _f64(src * 0.0 if nrm is None else nrm)
    idx = _i64(np.arange(src.shape[0]))
    out = np.zeros((ctr.shape[0], ncoef(p_qbx)), dtype=np.complex128)
    lib().oq_p2l_shared(KERNELS[kernel], p_qbx, ctr.shape[0], _p(ctr), len(idx), _p(idx),
                        _p(src), _p(nrm), _p(strength), _p(out), int(nthreads))
    return out


def local_normal_derivative(p, L, c, t, n):
    """d/dn of the local expansion L (order p, about c) at the point t, along the unit vector
    n.  The expansion is re-centred at t (L2L is exact for it); its degree-1 part about t is
    the linear term, so the derivative is that part evaluated at t + n."""
    L1 = l2l(p, 1, L, c, t)
    t, n = _f64(t), _f64(n)
    return eval_local(1, L1, t, t + n) - eval_local(0, L1[:1], t, t)


def direct_qbx_sprime(p_qbx, src, strength, ctr, tgt, tgt_center, tgt_normal, nthreads=0):
    """Tier A for the adjoint double layer S' (the normal derivative of the single layer at
    the target): the single-layer QBX coefficients of each target's center, differentiated
    along the target's unit normal (local_normal_derivative)."""
    tgt_center = _i64(tgt_center)
    Ls = qbx_locals("S", p_qbx, src, strength, ctr, nthreads=nthreads)
    ctr, tgt, tn = _f64(ctr).reshape(-1, 3), _f64(tgt).reshape(-1, 3), _f64(tgt_normal)
    return np.array([local_normal_derivative(p_qbx, Ls[tgt_center[i]], ctr[tgt_center[i]],
                                             tgt[i], tn[i]) for i in range(tgt.shape[0])])


def source_density(w):
    """Density at the sources, shape (n_densities, N_S): the workload's density itself, or,
    with an oversampled quadrature (Section 3: the density lives on the nodes of each
    element and the potential uses a finer quadrature on the same element), each
    element's node values mapped to its quadrature nodes by the interpolation matrix."""
    if getattr(w, "interp", None) is None:
        return w.density
    nd = w.density.shape[0]
    nodes = w.density.reshape(nd, w.n_elem, w.interp.shape[1])
    return np.einsum("dek,jk->dej", nodes, w.interp).reshape(nd, -1)


def strengths(w):
    """Quadrature strengths q_j = w_j mu_j at the sources (the discretized layer potential
    of Section 2.3), shape (n_densities, N_S)."""
    return source_density(w) * w.src_w[None, :]


def direct_qbx_sampled(w, center_ids, density_index=0, nthreads=0):
    """Tier A on a subset of centers of a workload: returns (target ids, potentials)."""
    center_ids = np.asarray(center_ids, dtype=np.int64)
    tmask = np.isin(w.tgt_center, center_ids)
    tids = np.nonzero(tmask)[0]
    remap = {int(c): i for i, c in enumerate(center_ids)}
    tc = np.array([remap[int(c)] for c in w.tgt_center[tids]], dtype=np.int64)
    pot, used = direct_qbx(w.kernel, w.p_qbx, w.src_xyz, strengths(w)[density_index],
                           w.ctr_xyz[center_ids], w.tgt_xyz[tids], tc,
                           nrm=w.src_normal, nthreads=nthreads)
    return tids, pot, used
