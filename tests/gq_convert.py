"""Test helpers: map the oracle's paper-form coefficients to the library's internal
real-packed solid-harmonic form (and back).  Pure bookkeeping of normalization constants:

  paper local L_n^m  <->  internal l_n^m = 4 pi s_m kappa_n N_nm L_n^m
  paper multipole M  <->  internal mu_n^m = 4 pi s_m kappa_n M_n^m / N_nm
  kappa_n = sqrt((2n+1)/(4 pi)),  N_nm = sqrt((n-m)!(n+m)!),  s_m = (-1)^m (m > 0), 1 (m <= 0)

Scaled box forms: mu~_n = mu_n / a^n, l~_n = a^(n+1) l_n.  Real packing per degree n:
[Re c_n^0, Re c_n^1, Im c_n^1, ..., Re c_n^n, Im c_n^n].
"""

import math

import numpy as np


def _fac(n, m):
    return math.sqrt(math.factorial(n - m) * math.factorial(n + m))


def _kappa(n):
    return math.sqrt((2 * n + 1) / (4 * math.pi))


def _sm(m):
    return -1.0 if (m > 0 and m % 2) else 1.0


def paper_local_to_packed(L, p, a=None):
    out = np.zeros((p + 1) ** 2)
    for n in range(p + 1):
        sc = 1.0 if a is None else a ** (n + 1)
        for m in range(n + 1):
            v = 4 * math.pi * _sm(m) * _kappa(n) * _fac(n, m) * L[n * n + n + m] * sc
            if m == 0:
                out[n * n] = v.real
            else:
                out[n * n + 2 * m - 1] = v.real
                out[n * n + 2 * m] = v.imag
    return out


def paper_mpole_to_packed(M, p, a=None):
    out = np.zeros((p + 1) ** 2)
    for n in range(p + 1):
        sc = 1.0 if a is None else a ** (-n)
        for m in range(n + 1):
            v = 4 * math.pi * _sm(m) * _kappa(n) / _fac(n, m) * M[n * n + n + m] * sc
            if m == 0:
                out[n * n] = v.real
            else:
                out[n * n + 2 * m - 1] = v.real
                out[n * n + 2 * m] = v.imag
    return out


def packed_local_to_paper(x, p):
    """Inverse of paper_local_to_packed (unscaled), filling negative m by symmetry."""
    out = np.zeros((p + 1) ** 2, dtype=np.complex128)
    for n in range(p + 1):
        for m in range(n + 1):
            v = x[n * n] if m == 0 else x[n * n + 2 * m - 1] + 1j * x[n * n + 2 * m]
            Lnm = v / (4 * math.pi * _sm(m) * _kappa(n) * _fac(n, m))
            out[n * n + n + m] = Lnm
            if m:
                out[n * n + n - m] = np.conj(Lnm)
    return out
