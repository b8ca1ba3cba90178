// Dense translation matrices for the FMM translations M2M, M2L and L2L (Section 4.2; the
// paper defers the formulas to Greengard's thesis).  Built on the host in FP64.
//
// Internal expansion form (solid harmonics with the Condon-Shortley phase):
//   R_n^m(v) = r^n P_n^m(cos t) e^{i m phi} / (n+m)!,   I_n^m(v) = (n-m)! P_n^m(cos t) e^{i m phi} / r^(n+1)
//   multipole  mu_n^m = sum_s q R_n^m(s - c),   potential  (1/4pi) sum mu_n^m conj(I_n^m)(x - c)
//   local      l_n^m  = sum_s q conj(I_n^m)(s - c), potential (1/4pi) sum l_n^m R_n^m(x - c)
// Real sources give mu_n^-m = (-1)^m conj(mu_n^m) (same for l), so only m >= 0 is stored,
// real-packed per degree n as [Re c_n^0, Re c_n^1, Im c_n^1, ..., Re c_n^n, Im c_n^n]
// (offset n^2; (p+1)^2 reals in total).
//
// Scaling: a box of half-width a stores mu~_n = mu_n / a^n and l~_n = a^(n+1) l_n.  Then
//   M2M child(octant o) -> parent:  mu~'_n^m = 2^-n  sum mu~_j^k R_{n-j}^{m-k}(s_o)
//   L2L parent -> child(octant o):  l~'_j^k = sum_{n>=j} 2^-(n+1) l~_n^m R_{n-j}^{m-k}(s_o)
//   M2L source -> target, same level, x_t - x_s = 2 a o:
//                                   l~_j^k = (-1)^j sum mu~_n^m conj(I_{n+j}^{m+k})(2 o)
// with s_o = (+-1, +-1, +-1) (bit 0: x, bit 1: y, bit 2: z set = +1).  None depends on the
// level, so one matrix per octant / offset serves the whole tree.
//
// Matrices are stored column-major: T[col * np + row], y = T x.
#include <cmath>
#include <complex>
#include <vector>

#include "planner.hpp"

namespace gq {

using cd = std::complex<double>;

int ncoef(int p) { return (p + 1) * (p + 1); }

namespace {

inline int cid(int n, int m) { return n * n + n + m; }

// R_n^m for all n <= p, |m| <= n
std::vector<cd> regular_all(int p, double x, double y, double z) {
  std::vector<cd> R((p + 1) * (p + 1), 0.0);
  double r2 = x * x + y * y + z * z;
  cd d = 1.0;
  for (int m = 0; m <= p; ++m) {
    if (m > 0) d *= -cd(x, y) / (2.0 * m);
    R[cid(m, m)] = d;
    if (m + 1 <= p) R[cid(m + 1, m)] = z * d;
    for (int n = m + 2; n <= p; ++n)
      R[cid(n, m)] = ((2.0 * n - 1.0) * z * R[cid(n - 1, m)] - r2 * R[cid(n - 2, m)]) /
                     (double)(n * n - m * m);
  }
  for (int n = 0; n <= p; ++n)
    for (int m = 1; m <= n; ++m) R[cid(n, -m)] = ((m & 1) ? -1.0 : 1.0) * std::conj(R[cid(n, m)]);
  return R;
}

// I_n^m for all n <= p, |m| <= n
std::vector<cd> irregular_all(int p, double x, double y, double z) {
  std::vector<cd> Ir((p + 1) * (p + 1), 0.0);
  double r2 = x * x + y * y + z * z;
  cd d = 1.0 / std::sqrt(r2);
  for (int m = 0; m <= p; ++m) {
    if (m > 0) d *= -(2.0 * m - 1.0) * cd(x, y) / r2;
    Ir[cid(m, m)] = d;
    if (m + 1 <= p) Ir[cid(m + 1, m)] = (2.0 * m + 1.0) * z * d / r2;
    for (int n = m + 2; n <= p; ++n)
      Ir[cid(n, m)] = ((2.0 * n - 1.0) * z * Ir[cid(n - 1, m)] -
                       (double)((n - 1) * (n - 1) - m * m) * Ir[cid(n - 2, m)]) / r2;
  }
  for (int n = 0; n <= p; ++n)
    for (int m = 1; m <= n; ++m) Ir[cid(n, -m)] = ((m & 1) ? -1.0 : 1.0) * std::conj(Ir[cid(n, m)]);
  return Ir;
}

inline cd getc(const std::vector<cd>& a, int pmax, int n, int m) {
  if (n < 0 || n > pmax || m < -n || m > n) return 0.0;
  return a[cid(n, m)];
}

// Fill T (column-major) from X(nout, mout, nin, min) = coefficient of in_{nin}^{min} in
// out_{nout}^{mout}, over all signed min, using in^-m = (-1)^m conj(in^m).
template <class F>
void real_pack(int p, F X, double* T) {
  const int np = ncoef(p);
  for (int i = 0; i < np * np; ++i) T[i] = 0.0;
  for (int no = 0; no <= p; ++no)
    for (int mo = 0; mo <= no; ++mo) {
      const int rre = no * no + (mo ? 2 * mo - 1 : 0);
      const int rim = no * no + 2 * mo;  // valid only for mo > 0
      for (int ni = 0; ni <= p; ++ni)
        for (int mi = 0; mi <= ni; ++mi) {
          cd A = X(no, mo, ni, mi);
          cd B = mi ? (((mi & 1) ? -1.0 : 1.0) * X(no, mo, ni, -mi)) : cd(0.0);
          const int cre = ni * ni + (mi ? 2 * mi - 1 : 0);
          const int cim = ni * ni + 2 * mi;
          if (mi == 0) {
            T[cre * np + rre] += A.real();
            if (mo) T[cre * np + rim] += A.imag();
          } else {
            T[cre * np + rre] += A.real() + B.real();
            T[cim * np + rre] += -A.imag() + B.imag();
            if (mo) {
              T[cre * np + rim] += A.imag() + B.imag();
              T[cim * np + rim] += A.real() - B.real();
            }
          }
        }
    }
}

inline void octant_vec(int o, double s[3]) {
  s[0] = (o & 1) ? 1.0 : -1.0;
  s[1] = (o & 2) ? 1.0 : -1.0;
  s[2] = (o & 4) ? 1.0 : -1.0;
}

}  // namespace

void m2m_matrix(int p, int octant, double* T) {
  double s[3];
  octant_vec(octant, s);
  auto R = regular_all(p, s[0], s[1], s[2]);
  real_pack(p, [&](int n, int m, int j, int k) -> cd {
    if (j > n) return 0.0;
    return std::ldexp(1.0, -n) * getc(R, p, n - j, m - k);
  }, T);
}

void l2l_matrix(int p, int octant, double* T) {
  double s[3];
  octant_vec(octant, s);
  auto R = regular_all(p, s[0], s[1], s[2]);
  real_pack(p, [&](int j, int k, int n, int m) -> cd {
    if (n < j) return 0.0;
    return std::ldexp(1.0, -(n + 1)) * getc(R, p, n - j, m - k);
  }, T);
}

void m2l_matrix(int p, int ox, int oy, int oz, double* T) {
  auto Ir = irregular_all(2 * p, 2.0 * ox, 2.0 * oy, 2.0 * oz);
  real_pack(p, [&](int j, int k, int n, int m) -> cd {
    cd v = std::conj(getc(Ir, 2 * p, n + j, m + k));
    return (j & 1) ? -v : v;
  }, T);
}

}  // namespace gq
