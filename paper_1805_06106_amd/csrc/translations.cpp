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
#include <algorithm>
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

namespace {

// M2L for a scaled offset t = x_target - x_source in units of the box half-width.
void m2l_matrix_vec(int p, double tx, double ty, double tz, double* T) {
  auto Ir = irregular_all(2 * p, tx, ty, tz);
  real_pack(p, [&](int j, int k, int n, int m) -> cd {
    cd v = std::conj(getc(Ir, 2 * p, n + j, m + k));
    return (j & 1) ? -v : v;
  }, T);
}

// Packed values of degree n, [Re c^0, Re c^1, Im c^1, ..., Re c^n, Im c^n], of a full
// signed-order table, each multiplied by w(m).
template <class W>
void pack_degree(const std::vector<cd>& a, int pmax, int n, W w, double* out) {
  out[0] = a[cid(n, 0)].real() * w(0);
  for (int m = 1; m <= n; ++m) {
    out[2 * m - 1] = a[cid(n, m)].real() * w(m);
    out[2 * m] = a[cid(n, m)].imag() * w(m);
  }
  (void)pmax;
}

// Solve G X = H for X (d x d), G symmetric positive definite (Gauss-Jordan with pivoting).
void solve_spd(int d, std::vector<double> G, std::vector<double>& H) {
  for (int c = 0; c < d; ++c) {
    int piv = c;
    for (int r = c + 1; r < d; ++r)
      if (std::fabs(G[r * d + c]) > std::fabs(G[piv * d + c])) piv = r;
    for (int k = 0; k < d; ++k) {
      std::swap(G[c * d + k], G[piv * d + k]);
      std::swap(H[c * d + k], H[piv * d + k]);
    }
    const double inv = 1.0 / G[c * d + c];
    for (int k = 0; k < d; ++k) {
      G[c * d + k] *= inv;
      H[c * d + k] *= inv;
    }
    for (int r = 0; r < d; ++r) {
      if (r == c) continue;
      const double f = G[r * d + c];
      if (f == 0.0) continue;
      for (int k = 0; k < d; ++k) {
        G[r * d + k] -= f * G[c * d + k];
        H[r * d + k] -= f * H[c * d + k];
      }
    }
  }
}

// The real (2n+1) x (2n+1) blocks D_n with pack(f_n(Q v)) = D_n pack(f_n(v)) for every v,
// where f = R (regular, irregular = false) or conj(I) (irregular = true); written into the
// column-major np x np matrix D (block diagonal by degree).  Each block is fitted by least
// squares on sample directions, in a basis where the orders have comparable size.
void rotation_blocks(int p, const double Q[9], bool irregular, double* D) {
  const int np = ncoef(p);
  for (int i = 0; i < np * np; ++i) D[i] = 0.0;
  std::vector<double> lf(2 * p + 2, 0.0);  // log factorials
  for (int i = 1; i < (int)lf.size(); ++i) lf[i] = lf[i - 1] + std::log((double)i);
  const int K = 8 * (2 * p + 1);
  std::vector<std::vector<cd>> F(K), FQ(K);
  for (int s = 0; s < K; ++s) {
    // a spread of unit directions (golden-angle spiral, slightly off the poles)
    const double z = 1.0 - (2.0 * s + 1.0) / K;
    const double rr = std::sqrt(1.0 - z * z), ph = 2.399963229728653 * s + 0.3;
    const double v[3] = {rr * std::cos(ph), rr * std::sin(ph), z};
    const double w[3] = {Q[0] * v[0] + Q[1] * v[1] + Q[2] * v[2],
                         Q[3] * v[0] + Q[4] * v[1] + Q[5] * v[2],
                         Q[6] * v[0] + Q[7] * v[1] + Q[8] * v[2]};
    if (irregular) {
      F[s] = irregular_all(p, v[0], v[1], v[2]);
      FQ[s] = irregular_all(p, w[0], w[1], w[2]);
      for (auto& x : F[s]) x = std::conj(x);
      for (auto& x : FQ[s]) x = std::conj(x);
    } else {
      F[s] = regular_all(p, v[0], v[1], v[2]);
      FQ[s] = regular_all(p, w[0], w[1], w[2]);
    }
  }
  for (int n = 0; n <= p; ++n) {
    const int d = 2 * n + 1;
    // |R_n^m| ~ 1 / sqrt((n+m)! (n-m)!), |I_n^m| ~ sqrt((n+m)! (n-m)!) on the unit sphere
    auto w = [&](int m) {
      const double e = 0.5 * (lf[n + m] + lf[n - m]);
      return std::exp(irregular ? -e : e);
    };
    std::vector<double> G(d * d, 0.0), H(d * d, 0.0), a(d), b(d);
    for (int s = 0; s < K; ++s) {
      pack_degree(F[s], p, n, w, a.data());
      pack_degree(FQ[s], p, n, w, b.data());
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
          G[i * d + j] += a[i] * a[j];  // sum a a^T
          H[i * d + j] += a[i] * b[j];  // sum a b^T
        }
    }
    // H = (sum a a^T)^-1 sum a b^T = Dhat^T, with one step of iterative refinement
    std::vector<double> H0 = H;
    solve_spd(d, G, H);
    std::vector<double> Rr(d * d);
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        double acc = H0[i * d + j];
        for (int k = 0; k < d; ++k) acc -= G[i * d + k] * H[k * d + j];
        Rr[i * d + j] = acc;
      }
    solve_spd(d, G, Rr);
    for (int i = 0; i < d * d; ++i) H[i] += Rr[i];
    // back to the unscaled packing: D = W^-1 Dhat W, Dhat[r][c] = H[c][r]
    auto wm = [&](int i) { return w((i + 1) / 2); };
    for (int r = 0; r < d; ++r)
      for (int c = 0; c < d; ++c)
        D[(size_t)(n * n + c) * np + n * n + r] = H[c * d + r] * wm(c) / wm(r);
  }
}

}  // namespace

void m2l_matrix(int p, int ox, int oy, int oz, double* T) {
  m2l_matrix_vec(p, 2.0 * ox, 2.0 * oy, 2.0 * oz, T);
}

// N_n^m = sqrt((n+m)! (n-m)!) at each packed index.  With it the normalized forms
// R_n^m N_n^m and I_n^m / N_n^m are bounded by r^n and r^-(n+1) (the Schmidt
// semi-normalized solid harmonics), so multipoles mu N and locals l / N of a box in its own
// scaled units are O(1) for every order, and so are the entries of the translations
// between them: at p = 20 the factorial form spans about 60 decades, beyond FP32's range.
void expansion_norms(int p, double* N) {
  std::vector<double> f(2 * p + 2, 1.0);
  for (int i = 1; i < (int)f.size(); ++i) f[i] = f[i - 1] * i;
  for (int n = 0; n <= p; ++n)
    for (int m = 0; m <= n; ++m) {
      const double v = std::sqrt(f[n + m] * f[n - m]);
      N[n * n + (m ? 2 * m - 1 : 0)] = v;
      if (m) N[n * n + 2 * m] = v;
    }
}

void m2l_rotation_factors(int p, int ox, int oy, int oz, double* A, double* Z, double* B) {
  // a rotation Q taking the offset direction u to +z (Rodrigues about u x z)
  const double len = std::sqrt((double)(ox * ox + oy * oy + oz * oz));
  const double u[3] = {ox / len, oy / len, oz / len};
  double Q[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  const double c = u[2];
  const double kx = u[1], ky = -u[0];  // u x z
  const double sn = std::sqrt(kx * kx + ky * ky);
  if (sn < 1e-14) {
    if (c < 0) {  // u = -z: half turn about x
      Q[4] = -1.0;
      Q[8] = -1.0;
    }
  } else {
    const double ax = kx / sn, ay = ky / sn;  // unit axis (z component 0)
    const double K[9] = {0, 0, ay, 0, 0, -ax, -ay, ax, 0};
    const double kk[9] = {ax * ax, ax * ay, 0, ay * ax, ay * ay, 0, 0, 0, 0};
    for (int i = 0; i < 9; ++i) Q[i] = (i % 4 == 0 ? c : 0.0) + sn * K[i] + (1.0 - c) * kk[i];
  }
  const double Qt[9] = {Q[0], Q[3], Q[6], Q[1], Q[4], Q[7], Q[2], Q[5], Q[8]};
  rotation_blocks(p, Q, false, A);   // multipoles into the rotated frame
  m2l_matrix_vec(p, 0.0, 0.0, 2.0 * len, Z);
  rotation_blocks(p, Qt, true, B);   // locals back to the original frame
}

}  // namespace gq
