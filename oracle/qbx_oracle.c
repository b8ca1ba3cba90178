/*
 * FP64 CPU oracle for 3D Laplace QBX and the GIGAQBX FMM.  TEST INFRASTRUCTURE ONLY:
 * it is called by the tests, by the smoke check and by the benchmark's CPU-baseline leg,
 * never by the library.  It shares no code with the HIP path.
 *
 * Everything here works in the paper's normalization (Section 2.1, the spherical-harmonic
 * expansion of the Green's function and the definition of Y_n^m):
 *
 *   Y_n^m(theta, phi) = sqrt((2n+1)/(4 pi) (n-|m|)!/(n+|m|)!) P_n^|m|(cos theta) e^{i m phi}
 *
 * with P_n^mu the associated Legendre function WITHOUT the Condon-Shortley phase (the paper
 * does not fix the phase; every result below carries it squared).  Coefficient vectors of
 * order p hold (p+1)^2 complex numbers, index n*n + n + m for |m| <= n (the paper's
 * ordering B_0^0, B_1^-1, B_1^0, B_1^1, ...).
 *
 *   local coefficients   (Section 2.1):  L_n^m = 1/(2n+1) |s-c|^-(n+1) Y_n^-m(s-c)
 *   local evaluation                   :  sum L_n^m |t-c|^n Y_n^m(t-c)
 *   multipole coefficients (Sec. 4.2)  :  M_n^m = 1/(2n+1) |s-c|^n Y_n^m(s-c)
 *   multipole evaluation               :  sum M_n^m |t-c|^-(n+1) Y_n^-m(t-c)
 *
 * The double layer uses the kernel d/dn_y G(x,y) with the outward source normal; its
 * coefficients are n_s . grad_s of the single-layer coefficient functions, with the
 * gradient taken in spherical coordinates (radial, polar and azimuthal derivatives).
 *
 * Translations (M2M, M2L, L2L; the paper defers the formulas to Greengard's thesis) are
 * evaluated by the addition theorems of the regular and irregular solid harmonics
 * R_n^m = r^n Y_n^m / (s_m kappa_n N_nm), I_n^m = r^-(n+1) Y_n^m N_nm / (s_m kappa_n),
 * kappa_n = sqrt((2n+1)/(4 pi)), N_nm = sqrt((n-|m|)!(n+|m|)!), s_m = (-1)^m for m > 0
 * and 1 otherwise, which are derived here from the same Y_n^m.  Plain O(p^4) loops, no
 * cached matrices, no real packing, no scaling.
 *
 * Spherical angles are taken from Cartesian components: cos(theta) = z/r,
 * sin(theta) = sqrt(x^2+y^2)/r, e^{i phi} = (x + i y)/sqrt(x^2+y^2) (phi = 0 on the axis);
 * this is the paper's theta = arccos(z/r), phi = atan2(y, x) without the cancellation of
 * arccos near the poles.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define OQ_PI 3.14159265358979323846

static inline int cidx(int n, int m) { return n * n + n + m; }

/* ---------------------------------------------------------------------------------------
 * Spherical harmonics and their angular derivatives
 * ------------------------------------------------------------------------------------- */

typedef struct {
  double r, ct, st, cp, sp;
} sph_t;

static void to_sph(double x, double y, double z, sph_t *s) {
  double rxy = sqrt(x * x + y * y);
  double r = sqrt(x * x + y * y + z * z);
  s->r = r;
  s->ct = z / r;
  s->st = rxy / r;
  if (rxy > 0.0) {
    s->cp = x / rxy;
    s->sp = y / rxy;
  } else {
    s->cp = 1.0;
    s->sp = 0.0;
  }
}

/* sqrt((2n+1)/(4 pi) (n-mu)!/(n+mu)!) */
static double ynorm(int n, int mu) {
  double ratio = 1.0;
  for (int k = n - mu + 1; k <= n + mu; ++k) ratio /= (double)k;
  return sqrt((2.0 * n + 1.0) / (4.0 * OQ_PI) * ratio);
}

/* sqrt((n-mu)!(n+mu)!) */
static double nfact(int n, int mu) {
  double f = 1.0;
  for (int k = 2; k <= n - mu; ++k) f *= (double)k;
  for (int k = 2; k <= n + mu; ++k) f *= (double)k;
  return sqrt(f);
}

/*
 * Y[cidx(n,m)] = Y_n^m, and optionally dY[.] = dY/dtheta and Ys[.] = Y/sin(theta) (m != 0;
 * finite at the poles because P_n^mu carries sin^mu(theta)), for 0 <= n <= p.
 */
static void ylm_all(int p, const sph_t *s, cplx *Y, cplx *dY, cplx *Ys) {
  const int L = p + 2;
  double Pb[(p + 2) * (p + 2)];
  double Ab[(p + 2) * (p + 2)];
  const int pp = p + 1; /* P_n^{mu+1} is needed for dP/dtheta */
  for (int mu = 0; mu <= pp; ++mu) {
    /* P_mu^mu = (2mu-1)!! sin^mu, A_mu^mu = P_mu^mu / sin = (2mu-1)!! sin^(mu-1) */
    double df = 1.0;
    for (int k = 1; k <= 2 * mu - 1; k += 2) df *= (double)k;
    double smu1 = 1.0;
    for (int k = 0; k < mu - 1; ++k) smu1 *= s->st;
    double pmm = (mu == 0) ? 1.0 : df * smu1 * s->st;
    double amm = (mu == 0) ? 0.0 : df * smu1;
    Pb[mu * L + mu] = pmm;
    Ab[mu * L + mu] = amm;
    if (mu + 1 <= pp) {
      Pb[(mu + 1) * L + mu] = (2.0 * mu + 1.0) * s->ct * pmm;
      Ab[(mu + 1) * L + mu] = (2.0 * mu + 1.0) * s->ct * amm;
    }
    for (int n = mu + 2; n <= pp; ++n) {
      Pb[n * L + mu] = ((2.0 * n - 1.0) * s->ct * Pb[(n - 1) * L + mu] -
                        (n + mu - 1.0) * Pb[(n - 2) * L + mu]) / (double)(n - mu);
      Ab[n * L + mu] = ((2.0 * n - 1.0) * s->ct * Ab[(n - 1) * L + mu] -
                        (n + mu - 1.0) * Ab[(n - 2) * L + mu]) / (double)(n - mu);
    }
  }
  /* e^{i m phi} for m = 0..p */
  cplx eim[p + 2];
  eim[0] = 1.0;
  cplx e1 = s->cp + I * s->sp;
  for (int m = 1; m <= p; ++m) eim[m] = eim[m - 1] * e1;
  for (int n = 0; n <= p; ++n) {
    for (int mu = 0; mu <= n; ++mu) {
      double N = ynorm(n, mu);
      double P = Pb[n * L + mu];
      double dP;
      if (mu == 0)
        dP = (n >= 1) ? -Pb[n * L + 1] : 0.0;
      else
        dP = mu * s->ct * Ab[n * L + mu] - ((mu + 1 <= n) ? Pb[n * L + mu + 1] : 0.0);
      cplx ep = eim[mu], em = conj(eim[mu]);
      Y[cidx(n, mu)] = N * P * ep;
      Y[cidx(n, -mu)] = N * P * em;
      if (dY) {
        dY[cidx(n, mu)] = N * dP * ep;
        dY[cidx(n, -mu)] = N * dP * em;
      }
      if (Ys) {
        Ys[cidx(n, mu)] = N * Ab[n * L + mu] * ep;
        Ys[cidx(n, -mu)] = N * Ab[n * L + mu] * em;
      }
    }
  }
}

/*
 * f = r^a Y_n^m(v) for all n <= p, |m| <= n, with a = n (regular) or -(n+1) (irregular).
 * If grad != NULL, grad[3*idx + k] = d f / d v_k:
 *   grad f = r^(a-1) [ a Y rhat + dY/dtheta thetahat + i m (Y / sin theta) phihat ].
 */
static void solid_all(int p, int irregular, const double v[3], cplx *f, cplx *grad) {
  sph_t s;
  to_sph(v[0], v[1], v[2], &s);
  cplx Y[(p + 1) * (p + 1)];
  cplx dY[(p + 1) * (p + 1)];
  cplx Ys[(p + 1) * (p + 1)];
  ylm_all(p, &s, Y, grad ? dY : NULL, grad ? Ys : NULL);
  const double rh[3] = {s.st * s.cp, s.st * s.sp, s.ct};
  const double th[3] = {s.ct * s.cp, s.ct * s.sp, -s.st};
  const double ph[3] = {-s.sp, s.cp, 0.0};
  for (int n = 0; n <= p; ++n) {
    double a = irregular ? -(n + 1.0) : (double)n;
    double ra = pow(s.r, a);
    double ra1 = pow(s.r, a - 1.0);
    for (int m = -n; m <= n; ++m) {
      int i = cidx(n, m);
      f[i] = ra * Y[i];
      if (grad) {
        for (int k = 0; k < 3; ++k)
          grad[3 * i + k] = ra1 * (a * Y[i] * rh[k] + dY[i] * th[k] + I * (double)m * Ys[i] * ph[k]);
      }
    }
  }
}

/* Y_n^m at direction v, paper normalization (exported for pin tests). */
void oq_ylm(int p, double x, double y, double z, double *out_re, double *out_im) {
  sph_t s;
  to_sph(x, y, z, &s);
  cplx Y[(p + 1) * (p + 1)];
  ylm_all(p, &s, Y, NULL, NULL);
  for (int i = 0; i < (p + 1) * (p + 1); ++i) {
    out_re[i] = creal(Y[i]);
    out_im[i] = cimag(Y[i]);
  }
}

/* ---------------------------------------------------------------------------------------
 * Expansion formation and evaluation (paper form)
 * kernel: 0 = single layer S (density times G), 1 = double layer D (dG/dn_y)
 * ------------------------------------------------------------------------------------- */

/* L += q * [1/(2n+1)] Phi_n^{-m}(s - c)  (or n_s . grad_s of it), order p */
static void p2l_one(int kernel, int p, const double *s, const double *nrm, double q,
                    const double *c, cplx *L) {
  double v[3] = {s[0] - c[0], s[1] - c[1], s[2] - c[2]};
  cplx f[(p + 1) * (p + 1)];
  cplx g[3 * (p + 1) * (p + 1)];
  solid_all(p, 1, v, f, kernel ? g : NULL);
  for (int n = 0; n <= p; ++n) {
    double w = q / (2.0 * n + 1.0);
    for (int m = -n; m <= n; ++m) {
      int src = cidx(n, -m); /* Y_n^{-m} */
      cplx val;
      if (kernel == 0)
        val = f[src];
      else
        val = nrm[0] * g[3 * src] + nrm[1] * g[3 * src + 1] + nrm[2] * g[3 * src + 2];
      L[cidx(n, m)] += w * val;
    }
  }
}

/* M += q * [1/(2n+1)] Psi_n^m(s - c)  (or n_s . grad_s of it), order p */
static void p2m_one(int kernel, int p, const double *s, const double *nrm, double q,
                    const double *c, cplx *M) {
  double v[3] = {s[0] - c[0], s[1] - c[1], s[2] - c[2]};
  cplx f[(p + 1) * (p + 1)];
  cplx g[3 * (p + 1) * (p + 1)];
  solid_all(p, 0, v, f, kernel ? g : NULL);
  for (int n = 0; n <= p; ++n) {
    double w = q / (2.0 * n + 1.0);
    for (int m = -n; m <= n; ++m) {
      int i = cidx(n, m);
      cplx val;
      if (kernel == 0)
        val = f[i];
      else
        val = nrm[0] * g[3 * i] + nrm[1] * g[3 * i + 1] + nrm[2] * g[3 * i + 2];
      M[i] += w * val;
    }
  }
}

/* Re sum_{n<=p} L_n^m |t-c|^n Y_n^m(t-c) */
static double eval_local(int p, const cplx *L, const double *c, const double *t) {
  double v[3] = {t[0] - c[0], t[1] - c[1], t[2] - c[2]};
  if (v[0] == 0.0 && v[1] == 0.0 && v[2] == 0.0) /* 0^0 = 1: only L_0^0 Y_0^0 remains */
    return creal(L[0]) * ynorm(0, 0);
  cplx f[(p + 1) * (p + 1)];
  solid_all(p, 0, v, f, NULL);
  cplx acc = 0.0;
  for (int i = 0; i < (p + 1) * (p + 1); ++i) acc += L[i] * f[i];
  return creal(acc);
}

/* Re sum_{n<=p} M_n^m |t-c|^-(n+1) Y_n^-m(t-c) */
static double eval_mpole(int p, const cplx *M, const double *c, const double *t) {
  double v[3] = {t[0] - c[0], t[1] - c[1], t[2] - c[2]};
  cplx f[(p + 1) * (p + 1)];
  solid_all(p, 1, v, f, NULL);
  cplx acc = 0.0;
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) acc += M[cidx(n, m)] * f[cidx(n, -m)];
  return creal(acc);
}

/* ---------------------------------------------------------------------------------------
 * Solid harmonics R, I and the addition-theorem translations
 * ------------------------------------------------------------------------------------- */

static inline double sgn_m(int m) { return (m > 0 && (m & 1)) ? -1.0 : 1.0; }
static inline double kappa(int n) { return sqrt((2.0 * n + 1.0) / (4.0 * OQ_PI)); }

/* R_n^m(v), n <= p: R = r^n Y_n^m / (s_m kappa_n N_nm) */
static void regular_RI(int p, const double *v, cplx *R) {
  if (v[0] == 0.0 && v[1] == 0.0 && v[2] == 0.0) {
    for (int i = 0; i < (p + 1) * (p + 1); ++i) R[i] = 0.0;
    R[0] = 1.0;
    return;
  }
  cplx f[(p + 1) * (p + 1)];
  solid_all(p, 0, v, f, NULL);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m)
      R[cidx(n, m)] = f[cidx(n, m)] / (sgn_m(m) * kappa(n) * nfact(n, abs(m)));
}

/* I_n^m(v), n <= p: I = r^-(n+1) Y_n^m N_nm / (s_m kappa_n) */
static void irregular_RI(int p, const double *v, cplx *Ir) {
  cplx f[(p + 1) * (p + 1)];
  solid_all(p, 1, v, f, NULL);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m)
      Ir[cidx(n, m)] = f[cidx(n, m)] * nfact(n, abs(m)) / (sgn_m(m) * kappa(n));
}

/* paper local L <-> R/I local l:  l = 4 pi s_m kappa_n N_nm L   (phi = 1/(4pi) sum l R) */
/* paper multipole M <-> R/I multipole mu:  mu = 4 pi s_m kappa_n M / N_nm
   (phi = 1/(4pi) sum mu conj(I)) */
static double loc_factor(int n, int m) { return 4.0 * OQ_PI * sgn_m(m) * kappa(n) * nfact(n, abs(m)); }
static double mp_factor(int n, int m) { return 4.0 * OQ_PI * sgn_m(m) * kappa(n) / nfact(n, abs(m)); }

static inline cplx getc(const cplx *a, int p, int n, int m) {
  if (n < 0 || n > p || m < -n || m > n) return 0.0;
  return a[cidx(n, m)];
}

/* multipole at c_from (order p) -> multipole at c_to (order p), accumulate (paper form) */
static void m2m_one(int p, const cplx *M, const double *cf, const double *ct, cplx *Mout) {
  double d[3] = {cf[0] - ct[0], cf[1] - ct[1], cf[2] - ct[2]};
  int np = (p + 1) * (p + 1);
  cplx *mu = malloc(sizeof(cplx) * np), *R = malloc(sizeof(cplx) * np);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) mu[cidx(n, m)] = mp_factor(n, m) * M[cidx(n, m)];
  regular_RI(p, d, R);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) {
      cplx acc = 0.0;
      for (int j = 0; j <= n; ++j)
        for (int k = -j; k <= j; ++k) acc += mu[cidx(j, k)] * getc(R, p, n - j, m - k);
      Mout[cidx(n, m)] += acc / mp_factor(n, m);
    }
  free(mu);
  free(R);
}

/* multipole at c_from (order p) -> local at c_to (order q), accumulate (paper form) */
static void m2l_one(int p, int q, const cplx *M, const double *cf, const double *ct, cplx *Lout) {
  double X[3] = {ct[0] - cf[0], ct[1] - cf[1], ct[2] - cf[2]};
  int pq = p + q;
  cplx *mu = malloc(sizeof(cplx) * (p + 1) * (p + 1));
  cplx *Ir = malloc(sizeof(cplx) * (pq + 1) * (pq + 1));
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) mu[cidx(n, m)] = mp_factor(n, m) * M[cidx(n, m)];
  irregular_RI(pq, X, Ir);
  for (int j = 0; j <= q; ++j)
    for (int k = -j; k <= j; ++k) {
      cplx acc = 0.0;
      for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m) acc += mu[cidx(n, m)] * conj(getc(Ir, pq, n + j, m + k));
      if (j & 1) acc = -acc;
      Lout[cidx(j, k)] += acc / loc_factor(j, k);
    }
  free(mu);
  free(Ir);
}

/* local at c_from (order p) -> local at c_to (order q), accumulate (paper form) */
static void l2l_one(int p, int q, const cplx *L, const double *cf, const double *ct, cplx *Lout) {
  double X[3] = {ct[0] - cf[0], ct[1] - cf[1], ct[2] - cf[2]};
  int np = (p + 1) * (p + 1);
  cplx *l = malloc(sizeof(cplx) * np), *R = malloc(sizeof(cplx) * np);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) l[cidx(n, m)] = loc_factor(n, m) * L[cidx(n, m)];
  regular_RI(p, X, R);
  for (int j = 0; j <= q; ++j)
    for (int k = -j; k <= j; ++k) {
      cplx acc = 0.0;
      for (int n = j; n <= p; ++n)
        for (int m = -n; m <= n; ++m) acc += l[cidx(n, m)] * getc(R, p, n - j, m - k);
      Lout[cidx(j, k)] += acc / loc_factor(j, k);
    }
  free(l);
  free(R);
}

/* ---------------------------------------------------------------------------------------
 * Exported single-expansion routines (complex vectors as interleaved re/im doubles)
 * ------------------------------------------------------------------------------------- */

void oq_p2l(int kernel, int p, int64_t ns, const double *src, const double *nrm,
            const double *q, const double *c, double *Lout) {
  cplx *L = (cplx *)Lout;
  for (int64_t j = 0; j < ns; ++j) p2l_one(kernel, p, src + 3 * j, nrm ? nrm + 3 * j : NULL, q[j], c, L);
}

void oq_p2m(int kernel, int p, int64_t ns, const double *src, const double *nrm,
            const double *q, const double *c, double *Mout) {
  cplx *M = (cplx *)Mout;
  for (int64_t j = 0; j < ns; ++j) p2m_one(kernel, p, src + 3 * j, nrm ? nrm + 3 * j : NULL, q[j], c, M);
}

double oq_eval_local(int p, const double *L, const double *c, const double *t) {
  return eval_local(p, (const cplx *)L, c, t);
}

double oq_eval_mpole(int p, const double *M, const double *c, const double *t) {
  return eval_mpole(p, (const cplx *)M, c, t);
}

void oq_m2m(int p, const double *M, const double *cf, const double *ct, double *Mout) {
  m2m_one(p, (const cplx *)M, cf, ct, (cplx *)Mout);
}

void oq_m2l(int p, int q, const double *M, const double *cf, const double *ct, double *Lout) {
  m2l_one(p, q, (const cplx *)M, cf, ct, (cplx *)Lout);
}

void oq_l2l(int p, int q, const double *L, const double *cf, const double *ct, double *Lout) {
  l2l_one(p, q, (const cplx *)L, cf, ct, (cplx *)Lout);
}

/* R_n^m and I_n^m (for pin tests of the addition theorems) */
void oq_regular_RI(int p, const double *v, double *out) { regular_RI(p, v, (cplx *)out); }
void oq_irregular_RI(int p, const double *v, double *out) { irregular_RI(p, v, (cplx *)out); }

/* ---------------------------------------------------------------------------------------
 * Batched routines (OpenMP over the destinations; each destination owns its output)
 * ------------------------------------------------------------------------------------- */

static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

/*
 * Local coefficients (order p) at n_ctr centers that all see the same sources
 * src_idx[0..n_idx) (src_idx == NULL: sources 0..n_idx-1).
 * Lout: n_ctr * (p+1)^2 complex, overwritten.
 */
void oq_p2l_shared(int kernel, int p, int64_t n_ctr, const double *ctr, int64_t n_idx,
                   const int64_t *src_idx, const double *src, const double *nrm,
                   const double *q, double *Lout, int nthreads) {
  set_threads(nthreads);
  const int np = (p + 1) * (p + 1);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t c = 0; c < n_ctr; ++c) {
    cplx *L = (cplx *)Lout + c * np;
    for (int i = 0; i < np; ++i) L[i] = 0.0;
    for (int64_t k = 0; k < n_idx; ++k) {
      int64_t j = src_idx ? src_idx[k] : k;
      p2l_one(kernel, p, src + 3 * j, nrm ? nrm + 3 * j : NULL, q[j], ctr + 3 * c, L);
    }
  }
}

/* Multipoles (order p) of n_box boxes, each from a CSR list of sources. Overwrites Mout. */
void oq_p2m_csr(int kernel, int p, int64_t n_box, const double *ctr, const int64_t *ptr,
                const int64_t *src_idx, const double *src, const double *nrm, const double *q,
                double *Mout, int nthreads) {
  set_threads(nthreads);
  const int np = (p + 1) * (p + 1);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < n_box; ++b) {
    cplx *M = (cplx *)Mout + b * np;
    for (int i = 0; i < np; ++i) M[i] = 0.0;
    for (int64_t k = ptr[b]; k < ptr[b + 1]; ++k) {
      int64_t j = src_idx[k];
      p2m_one(kernel, p, src + 3 * j, nrm ? nrm + 3 * j : NULL, q[j], ctr + 3 * b, M);
    }
  }
}

/*
 * Multipole-to-local: destination i (center dst[3i]) receives, for each k in
 * [ptr[i], ptr[i+1]), the order-q local of multipole M[src_box[k]] (order p, center
 * mcen[3*src_box[k]]).  Lout: n_dst * (q+1)^2 complex, ACCUMULATED.
 */
void oq_m2l_csr(int p, int q, int64_t n_dst, const double *dst, const int64_t *ptr,
                const int64_t *src_box, const double *M, const double *mcen, double *Lout,
                int nthreads) {
  set_threads(nthreads);
  const int np = (p + 1) * (p + 1), nq = (q + 1) * (q + 1);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n_dst; ++i)
    for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
      int64_t d = src_box[k];
      m2l_one(p, q, (const cplx *)M + d * np, mcen + 3 * d, dst + 3 * i, (cplx *)Lout + i * nq);
    }
}

/* Local-to-local with the same CSR layout as oq_m2l_csr (L: order p, Lout: order q). */
void oq_l2l_csr(int p, int q, int64_t n_dst, const double *dst, const int64_t *ptr,
                const int64_t *src_box, const double *L, const double *lcen, double *Lout,
                int nthreads) {
  set_threads(nthreads);
  const int np = (p + 1) * (p + 1), nq = (q + 1) * (q + 1);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n_dst; ++i)
    for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
      int64_t d = src_box[k];
      l2l_one(p, q, (const cplx *)L + d * np, lcen + 3 * d, dst + 3 * i, (cplx *)Lout + i * nq);
    }
}

/* phi[t] = eval of local L[tgt_center[t]] (order q, center ctr) at tgt[t] */
void oq_eval_locals(int q, int64_t n_tgt, const double *tgt, const int64_t *tgt_center,
                    const double *ctr, const double *L, double *out, int nthreads) {
  set_threads(nthreads);
  const int nq = (q + 1) * (q + 1);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < n_tgt; ++t) {
    int64_t c = tgt_center[t];
    out[t] = eval_local(q, (const cplx *)L + c * nq, ctr + 3 * c, tgt + 3 * t);
  }
}

/*
 * Tier A: direct (unaccelerated) QBX.  For each center, the order-q local expansion of
 * the layer potential discretized by the quadrature sum (all sources); each target is
 * evaluated through its center.  Centers/targets may be any subset (sampling).
 * strength = w * mu.  Returns the number of threads used.
 */
int oq_direct_qbx(int kernel, int q, int64_t n_src, const double *src, const double *nrm,
                  const double *strength, int64_t n_ctr, const double *ctr, int64_t n_tgt,
                  const double *tgt, const int64_t *tgt_center, double *out, int nthreads) {
  const int nq = (q + 1) * (q + 1);
  double *L = malloc(sizeof(cplx) * nq * (size_t)(n_ctr > 0 ? n_ctr : 1));
  oq_p2l_shared(kernel, q, n_ctr, ctr, n_src, NULL, src, nrm, strength, L, nthreads);
  oq_eval_locals(q, n_tgt, tgt, tgt_center, ctr, L, out, nthreads);
  free(L);
  int used = 1;
#ifdef _OPENMP
#pragma omp parallel
  {
#pragma omp single
    used = omp_get_num_threads();
  }
#endif
  return used;
}
