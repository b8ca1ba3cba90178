// Conventional (point) targets on gfx950, FP64: Algorithm 5 Stages 3, 5(a), 6(a) (direct
// sums over the near sources), 5(b) (multipole evaluation of List 3 far boxes) and 9 (the
// owning box's local evaluated at the target), for targets that have no QBX center.
//
// Kernels (G(x, y) = 1 / (4 pi |x - y|), source normal n_y):
//   single layer  phi(t) = sum_s q_s G(t, s)
//   double layer  phi(t) = sum_s q_s dG/dn_y(t, s) = sum_s q_s n_s . (t - s) / (4 pi |t - s|^3)
// Expansion conventions as in kernels.hip (CS-phase solid harmonics, J = conj(I), scaled
// box expansions mu~ = mu / a^n and l~ = a^(n+1) l, real-packed per degree):
//   multipole at t:  phi = (1/4pi) sum_n [mu_n^0 J_n^0 + 2 sum_{m>0} Re(mu_n^m J_n^m)](t - x_d)
//   local at t:      phi = (1/4pi) sum_n [l_n^0 R_n^0 + 2 sum_{m>0} Re(l_n^m R_n^m)](t - x_b)
// Point targets are in tree order (grouped by owning box); phi[i] accumulates over the
// three launches and the last one writes the potential in input order.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace gq {

namespace {

constexpr double kInv4PiPt = 0.07957747154594767;  // 1/(4 pi)

// Direct sums: one 64-lane wave per item of at most 64 targets of one box; with nt
// targets the wave splits into 64/nt source slices.  Near sources are staged in LDS.
template <int KERN>
__global__ __launch_bounds__(64) void k_p2p(const int* __restrict__ it_box,
                                            const int* __restrict__ it_t0,
                                            const int* __restrict__ it_nt,
                                            const int64_t* __restrict__ near_ptr,
                                            const int* __restrict__ near_idx, SrcSoA src,
                                            const double* __restrict__ qs,
                                            const double* __restrict__ px,
                                            const double* __restrict__ py,
                                            const double* __restrict__ pz,
                                            double* __restrict__ phi) {
  constexpr int NF = KERN ? 6 : 4;
  __shared__ double ss[NF * 64];
  __shared__ double red[64];
  const int item = blockIdx.x;
  const int b = it_box[item];
  const int t0 = it_t0[item], nt = it_nt[item];
  const int S = 64 / nt;
  const int lane = threadIdx.x;
  const int ti = lane % nt, sl = lane / nt;
  const bool active = sl < S;
  const int64_t t = (int64_t)t0 + ti;
  const double xt = px[t], yt = py[t], zt = pz[t];
  double acc = 0.0;
  const int64_t fb = near_ptr[b], fe = near_ptr[b + 1];
  for (int64_t f0 = fb; f0 < fe; f0 += 64) {
    const int n = (int)min((int64_t)64, fe - f0);
    __syncthreads();
    if (lane < n) {
      const int64_t s = near_idx[f0 + lane];
      const double qq = qs[s];
      ss[lane] = src.x[s];
      ss[64 + lane] = src.y[s];
      ss[128 + lane] = src.z[s];
      if constexpr (KERN != 0) {
        ss[192 + lane] = qq * src.nx[s];
        ss[256 + lane] = qq * src.ny[s];
        ss[320 + lane] = qq * src.nz[s];
      } else {
        ss[192 + lane] = qq;
      }
    }
    __syncthreads();
    if (active)
      for (int j = sl; j < n; j += S) {
        const double dx = xt - ss[j], dy = yt - ss[64 + j], dz = zt - ss[128 + j];
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const double ir = 1.0 / sqrt(r2);
        if constexpr (KERN != 0)
          acc = fma(fma(ss[192 + j], dx, fma(ss[256 + j], dy, ss[320 + j] * dz)), ir * ir * ir,
                    acc);
        else
          acc = fma(ss[192 + j], ir, acc);
      }
  }
  __syncthreads();
  red[lane] = active ? acc : 0.0;
  __syncthreads();
  if (sl == 0 && active) {
    double s = 0.0;
    for (int k = 0; k < S; ++k) s += red[k * nt + ti];
    phi[t] += kInv4PiPt * s;
  }
}

// Multipole evaluation: one thread per target, looping over the List 3 far boxes of its
// box (item: targets [t0, t0 + nt) of one box, boxes wf_box[w0 .. w1)).
__global__ __launch_bounds__(64) void k_m2p(int P, const int* __restrict__ it_t0,
                                            const int* __restrict__ it_nt,
                                            const int* __restrict__ it_w0,
                                            const int* __restrict__ it_w1,
                                            const int* __restrict__ wf_box,
                                            const double* __restrict__ bctr,
                                            const double* __restrict__ bh,
                                            const double* __restrict__ M,
                                            const double* __restrict__ px,
                                            const double* __restrict__ py,
                                            const double* __restrict__ pz,
                                            double* __restrict__ phi) {
  const int item = blockIdx.x;
  if ((int)threadIdx.x >= it_nt[item]) return;
  const int64_t t = (int64_t)it_t0[item] + threadIdx.x;
  const double xt = px[t], yt = py[t], zt = pz[t];
  const int np = (P + 1) * (P + 1);
  double sum = 0.0;
  for (int w = it_w0[item]; w < it_w1[item]; ++w) {
    const int d = wf_box[w];
    const double* mu = M + (int64_t)d * np;
    const double a = bh[d];
    const double vx = xt - bctr[3 * d], vy = yt - bctr[3 * d + 1], vz = zt - bctr[3 * d + 2];
    const double ir2 = 1.0 / fma(vx, vx, fma(vy, vy, vz * vz)), zr = vz * ir2;
    double dr = sqrt(ir2), di = 0.0;  // J_0^0
    double box = 0.0;
    for (int m = 0; m <= P; ++m) {
      if (m > 0) {  // J_m^m = -(2m-1)(x - i y)/r^2 J_{m-1}^{m-1}
        const double f = -(2.0 * m - 1.0) * ir2;
        const double fr = f * vx, fi = -f * vy;
        const double nr = fma(dr, fr, -di * fi), ni = fma(dr, fi, di * fr);
        dr = nr;
        di = ni;
      }
      double p1r = dr, p1i = di, p2r = 0.0, p2i = 0.0;
      double an = pow(a, (double)m);  // a^n: the multipole is stored scaled by a^-n
      for (int n = m; n <= P; ++n) {
        double jr = p1r, ji = p1i;
        if (n > m) {
          const double c1 = (2.0 * n - 1.0) * zr;
          const double c2 = (double)((n - 1) * (n - 1) - m * m) * ir2;
          jr = fma(c1, p1r, -c2 * p2r);
          ji = fma(c1, p1i, -c2 * p2i);
          p2r = p1r;
          p2i = p1i;
          p1r = jr;
          p1i = ji;
          an *= a;
        }
        const int o = n * n;
        if (m == 0)
          box = fma(an * mu[o], jr, box);
        else
          box = fma(2.0 * an, mu[o + 2 * m - 1] * jr - mu[o + 2 * m] * ji, box);
      }
    }
    sum += box;
  }
  phi[t] += kInv4PiPt * sum;
}

// Local evaluation and output: one thread per target; its box's local, order P.
__global__ __launch_bounds__(256) void k_l2p(int P, int64_t npt, const int* __restrict__ pt_box,
                                             const double* __restrict__ bctr,
                                             const double* __restrict__ bh,
                                             const double* __restrict__ L,
                                             const double* __restrict__ px,
                                             const double* __restrict__ py,
                                             const double* __restrict__ pz,
                                             const double* __restrict__ phi,
                                             const int64_t* __restrict__ out_idx,
                                             double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= npt) return;
  const int b = pt_box[t];
  const int np = (P + 1) * (P + 1);
  const double* l = L + (int64_t)b * np;
  const double a = bh[b], ia = 1.0 / a;
  const double vx = px[t] - bctr[3 * b], vy = py[t] - bctr[3 * b + 1], vz = pz[t] - bctr[3 * b + 2];
  const double r2 = fma(vx, vx, fma(vy, vy, vz * vz));
  double dr = 1.0, di = 0.0;  // R_0^0
  double sum = 0.0;
  for (int m = 0; m <= P; ++m) {
    if (m > 0) {  // R_m^m = -(x + i y)/(2m) R_{m-1}^{m-1}
      const double f = -0.5 / m;
      const double fr = f * vx, fi = f * vy;
      const double nr = fma(dr, fr, -di * fi), ni = fma(dr, fi, di * fr);
      dr = nr;
      di = ni;
    }
    double p1r = dr, p1i = di, p2r = 0.0, p2i = 0.0;
    double sc = pow(ia, (double)(m + 1));  // the local is stored scaled by a^(n+1)
    for (int n = m; n <= P; ++n) {
      double rr = p1r, ri = p1i;
      if (n > m) {  // R_n^m = [(2n-1) z R_{n-1}^m - r^2 R_{n-2}^m] / (n^2 - m^2)
        const double inv = 1.0 / (double)(n * n - m * m);
        rr = fma((2.0 * n - 1.0) * vz, p1r, -r2 * p2r) * inv;
        ri = fma((2.0 * n - 1.0) * vz, p1i, -r2 * p2i) * inv;
        p2r = p1r;
        p2i = p1i;
        p1r = rr;
        p1i = ri;
        sc *= ia;
      }
      const int o = n * n;
      if (m == 0)
        sum = fma(sc * l[o], rr, sum);
      else
        sum = fma(2.0 * sc, l[o + 2 * m - 1] * rr - l[o + 2 * m] * ri, sum);
    }
  }
  out[out_idx[t]] = phi[t] + kInv4PiPt * sum;
}

}  // namespace

void launch_p2p(hipStream_t s, int kernel, int nitem, const int* it_box, const int* it_t0,
                const int* it_nt, const int64_t* near_ptr, const int* near_idx, SrcSoA src,
                const double* qs, const double* px, const double* py, const double* pz,
                double* phi) {
  if (nitem <= 0) return;
  if (kernel)
    k_p2p<1><<<nitem, 64, 0, s>>>(it_box, it_t0, it_nt, near_ptr, near_idx, src, qs, px, py, pz,
                                  phi);
  else
    k_p2p<0><<<nitem, 64, 0, s>>>(it_box, it_t0, it_nt, near_ptr, near_idx, src, qs, px, py, pz,
                                  phi);
}

void launch_m2p(hipStream_t s, int p, int nitem, const int* it_t0, const int* it_nt,
                const int* it_w0, const int* it_w1, const int* wf_box, const double* bctr,
                const double* bh, const double* M, const double* px, const double* py,
                const double* pz, double* phi) {
  if (nitem <= 0) return;
  k_m2p<<<nitem, 64, 0, s>>>(p, it_t0, it_nt, it_w0, it_w1, wf_box, bctr, bh, M, px, py, pz, phi);
}

void launch_l2p(hipStream_t s, int p, int64_t npt, const int* pt_box, const double* bctr,
                const double* bh, const double* L, const double* px, const double* py,
                const double* pz, const double* phi, const int64_t* out_idx, double* out) {
  if (npt <= 0) return;
  const int64_t blocks = (npt + 255) / 256;
  k_l2p<<<(unsigned)blocks, 256, 0, s>>>(p, npt, pt_box, bctr, bh, L, px, py, pz, phi, out_idx,
                                        out);
}

}  // namespace gq
