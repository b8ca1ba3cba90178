// Source-to-box expansions on gfx950: P2M of leaf boxes (Algorithm 5, Stage 2) and P2L
// from the sources of List 4 far boxes (Stage 6(b)), FP64.
//
// Conventions as in kernels.hip: scaled box expansions (mu~ = mu / a^n, l~ = a^(n+1) l,
// a the box half-width), real-packed per degree.  The table H of solid harmonics of the
// scaled source offset u = (s - x_b) / a is H = R (regular, P2M) or H = J = conj(I)
// (irregular, P2L), degrees N = 0..NT.  The kernel accumulates the moments
//   single layer:  A_N^m = sum_s q_s H_N^m
//   double layer:  A_N^m = sum w_z H_N^m,  B_N^m = sum beta H_N^m,  C_N^m = sum conj(beta) H_N^m
// (w_z, beta from the source weight, normal and scale; see the staging step) and combines
// them into the output coefficient of degree n and order m as
//   P2M:  mu_n^m = A_{n-1}^m + B_{n-1}^{m+1} - C_{n-1}^{m-1}
//   P2L:  l_n^m  = A_{n+1}^m + B_{n+1}^{m+1} - C_{n+1}^{m-1}
// with H^-1 = -conj(H^1), so the order-0 output is A^0 + 2 Re(B^1).
//
// Work split: a 256-thread block per box.  Sources are staged in LDS 64 at a time; one
// thread per source computes the scaled offset, the weights and the diagonal H_m^m,
// m = 0..NT.  Every thread then owns one moment t and the two orders m and NT - m (their
// columns together have NT + 2 entries, so all threads carry the same load) for a slice of
// the staged sources: it runs the upward degree recurrence of its two columns from the
// staged diagonal and accumulates in registers.  No cross-lane reduction happens per
// source; at the end each thread adds its column entries into an LDS moment table, with LDS
// atomics or (ordered, for reproducible results) one slice at a time in slice order, and the
// block combines the moments into the output.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace gq {

namespace {

constexpr int kChunk = 64;                              // sources staged per round
constexpr int kInv = kPmax + 3;                          // 1/(N^2 - m^2) table side
constexpr int kTri = (kPmax + 2) * (kPmax + 3) / 2;     // entries 0 <= m <= N <= kPmax + 1

__device__ __forceinline__ int tri(int N, int m) { return N * (N + 1) / 2 + m; }

// EMAX >= NT + 2: entries per thread (its two columns); the diagonal table holds NT + 1.
// Up to EMAX = 18 (p = 15 and below) the registers are capped for 4 waves per SIMD, which
// the LDS footprint of a block also allows.
template <int KERN, bool IRR, int EMAX>
__global__ __launch_bounds__(256, EMAX <= 18 ? 4 : 1) void k_p2x(int P, const int* __restrict__ boxes,
                                             const int64_t* __restrict__ ptr,
                                             const int* __restrict__ idx,
                                             const double* __restrict__ bctr,
                                             const double* __restrict__ bh, SrcSoA src,
                                             const double* __restrict__ q,
                                             double* __restrict__ out, int ordered) {
  constexpr int NMOM = KERN ? 3 : 1;
  constexpr int DMAX = EMAX - 1;
  __shared__ double sdiag[kChunk][DMAX][2];  // H_m^m of each staged source
  __shared__ double sgeo[kChunk][2];         // IRR: (u_z / |u|^2, 1 / |u|^2); else (u_z, |u|^2)
  __shared__ double swt[kChunk][3];          // S: q; D: (w_z, Re beta, Im beta)
  __shared__ double res[NMOM][kTri][2];
  __shared__ double invtab[kInv * kInv];     // 1/(N^2 - m^2), regular recurrence only
  const int NT = IRR ? P + KERN : P - KERN;
  const int tid = threadIdx.x;
  for (int i = tid; i < NMOM * kTri * 2; i += 256) (&res[0][0][0])[i] = 0.0;
  if (!IRR)
    for (int i = tid; i < kInv * kInv; i += 256) {
      const int n = i / kInv, m = i % kInv;
      invtab[i] = n > m ? 1.0 / (double)(n * n - m * m) : 0.0;
    }
  const int item = blockIdx.x;
  const int b = boxes[item];
  const double a = bh[b], inv_a = 1.0 / a;
  const double xb = bctr[3 * b], yb = bctr[3 * b + 1], zb = bctr[3 * b + 2];
  const int64_t f0 = ptr[item], f1 = ptr[item + 1];
  // thread -> (moment t, column pair (mA, mB = NT - mA), source slice)
  const int npairs = NT >= 0 ? NT / 2 + 1 : 1;
  const int G = npairs * NMOM;
  const int S = 256 / G;
  const int g = tid % G, sl = tid / G;
  const bool active = NT >= 0 && sl < S;
  const int t = g % NMOM, mA = g / NMOM, mB = NT - mA;
  const int LA = NT + 1 - mA;                  // entries N = mA..NT of column mA
  const int ntot = mB > mA ? NT + 2 : LA;      // plus N = mB..NT of column mB
  double acc[EMAX][2];
#pragma unroll
  for (int i = 0; i < EMAX; ++i) acc[i][0] = acc[i][1] = 0.0;
  for (int64_t base = f0; base < f1; base += kChunk) {
    const int n = (int)min((int64_t)kChunk, f1 - base);
    __syncthreads();
    if (tid < n && NT >= 0) {
      const int64_t s = idx[base + tid];
      const double ux = (src.x[s] - xb) * inv_a, uy = (src.y[s] - yb) * inv_a,
                   uz = (src.z[s] - zb) * inv_a;
      const double r2 = fma(ux, ux, fma(uy, uy, uz * uz));
      const double qq = q[s];
      double dr, di = 0.0;
      if (IRR) {
        const double ir2 = 1.0 / r2;
        sgeo[tid][0] = uz * ir2;
        sgeo[tid][1] = ir2;
        dr = sqrt(ir2);  // J_0^0 = 1/|u|
      } else {
        sgeo[tid][0] = uz;
        sgeo[tid][1] = r2;
        dr = 1.0;  // R_0^0
      }
      sdiag[tid][0][0] = dr;
      sdiag[tid][0][1] = 0.0;
      for (int m = 1; m <= NT; ++m) {
        double fr, fi;
        if (IRR) {  // J_m^m = -(2m-1)(x - i y)/|u|^2 J_{m-1}^{m-1}
          const double c = -(2.0 * m - 1.0) * sgeo[tid][1];
          fr = c * ux;
          fi = -c * uy;
        } else {  // R_m^m = -(x + i y)/(2m) R_{m-1}^{m-1}
          const double c = -0.5 / m;
          fr = c * ux;
          fi = c * uy;
        }
        const double nr = fma(dr, fr, -di * fi), ni = fma(dr, fi, di * fr);
        dr = nr;
        di = ni;
        sdiag[tid][m][0] = dr;
        sdiag[tid][m][1] = di;
      }
      if (KERN) {
        // P2M (R ladders): w_z = q n_z / a, beta = q (n_x - i n_y) / (2a);
        // P2L (J ladders): w_z = -q n_z / a, beta = q (n_x + i n_y) / (2a)
        const double sz = IRR ? -1.0 : 1.0, sy = IRR ? 1.0 : -1.0;
        swt[tid][0] = sz * qq * src.nz[s] * inv_a;
        swt[tid][1] = 0.5 * qq * src.nx[s] * inv_a;
        swt[tid][2] = sy * 0.5 * qq * src.ny[s] * inv_a;
      } else {
        swt[tid][0] = qq;
      }
    }
    __syncthreads();
    if (active) {
      for (int j = sl; j < n; j += S) {
        double wr, wi;
        if (!KERN) {
          wr = swt[j][0];
          wi = 0.0;
        } else if (t == 0) {
          wr = swt[j][0];
          wi = 0.0;
        } else {
          wr = swt[j][1];
          wi = t == 1 ? swt[j][2] : -swt[j][2];
        }
        const double g0 = sgeo[j][0], g1 = sgeo[j][1];
        double p1r = sdiag[j][mA][0], p1i = sdiag[j][mA][1], p2r = 0.0, p2i = 0.0;
        int N = mA, m = mA;
#pragma unroll
        for (int i = 0; i < EMAX; ++i) {
          if (i < ntot) {
            double hr, hi;
            if (i == 0) {
              hr = p1r;
              hi = p1i;
            } else if (i == LA) {  // second column: restart from its diagonal
              N = mB;
              m = mB;
              p1r = sdiag[j][mB][0];
              p1i = sdiag[j][mB][1];
              p2r = p2i = 0.0;
              hr = p1r;
              hi = p1i;
            } else {
              ++N;
              if (IRR) {  // J_N^m = [(2N-1) z J_{N-1}^m - ((N-1)^2 - m^2) J_{N-2}^m] / |u|^2
                const double c1 = (2.0 * N - 1.0) * g0;
                const double c2 = (double)((N - 1) * (N - 1) - m * m) * g1;
                hr = fma(c1, p1r, -c2 * p2r);
                hi = fma(c1, p1i, -c2 * p2i);
              } else {  // R_N^m = [(2N-1) z R_{N-1}^m - |u|^2 R_{N-2}^m] / (N^2 - m^2)
                const double c1 = (2.0 * N - 1.0) * g0;
                const double tt = invtab[N * kInv + m];
                hr = fma(c1, p1r, -g1 * p2r) * tt;
                hi = fma(c1, p1i, -g1 * p2i) * tt;
              }
              p2r = p1r;
              p2i = p1i;
              p1r = hr;
              p1i = hi;
            }
            acc[i][0] = fma(wr, hr, fma(-wi, hi, acc[i][0]));
            acc[i][1] = fma(wr, hi, fma(wi, hr, acc[i][1]));
          }
        }
      }
    }
  }
  // moments of all slices into the LDS table
  __syncthreads();  // the table's clearing is complete even when the item has no sources
  if (ordered) {
    // one slice after the other in slice order: within a slice every table entry belongs
    // to one thread, so the sums are plain adds in a fixed order, the same on every run
    for (int r = 0; r < S; ++r) {
      if (active && sl == r) {
#pragma unroll
        for (int i = 0; i < EMAX; ++i) {
          if (i < ntot) {
            const int m = i < LA ? mA : mB;
            const int N = i < LA ? mA + i : mB + (i - LA);
            res[t][tri(N, m)][0] += acc[i][0];
            res[t][tri(N, m)][1] += acc[i][1];
          }
        }
      }
      __syncthreads();
    }
  } else {
    if (active) {
#pragma unroll
      for (int i = 0; i < EMAX; ++i) {
        if (i < ntot) {
          const int m = i < LA ? mA : mB;
          const int N = i < LA ? mA + i : mB + (i - LA);
          atomicAdd(&res[t][tri(N, m)][0], acc[i][0]);
          atomicAdd(&res[t][tri(N, m)][1], acc[i][1]);
        }
      }
    }
    __syncthreads();
  }
  auto mom = [&](int tt, int N, int m, int c) -> double { return res[tt][tri(N, m)][c]; };
  const int np = (P + 1) * (P + 1);
  double* o = out + (int64_t)b * np;
  for (int i = tid; i < np; i += 256) {
    int n = (int)sqrt((double)i);
    while (n * n > i) --n;
    while ((n + 1) * (n + 1) <= i) ++n;
    const int off = i - n * n;
    const int m = (off + 1) >> 1;
    const int c = (off == 0) ? 0 : ((off & 1) ? 0 : 1);
    double v;
    if (!KERN) {
      v = mom(0, n, m, c);
    } else {
      const int N = IRR ? n + 1 : n - 1;
      if (N < 0) {
        v = 0.0;
      } else {
        v = (m <= N) ? mom(0, N, m, c) : 0.0;
        if (m == 0) {
          v += (N >= 1) ? 2.0 * mom(1, N, 1, 0) : 0.0;
        } else {
          if (m + 1 <= N) v += mom(1, N, m + 1, c);
          if (m - 1 <= N) v -= mom(NMOM - 1, N, m - 1, c);
        }
      }
    }
    if (IRR)
      o[i] += v;
    else
      o[i] = v;
  }
}

template <int KERN, bool IRR>
void launch_p2x_k(hipStream_t s, int p, int nitem, const int* boxes, const int64_t* ptr,
                  const int* idx, const double* bctr, const double* bh, SrcSoA src,
                  const double* q, double* out, int ordered) {
  const int NT = IRR ? p + KERN : p - KERN;
  const int e = NT + 2;
  if (e <= 8)
    k_p2x<KERN, IRR, 8><<<nitem, 256, 0, s>>>(p, boxes, ptr, idx, bctr, bh, src, q, out, ordered);
  else if (e <= 12)
    k_p2x<KERN, IRR, 12><<<nitem, 256, 0, s>>>(p, boxes, ptr, idx, bctr, bh, src, q, out, ordered);
  else if (e <= 16)
    k_p2x<KERN, IRR, 16><<<nitem, 256, 0, s>>>(p, boxes, ptr, idx, bctr, bh, src, q, out, ordered);
  else if (e <= 18)
    k_p2x<KERN, IRR, 18><<<nitem, 256, 0, s>>>(p, boxes, ptr, idx, bctr, bh, src, q, out, ordered);
  else if (e <= 20)
    k_p2x<KERN, IRR, 20><<<nitem, 256, 0, s>>>(p, boxes, ptr, idx, bctr, bh, src, q, out, ordered);
  else
    k_p2x<KERN, IRR, 24><<<nitem, 256, 0, s>>>(p, boxes, ptr, idx, bctr, bh, src, q, out, ordered);
}

}  // namespace

void launch_p2m(hipStream_t s, int kernel, int p, int nitem, const int* boxes,
                const int64_t* ptr, const int* idx, const double* bctr, const double* bh,
                SrcSoA src, const double* q, double* M, bool ordered) {
  if (nitem <= 0) return;
  if (kernel)
    launch_p2x_k<1, false>(s, p, nitem, boxes, ptr, idx, bctr, bh, src, q, M, ordered);
  else
    launch_p2x_k<0, false>(s, p, nitem, boxes, ptr, idx, bctr, bh, src, q, M, ordered);
}

void launch_p2l(hipStream_t s, int kernel, int p, int nitem, const int* boxes,
                const int64_t* ptr, const int* idx, const double* bctr, const double* bh,
                SrcSoA src, const double* q, double* L, bool ordered) {
  if (nitem <= 0) return;
  if (kernel)
    launch_p2x_k<1, true>(s, p, nitem, boxes, ptr, idx, bctr, bh, src, q, L, ordered);
  else
    launch_p2x_k<0, true>(s, p, nitem, boxes, ptr, idx, bctr, bh, src, q, L, ordered);
}

}  // namespace gq
