// Target association on gfx950 (Algorithm 3 with the side preference of Section 3).
//
// The host sorts sources and centers into a uniform grid whose cell is at least the
// largest query radius (the source danger radii and the tolerance-widened center radii),
// so every source or center within reach of a target lies in the 27 cells around the
// target's cell.  One thread per target, from the target's point of view (as the paper's
// own parallel implementation): first "is some source's danger zone around me", then "which
// admissible center ball holds me, closest first".  Squared distances are formed without
// fused multiply-adds, ((dx*dx + dy*dy) + dz*dz), so every decision matches a plain FP64
// evaluation in that order bit for bit.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace gq {

namespace {

// No contraction into fused multiply-adds here: hipcc fuses a*b + c by default, which
// would round differently from the separate products and sums the decisions are defined by.
__device__ __forceinline__ double dist2(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ double sq(double r) {
#pragma clang fp contract(off)
  return r * r;
}

__device__ __forceinline__ int cell_of(double x, double lo, double h, int n) {
  const int i = (int)floor((x - lo) / h);
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

__global__ __launch_bounds__(256) void k_associate(int64_t nt, const double* __restrict__ tx,
                                                   const double* __restrict__ ty,
                                                   const double* __restrict__ tz,
                                                   const int8_t* __restrict__ tside,
                                                   AssocGrid g, AssocCells src, AssocCells ctr,
                                                   int64_t* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const double x = tx[t], y = ty[t], z = tz[t];
  const int ix = cell_of(x, g.lo[0], g.h, g.n[0]);
  const int iy = cell_of(y, g.lo[1], g.h, g.n[1]);
  const int iz = cell_of(z, g.lo[2], g.h, g.n[2]);
  const int x0 = max(ix - 1, 0), x1 = min(ix + 1, g.n[0] - 1);
  const int y0 = max(iy - 1, 0), y1 = min(iy + 1, g.n[1] - 1);
  const int z0 = max(iz - 1, 0), z1 = min(iz + 1, g.n[2] - 1);
  bool endangered = false;
  for (int cz = z0; cz <= z1 && !endangered; ++cz)
    for (int cy = y0; cy <= y1 && !endangered; ++cy)
      for (int cx = x0; cx <= x1 && !endangered; ++cx) {
        const int64_t cell = ((int64_t)cz * g.n[1] + cy) * g.n[0] + cx;
        for (int64_t k = src.start[cell]; k < src.start[cell + 1]; ++k) {
          const double r = src.r[k];
          if (dist2(x - src.x[k], y - src.y[k], z - src.z[k]) <= sq(r)) {
            endangered = true;
            break;
          }
        }
      }
  if (!endangered) {
    out[t] = -1;
    return;
  }
  const int side = tside ? (int)tside[t] : 0;
  int64_t best = -2;
  double bestd = 0.0;
  for (int cz = z0; cz <= z1; ++cz)
    for (int cy = y0; cy <= y1; ++cy)
      for (int cx = x0; cx <= x1; ++cx) {
        const int64_t cell = ((int64_t)cz * g.n[1] + cy) * g.n[0] + cx;
        for (int64_t k = ctr.start[cell]; k < ctr.start[cell + 1]; ++k) {
          if (side != 0 && (int)ctr.side[k] != side) continue;
          const double r = ctr.r[k];
          const double d = dist2(x - ctr.x[k], y - ctr.y[k], z - ctr.z[k]);
          if (d <= sq(r)) {
            const int64_t id = ctr.id[k];
            if (best < 0 || d < bestd || (d == bestd && id < best)) {
              best = id;
              bestd = d;
            }
          }
        }
      }
  out[t] = best;
}

// One thread per query: does any point of the grid lie within r of it?
__global__ __launch_bounds__(256) void k_points_near(int64_t nq, const double* __restrict__ qx,
                                                     const double* __restrict__ qy,
                                                     const double* __restrict__ qz,
                                                     const double* __restrict__ qr, int strict,
                                                     AssocGrid g, AssocCells pts,
                                                     uint8_t* __restrict__ hit) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nq) return;
  const double x = qx[t], y = qy[t], z = qz[t], r2 = sq(qr[t]);
  const int ix = cell_of(x, g.lo[0], g.h, g.n[0]);
  const int iy = cell_of(y, g.lo[1], g.h, g.n[1]);
  const int iz = cell_of(z, g.lo[2], g.h, g.n[2]);
  bool found = false;
  for (int cz = max(iz - 1, 0); cz <= min(iz + 1, g.n[2] - 1) && !found; ++cz)
    for (int cy = max(iy - 1, 0); cy <= min(iy + 1, g.n[1] - 1) && !found; ++cy)
      for (int cx = max(ix - 1, 0); cx <= min(ix + 1, g.n[0] - 1) && !found; ++cx) {
        const int64_t cell = ((int64_t)cz * g.n[1] + cy) * g.n[0] + cx;
        for (int64_t k = pts.start[cell]; k < pts.start[cell + 1]; ++k) {
          const double d = dist2(x - pts.x[k], y - pts.y[k], z - pts.z[k]);
          if (strict ? d < r2 : d <= r2) {
            found = true;
            break;
          }
        }
      }
  hit[t] = found ? 1 : 0;
}

}  // namespace

void launch_points_near(hipStream_t s, int64_t nq, const double* qx, const double* qy,
                        const double* qz, const double* r, int strict, const AssocGrid& g,
                        const AssocCells& pts, uint8_t* hit) {
  if (nq <= 0) return;
  const int64_t blocks = (nq + 255) / 256;
  k_points_near<<<(unsigned)blocks, 256, 0, s>>>(nq, qx, qy, qz, r, strict, g, pts, hit);
}

void launch_associate(hipStream_t s, int64_t nt, const double* tx, const double* ty,
                      const double* tz, const int8_t* tside, const AssocGrid& g,
                      const AssocCells& src, const AssocCells& ctr, int64_t* out) {
  if (nt <= 0) return;
  const int64_t blocks = (nt + 255) / 256;
  k_associate<<<(unsigned)blocks, 256, 0, s>>>(nt, tx, ty, tz, tside, g, src, ctr, out);
}

}  // namespace gq
