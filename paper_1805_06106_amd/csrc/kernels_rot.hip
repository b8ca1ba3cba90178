// M2L (Algorithm 5, Stage 4) by rotation on gfx950, FP64 matrix cores.
//
// For an offset class the dense real-packed M2L matrix factors as T = B Z A (built on the
// host, translations.cpp): A rotates the source multipoles into a frame where the offset
// points along +z, Z translates along z, which couples only equal orders m, and B rotates
// the local expansions back.  A and B are block diagonal by degree (blocks of 2n+1), Z
// block diagonal by order once its rows are grouped by (order, real/imaginary part) (blocks
// of p+1-m).  With 16 x 16 tiles, A and B have 44 nonzero tiles at p = 15 and Z 31 diagonal
// blocks, against 256 tiles of the dense matrix: about half the matrix-core work.
//
// One workgroup of 4 waves per tile of up to 32 pairs of one class; the 256 x 32 working
// matrix lives in LDS between the three products.
//   stage 0  Y = X          the source multipoles, one coalesced 2 KB read per pair
//   stage 1  Y = A Y        all products read before any row is written back
//   stage 2  Y = Z Y        in place, one order block at a time (row gather/scatter)
//   stage 3  L += B Y       computed transposed (L^T = Y^T B^T) so that the atomic adds of
//                           16 lanes go to 16 consecutive coefficients of one pair (or, with
//                           to_slots, the stores to the pair's own slot)
// MFMA layout of v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register r of lane l holds D[l / 16 + 4 r][l % 16].
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace gq {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kRC = kRotCols;  // pairs per tile, columns of the LDS working matrix
constexpr int kRotXcds = 8;    // MI355X: 8 accelerator complex dies, one L2 each

// LDS address of working-matrix element (row, col): rows of kRC doubles with the column
// XOR-swizzled by the row, so that a wave touching 64 consecutive rows of one column (the
// staging) or 16 columns of 4 rows (the matrix-core operands) spreads over the banks.
__device__ __forceinline__ int wsw(int row, int col) { return row * kRC + (col ^ (row & 31)); }

// Each wave owns up to kSlots row tiles (R.row_order[wave + 4 j]); its products for all of
// them are issued interleaved, tile index k outermost, so up to 2 kSlots independent
// accumulation chains are in flight.
constexpr int kSlots = 4;

// TO_SLOTS: each pair's result is stored to its own slot Y[pair position] instead of added
// into Y[dst] (deterministic plans).
template <bool TO_SLOTS>
__global__ __launch_bounds__(256) void k_m2l_rot(int np, const int* __restrict__ tile_cls,
                                                 const int* __restrict__ tile_beg,
                                                 const int* __restrict__ tile_cnt,
                                                 const int* __restrict__ pair_src,
                                                 const int* __restrict__ pair_dst, RotMats R,
                                                 const double* __restrict__ X,
                                                 double* __restrict__ Y, int ntile,
                                                 int per_xcd) {
  __shared__ double W[kRotRows * kRC];
  const int t = per_xcd ? (blockIdx.x % kRotXcds) * per_xcd + blockIdx.x / kRotXcds : blockIdx.x;
  if (t >= ntile) return;
  const int cls = tile_cls[t], beg = tile_beg[t], cnt = tile_cnt[t];
  const double* A = R.A + (size_t)cls * R.ntile * 256;
  const double* Z = R.Z + (size_t)cls * R.nblk * 256;
  const double* B = R.B + (size_t)cls * R.ntile * 256;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  // stage 0: W = X, one pair's coefficients per 256 consecutive threads (coalesced)
  for (int col = 0; col < kRC; ++col) {
    const int row = threadIdx.x;
    double v = 0.0;
    if (col < cnt && row < np) v = X[(int64_t)pair_src[beg + col] * np + row];
    W[wsw(row, col)] = v;
  }
  // this wave's row tiles and their tile ranges
  int rr[kSlots], tb[kSlots], te[kSlots], kmax = 0;
#pragma unroll
  for (int j = 0; j < kSlots; ++j) {
    rr[j] = R.row_order[wave + 4 * j];  // 16 entries, -1 = none
    tb[j] = rr[j] >= 0 ? R.row_beg[rr[j]] : 0;
    te[j] = rr[j] >= 0 ? R.row_beg[rr[j] + 1] : 0;
    kmax = max(kmax, te[j] - tb[j]);
  }
  __syncthreads();
  // stage 1: W = A W, all of the wave's row tiles computed before any is written back
  d4 acc[kSlots][2];
#pragma unroll
  for (int j = 0; j < kSlots; ++j) acc[j][0] = acc[j][1] = d4{0, 0, 0, 0};
  for (int k = 0; k < kmax; ++k)
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
      const int ti = tb[j] + k;
      if (ti >= te[j]) continue;  // uniform over the wave
      const int c = R.tile_c[ti];
      const double* At = A + (size_t)ti * 256;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double a = At[(4 * s + lk) * 16 + li];
        const int krow = 16 * c + 4 * s + lk;
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[j][h] = mfma16(a, W[wsw(krow, 16 * h + li)], acc[j][h]);
      }
    }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kSlots; ++j)
    if (rr[j] >= 0)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) W[wsw(16 * rr[j] + lk + 4 * i, 16 * h + li)] = acc[j][h][i];
  __syncthreads();
  // stage 2: W = Z W in place; block b holds the rows of one (order, re/im) group, so the
  // blocks touch disjoint rows and each is read completely before it is written
  for (int b0 = wave; b0 < R.nblk; b0 += 4 * kSlots) {
    d4 zc[kSlots][2];
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
      zc[j][0] = zc[j][1] = d4{0, 0, 0, 0};
      const int b = b0 + 4 * j;
      if (b >= R.nblk) continue;
      const double* Zt = Z + (size_t)b * 256;
      const int* rm = R.rowmap + b * 16;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double a = Zt[(4 * s + lk) * 16 + li];
        const int kr = rm[4 * s + lk];
        const int row = kr < 0 ? 0 : kr;  // padding: Z is zero there
#pragma unroll
        for (int h = 0; h < 2; ++h) zc[j][h] = mfma16(a, W[wsw(row, 16 * h + li)], zc[j][h]);
      }
    }
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
      const int b = b0 + 4 * j;
      if (b >= R.nblk) continue;
      const int* rm = R.rowmap + b * 16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rm[lk + 4 * i];
        if (row >= 0)
#pragma unroll
          for (int h = 0; h < 2; ++h) W[wsw(row, 16 * h + li)] = zc[j][h][i];
      }
    }
  }
  __syncthreads();
  // stage 3: L^T += W^T B^T per row tile r of L; lane holds (pair lk + 4 i, row 16 r + li)
#pragma unroll
  for (int j = 0; j < kSlots; ++j) acc[j][0] = acc[j][1] = d4{0, 0, 0, 0};
  for (int k = 0; k < kmax; ++k)
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
      const int ti = tb[j] + k;
      if (ti >= te[j]) continue;
      const int c = R.tile_c[ti];
      const double* Bt = B + (size_t)ti * 256;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double bb = Bt[(4 * s + lk) * 16 + li];
        const int krow = 16 * c + 4 * s + lk;
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[j][h] = mfma16(W[wsw(krow, 16 * h + li)], bb, acc[j][h]);
      }
    }
#pragma unroll
  for (int j = 0; j < kSlots; ++j) {
    if (rr[j] < 0) continue;
    const int row = 16 * rr[j] + li;
    if (row >= np) continue;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pair = 16 * h + lk + 4 * i;
        if (pair >= cnt) continue;
        if constexpr (TO_SLOTS)
          Y[(int64_t)(beg + pair) * np + row] = acc[j][h][i];
        else
          unsafeAtomicAdd(&Y[(int64_t)pair_dst[beg + pair] * np + row], acc[j][h][i]);
      }
  }
}

}  // namespace

void launch_m2l_rot(hipStream_t s, int np, int ntile, const int* tile_cls, const int* tile_beg,
                    const int* tile_cnt, const int* pair_src, const int* pair_dst,
                    const RotMats& R, const double* X, double* Y, bool xcd_order,
                    bool to_slots) {
  if (ntile <= 0) return;
  const int per_xcd = xcd_order ? (ntile + kRotXcds - 1) / kRotXcds : 0;
  const dim3 grid(xcd_order ? per_xcd * kRotXcds : ntile);
  auto k = to_slots ? k_m2l_rot<true> : k_m2l_rot<false>;
  k<<<grid, 256, 0, s>>>(np, tile_cls, tile_beg, tile_cnt, pair_src, pair_dst, R, X, Y, ntile,
                         per_xcd);
}

}  // namespace gq
