// M2L (Algorithm 5, Stage 4) by rotation on gfx950, FP64 matrix cores.
//
// For an offset class the dense real-packed M2L matrix factors as T = B Z A (built on the
// host, translations.cpp): A rotates the source multipoles into a frame where the offset
// points along +z, Z translates along z, which couples only equal orders m, and B rotates
// the local expansions back.  A and B are block diagonal by degree (blocks of 2n+1), Z
// block diagonal by order once its rows are grouped by (order, real/imaginary part) (blocks
// of p+1-m).  With 16 x 16 tiles, A and B have 44 nonzero tiles at p = 15 and Z 31 order
// blocks (76 matrix-core steps of 4 once their zero padding is skipped), against 256 tiles
// of the dense matrix: 428 against 1024 steps per 16 pairs.
// MFMA layout of v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register r of lane l holds D[l / 16 + 4 r][l % 16].
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "kernels.hpp"

namespace gq {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kRotXcds = 8;  // MI355X: 8 accelerator complex dies, one L2 each

// ------------------------------------------------------------------------------------
// M2L by rotation with the working matrix in registers: one wave per 16 pairs.
//
// The accumulator layout of v_mfma_f64_16x16x4f64 is also its operand layout for a chained
// product: register r of lane l holds D[l/16 + 4 r][l % 16], which is the B operand
// B[4 s + l/16][l % 16] of k-step s = r, and (read transposed) the A operand of the
// transposed product.  So a wave keeps its 16 pairs' (p+1)^2 x 16 working matrix in
// registers, 4 doubles per lane per row tile, and runs the products by A and B there:
//   stage 0  x = X          rows 16 t + l/16 + 4 r of pair l % 16, straight from HBM
//   stage 1  y = A x        A block diagonal by degree: each row tile needs <= 5 tiles of x
//   stage 2  y = Z y        through LDS: y is written out grouped by (order, re/im), each
//                           order block multiplied with its rows read as operands, and read
//                           back; in NH passes over groups of blocks to bound the LDS
//   stage 3  L^T += y^T B^T transposed, so that 16 lanes add to 16 consecutive
//                           coefficients of one pair's destination (or store to its slot)
// The sparsity of A and B and the row grouping of Z depend on p only and are compile-time
// tables, so every register index is static.  Each wave is independent: no barriers.
// ------------------------------------------------------------------------------------

// Compile-time shape of the factors at order P, with the LDS groups of Z's order blocks.
// Block b gathers the rows n^2 + b for n >= m = (b + 1) / 2 (block 0: m = 0, real parts;
// odd b: (m, real), even b > 0: (m, imaginary)), b_len = P + 1 - m rows.
template <int P, int NH>
struct RotW {
  static_assert(NH == 1 || NH == 2, "one or two LDS groups");
  static_assert(P <= 15, "an order block of Z spans more than one 16-row tile beyond p = 15");
  static constexpr int NP = (P + 1) * (P + 1);
  static constexpr int NTR = (NP + 15) / 16;
  static constexpr int NBLK = 2 * P + 1;
  int row_beg[NTR + 1] = {};
  int tile_c[NTR * NTR] = {};
  int tile_r[NTR * NTR] = {};
  int ntile = 0;
  int blen[NBLK] = {};
  int grp_beg[NH + 1] = {};  // blocks [grp_beg[h], grp_beg[h + 1]) form LDS group h
  int sbase[NBLK] = {};      // LDS row of block b's first row within its group
  int grp_rows[NH] = {};
  int rows_max = 0;
  int row_grp[NTR * 16] = {};   // group of row R (-1 beyond NP)
  int row_slot[NTR * 16] = {};  // LDS row of row R within its group
  constexpr RotW() {
    for (int r = 0; r < NTR; ++r) {
      row_beg[r] = ntile;
      for (int c = 0; c < NTR; ++c) {
        bool nz = false;
        for (int n = 0; n <= P && !nz; ++n) {
          const int lo = n * n, hi = (n + 1) * (n + 1) - 1;
          nz = lo <= 16 * r + 15 && hi >= 16 * r && lo <= 16 * c + 15 && hi >= 16 * c;
        }
        if (nz) {
          tile_r[ntile] = r;
          tile_c[ntile++] = c;
        }
      }
    }
    row_beg[NTR] = ntile;
    for (int b = 0; b < NBLK; ++b) blen[b] = P + 1 - (b + 1) / 2;
    // groups: contiguous block ranges, the split that minimizes the largest group
    grp_beg[0] = 0;
    grp_beg[NH] = NBLK;
    if (NH == 2) {
      int best = NP + 1, bs = 1;
      for (int s = 1; s < NBLK; ++s) {
        int a = 0;
        for (int b = 0; b < s; ++b) a += blen[b];
        const int m = a > NP - a ? a : NP - a;
        if (m < best) {
          best = m;
          bs = s;
        }
      }
      grp_beg[1] = bs;
    }
    for (int h = 0; h < NH; ++h) {
      int k = 0;
      for (int b = grp_beg[h]; b < grp_beg[h + 1]; ++b) {
        sbase[b] = k;
        k += blen[b];
      }
      grp_rows[h] = k;
      if (k > rows_max) rows_max = k;
    }
    for (int R = 0; R < NTR * 16; ++R) {
      row_grp[R] = -1;
      row_slot[R] = 0;
      if (R >= NP) continue;
      int n = 0;
      while ((n + 1) * (n + 1) <= R) ++n;
      const int b = R - n * n, m = (b + 1) / 2;
      for (int h = 0; h < NH; ++h)
        if (b >= grp_beg[h] && b < grp_beg[h + 1]) row_grp[R] = h;
      row_slot[R] = sbase[b] + n - m;
    }
  }
  // LDS rows of the four rows 16 t + 4 r + g (g = 0..3) held by register r of row tile t,
  // 16 bits each, 0xffff where the row is not in group h
  constexpr uint64_t pack(int t, int r, int h) const {
    uint64_t k = 0;
    for (int g = 0; g < 4; ++g) {
      const int R = 16 * t + 4 * r + g;
      const uint64_t v = row_grp[R] == h ? (uint64_t)row_slot[R] : 0xffffu;
      k |= v << (16 * g);
    }
    return k;
  }
};

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

constexpr int kRotwNH = 2;    // LDS groups of Z's order blocks
constexpr int kRotwD = 4;     // factor tiles in flight ahead of the one being multiplied

// One workgroup of kRotCols / 16 waves per tile of up to kRotCols pairs of one class; wave
// w takes pairs 16 w .. 16 w + 15, and the waves of a tile read the same factor tiles.
// 17 KB of LDS per wave at p = 15, so two workgroups of four waves fit on a CU.
constexpr int kRotwWaves = kRotCols / 16;
constexpr int kRotwOcc = 2;  // waves per SIMD the registers are sized for
template <int P, bool TO_SLOTS>
__global__ __launch_bounds__(64 * kRotwWaves, kRotwOcc) void k_m2l_rotw(
    const int* __restrict__ tile_cls, const int* __restrict__ tile_beg,
    const int* __restrict__ tile_cnt, const int* __restrict__ pair_src,
    const int* __restrict__ pair_dst, const double* __restrict__ RA,
    const double* __restrict__ RZ, const double* __restrict__ RB,
    const double* __restrict__ X, double* __restrict__ Y, int ntile, int per_xcd) {
  using S_t = RotW<P, kRotwNH>;
  constexpr S_t S{};
  constexpr int NP = S_t::NP, NTR = S_t::NTR, NBLK = S_t::NBLK;
  constexpr int TR = S.rows_max;  // a trash row: the target of the stores a lane skips
  __shared__ double Wsh[kRotwWaves][(TR + 1) * 16];
  const int t_id = per_xcd ? (blockIdx.x % kRotXcds) * per_xcd + blockIdx.x / kRotXcds
                           : blockIdx.x;
  if (t_id >= ntile) return;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  const int cls = tile_cls[t_id], cnt = tile_cnt[t_id] - 16 * wave;
  if (cnt <= 0) return;  // uniform over the wave
  const int beg = tile_beg[t_id] + 16 * wave;
  // factor tiles lane-major: lane l's operands of the four k-steps are 32 contiguous bytes
  const d2* A = reinterpret_cast<const d2*>(RA + (size_t)cls * S.ntile * 256 + 4 * l);
  const d2* Z = reinterpret_cast<const d2*>(RZ + (size_t)cls * NBLK * 256 + 4 * l);
  const d2* B = reinterpret_cast<const d2*>(RB + (size_t)cls * S.ntile * 256 + 4 * l);
  double* W = Wsh[wave];
  // stage 0: x[t][r] = X[row 16 t + 4 r + lk][pair li]
  const double* xs = X + (int64_t)pair_src[beg + (li < cnt ? li : 0)] * NP + lk;
  d4 x[NTR];
  static_for<0, NTR>([&](auto tt) {
    constexpr int t = decltype(tt)::value;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * t + 4 * r + lk;
      const double v = xs[min(16 * t + 4 * r, NP - 1 - lk)];  // in bounds for every lane
      x[t][r] = row < NP ? v : 0.0;
    }
  });
  // stage 1: y = A x over the nonzero tiles of A in row-tile order.  The operands of tile
  // j + D are loaded while tile j is multiplied (a ring of D tiles), and scheduling barriers
  // keep the compiler from moving the loads next to their use (stage 2 has none: there the
  // compiler overlaps one order block's LDS reads with the previous block's products).
  constexpr int NT = S.ntile, D = kRotwD;
  d2 ra[D][2];
  static_for<0, (D < NT ? D : NT)>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    ra[j][0] = A[j * 128];
    ra[j][1] = A[j * 128 + 1];
  });
  d4 y[NTR];
  d4 acc = d4{0, 0, 0, 0};
  static_for<0, NT>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    constexpr int t = S.tile_r[j], c = S.tile_c[j];
    const d2 a01 = ra[j % D][0], a23 = ra[j % D][1];
    if constexpr (j + D < NT) {
      ra[j % D][0] = A[(j + D) * 128];
      ra[j % D][1] = A[(j + D) * 128 + 1];
    }
    if constexpr (j == S.row_beg[t]) acc = d4{0, 0, 0, 0};
    acc = mfma16(a01[0], x[c][0], acc);
    acc = mfma16(a01[1], x[c][1], acc);
    acc = mfma16(a23[0], x[c][2], acc);
    acc = mfma16(a23[1], x[c][3], acc);
    if constexpr (j + 1 == S.row_beg[t + 1]) y[t] = acc;
    __builtin_amdgcn_sched_barrier(0);
  });
  // the first operands of stage 2, in flight while the LDS is written
  d2 rz[D][2];
  static_for<0, (D < NBLK ? D : NBLK)>([&](auto bb) {
    constexpr int b = decltype(bb)::value;
    rz[b][0] = Z[b * 128];
    rz[b][1] = Z[b * 128 + 1];
  });
  __builtin_amdgcn_sched_barrier(0);
  // stage 2: y = Z y, one LDS group of order blocks at a time
  static_for<0, kRotwNH>([&](auto hh) {
    constexpr int h = decltype(hh)::value;
    static_for<0, NTR>([&](auto tt) {
      constexpr int t = decltype(tt)::value;
      static_for<0, 4>([&](auto rr) {
        constexpr int r = decltype(rr)::value;
        constexpr uint64_t K = S.pack(t, r, h);
        if constexpr (K != 0xffffffffffffffffull) {
          const int slot = (int)((K >> (16 * lk)) & 0xffffu);
          W[min(slot, TR) * 16 + li] = y[t][r];
        }
      });
    });
    static_for<S.grp_beg[h], S.grp_beg[h + 1]>([&](auto bb) {
      constexpr int b = decltype(bb)::value;
      constexpr int len = S.blen[b], base = S.sbase[b];
      d4 acc = d4{0, 0, 0, 0};
      const d2 z01 = rz[b % D][0], z23 = rz[b % D][1];
      if constexpr (b + D < NBLK) {
        rz[b % D][0] = Z[(b + D) * 128];
        rz[b % D][1] = Z[(b + D) * 128 + 1];
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (4 * s < len) {  // beyond: padding of Z's block
          const int i = min(4 * s + lk, len - 1);  // padding rows: any row of the block
          acc = mfma16(s < 2 ? z01[s] : z23[s - 2], W[(base + i) * 16 + li], acc);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = lk + 4 * r;
        if (4 * r < len) W[(i < len ? base + i : TR) * 16 + li] = acc[r];
      }
    });
    static_for<0, NTR>([&](auto tt) {
      constexpr int t = decltype(tt)::value;
      static_for<0, 4>([&](auto rr) {
        constexpr int r = decltype(rr)::value;
        constexpr uint64_t K = S.pack(t, r, h);
        if constexpr (K != 0xffffffffffffffffull) {
          const int slot = (int)((K >> (16 * lk)) & 0xffffu);
          const double v = W[min(slot, TR) * 16 + li];
          y[t][r] = slot != 0xffff ? v : y[t][r];
        }
      });
    });
  });
  // stage 3: L^T += y^T B^T; register r of lane l: pair lk + 4 r, row 16 t + li.  Its
  // first operands are loaded only now: in flight during stage 2 they cost spills.
  d2 rb[D][2];
  static_for<0, (D < NT ? D : NT)>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    rb[j][0] = B[j * 128];
    rb[j][1] = B[j * 128 + 1];
  });
  int dst[4];
  bool ok[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    ok[r] = lk + 4 * r < cnt;
    // a lane past the tile's end adds zero to the first pair's destination instead
    dst[r] = TO_SLOTS ? beg + lk + 4 * r : pair_dst[beg + (ok[r] ? lk + 4 * r : 0)];
  }
  static_for<0, NT>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    constexpr int t = S.tile_r[j], c = S.tile_c[j];
    const d2 b01 = rb[j % D][0], b23 = rb[j % D][1];
    if constexpr (j + D < NT) {
      rb[j % D][0] = B[(j + D) * 128];
      rb[j % D][1] = B[(j + D) * 128 + 1];
    }
    if constexpr (j == S.row_beg[t]) acc = d4{0, 0, 0, 0};
    acc = mfma16(y[c][0], b01[0], acc);
    acc = mfma16(y[c][1], b01[1], acc);
    acc = mfma16(y[c][2], b23[0], acc);
    acc = mfma16(y[c][3], b23[1], acc);
    if constexpr (j + 1 == S.row_beg[t + 1]) {
      const int row = 16 * t + li;
      if constexpr (TO_SLOTS) {
        if (row < NP) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (ok[r]) Y[(int64_t)dst[r] * NP + row] = acc[r];
        }
      } else {
        // branch-free: a lane beyond the rows or pairs adds zero to a row that exists
        const int rc = min(row, NP - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          unsafeAtomicAdd(&Y[(int64_t)dst[r] * NP + rc], ok[r] && row < NP ? acc[r] : 0.0);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  });
}

using RotwFn = void (*)(const int*, const int*, const int*, const int*, const int*,
                        const double*, const double*, const double*, const double*, double*,
                        int, int);

template <bool TO_SLOTS, int... Ps>
RotwFn rotw_pick(int p, std::integer_sequence<int, Ps...>) {
  RotwFn f = nullptr;
  ((p == Ps ? (f = k_m2l_rotw<Ps, TO_SLOTS>) : f), ...);
  return f;
}

template <int... Ps>
int rotw_tiles(int p, std::integer_sequence<int, Ps...>) {
  int n = -1;
  ((p == Ps ? (n = RotW<Ps, kRotwNH>{}.ntile) : n), ...);
  return n;
}

}  // namespace

int m2l_rot_tiles(int p) { return rotw_tiles(p, std::make_integer_sequence<int, 16>{}); }

void launch_m2l_rot(hipStream_t s, int np, int ntile, const int* tile_cls, const int* tile_beg,
                    const int* tile_cnt, const int* pair_src, const int* pair_dst,
                    const RotMats& R, const double* X, double* Y, bool xcd_order,
                    bool to_slots) {
  if (ntile <= 0) return;
  const int per_xcd = xcd_order ? (ntile + kRotXcds - 1) / kRotXcds : 0;
  const dim3 grid(xcd_order ? per_xcd * kRotXcds : ntile);
  int p = 0;
  while ((p + 1) * (p + 1) < np) ++p;
  auto seq = std::make_integer_sequence<int, 16>{};  // p = 0 .. 15
  RotwFn k = nullptr;
  if (to_slots)
    k = rotw_pick<true>(p, seq);
  else
    k = rotw_pick<false>(p, seq);
  if (!k) return;  // p > 15 is rejected at plan creation
  k<<<grid, 64 * kRotwWaves, 0, s>>>(tile_cls, tile_beg, tile_cnt, pair_src, pair_dst, R.A, R.Z,
                                     R.B, X, Y, ntile, per_xcd);
}

}  // namespace gq
