// GIGAQBX FMM device kernels for gfx950 (CDNA4, 64-wide wavefronts), FP64 throughout.
//
// Expansion conventions (see translations.cpp for the derivations):
//   * solid harmonics with the Condon-Shortley phase; J_n^m := conj(I_n^m)
//   * multipoles and box locals are scaled by the box half-width a:
//       mu~_n^m = a^-n sum q R_n^m(s - x_b),   l~_n^m = a^(n+1) sum q J_n^m(s - x_b)
//   * QBX locals are unscaled: l_n^m(c) = sum q J_n^m(s - c), potential
//       phi(t) = (1/4pi) sum_n [l_n^0 R_n^0 + 2 sum_{m>0} Re(l_n^m R_n^m)](t - c)
//   * coefficient vectors are real-packed per degree n: offset n^2,
//       [Re c_n^0, Re c_n^1, Im c_n^1, ..., Re c_n^n, Im c_n^n]
//   * QBX locals are stored coefficient-major, Lq[k * nctr + c], so consecutive centers
//     (consecutive lanes) touch consecutive addresses.
//   * double layer: the source factor is n_s . grad_s, applied with the ladders
//       d_z R_n^m = R_{n-1}^m, (d_x + i d_y) R_n^m = R_{n-1}^{m+1}, (d_x - i d_y) R_n^m = -R_{n-1}^{m-1}
//       d_z I_n^m = -I_{n+1}^m, (d_x + i d_y) I_n^m = I_{n+1}^{m+1}, (d_x - i d_y) I_n^m = -I_{n+1}^{m-1}
//     and n.grad = n_z d_z + (n_x - i n_y)/2 (d_x + i d_y) + (n_x + i n_y)/2 (d_x - i d_y).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace gq {

namespace {

__device__ __forceinline__ int pkre(int n, int m) { return n * n + (m ? 2 * m - 1 : 0); }
__device__ __forceinline__ int pkim(int n, int m) { return n * n + 2 * m; }
__host__ __device__ constexpr int cpk_re(int n, int m) { return n * n + (m ? 2 * m - 1 : 0); }
__host__ __device__ constexpr int cpk_im(int n, int m) { return n * n + 2 * m; }
__device__ __forceinline__ int cidx(int n, int m) { return n * n + n + m; }

constexpr double kInv4Pi = 0.07957747154594767;  // 1/(4 pi)

// ------------------------------------------------------------------------------------
// simple elementwise kernels
// ------------------------------------------------------------------------------------

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_strength(int64_t n, const int64_t* __restrict__ order,
                           const double* __restrict__ w, const double* __restrict__ dens,
                           double* __restrict__ q) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) q[i] = w[i] * dens[order[i]];
}

// ------------------------------------------------------------------------------------
// P2M and P2L
// ------------------------------------------------------------------------------------

constexpr int kInvTab = kPmax + 3;

__device__ __forceinline__ void fill_invtab(double* tab) {
  // tab[n * kInvTab + m] = 1/(n^2 - m^2) for n > m
  for (int i = threadIdx.x; i < kInvTab * kInvTab; i += blockDim.x) {
    int n = i / kInvTab, m = i % kInvTab;
    tab[i] = n > m ? 1.0 / (double)(n * n - m * m) : 0.0;
  }
}

// ------------------------------------------------------------------------------------
// Batched dense translation on the FP64 matrix cores: for each tile (up to kTileCols = 64
// pairs of one matrix class) Y[dst_c] += T X[src_c], T column-major np x np.
// v_mfma_f64_16x16x4f64: D(16x16) += A(16x4) B(4x16); lane l supplies A[l%16][l/16] and
// B[l/16][l%16] and holds D[l/16 + 4r][l%16], r = 0..3 (register r, lane l).
// The product is formed transposed, Y^T = X^T T^T (inputs as the A operand, matrix as the
// B operand), so that the 16 lanes sharing a register hold 16 consecutive output
// coefficients of one destination and its atomic adds coalesce.  A block (4 waves) walks the
// matrix rows in rounds of 4 RB row-blocks; wave w owns row-blocks w, w+4, ... of the round
// and all column blocks of the tile, so each matrix element is read once per tile.  RB = 4
// (16 row blocks, p <= 15: one round); for p = 16..20 (19 to 28 row blocks) RB = 7 makes it
// one round too, instead of a second, partly idle round that stages the inputs again.
// The input expansions are staged in LDS in chunks of kKc coefficients; outputs are added
// atomically (several classes can target one box), or stored to per-pair slots (KIND 3).
// XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs, each with its
// own L2, and tiles are sorted by class; block i therefore takes tile
// (i % 8) * per_xcd + i / 8, so each XCD walks one contiguous range of classes and reads
// each class matrix into its L2 once.
// ------------------------------------------------------------------------------------

typedef double d4_t __attribute__((ext_vector_type(4)));
constexpr int kKc = kTransKc;
constexpr int kXcds = 8;            // MI355X: 8 accelerator complex dies, one L2 each
constexpr int kPf64 = 2;            // K-steps of matrix prefetch, FP64 kernel
constexpr int kPf32 = 4;            // K-steps of matrix prefetch, FP32 kernel

// KIND (0 M2M, 1 L2L, 2 M2L) only names the instantiation, so that profiles tell the
// three uses apart; the code is the same.  KIND 3 is any of them with each pair's result
// stored to its own slot Y[pair position] instead of added into Y[dst] (deterministic
// plans, summed afterwards by k_slot_sum).
template <int KIND, int CB, int RB = 4>
__global__ __launch_bounds__(256) void k_translate(int np, const int* __restrict__ tile_cls,
                                                   const int* __restrict__ tile_beg,
                                                   const int* __restrict__ tile_cnt,
                                                   const int* __restrict__ pair_src,
                                                   const int* __restrict__ pair_dst,
                                                   const double* __restrict__ T,
                                                   const double* __restrict__ X,
                                                   double* __restrict__ Y, int ntile,
                                                   int per_xcd) {
  constexpr bool to_slots = KIND == 3;
  constexpr int kXs = 16 * CB + 1;  // padded LDS row
  __shared__ double xs[2][kKc * kXs];  // double-buffered [k][col]
  const int t = per_xcd ? (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds)
                        : (int)blockIdx.x;
  if (t >= ntile) return;
  const int cls = tile_cls[t], beg = tile_beg[t], cnt = tile_cnt[t];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ld = trans_ld(np), kd = trans_kd(np);
  const double* Tc = T + (int64_t)cls * ld * kd;
  const int nrb = ld >> 4;
  // staging of one K-chunk of the input columns: lane -> k, wave w -> columns w + 4u, so
  // the column offsets are wave-uniform and live in scalar registers
  static_assert(kKc == 64, "staging maps one lane to one k of a chunk");
  constexpr int kStage = 16 * CB / 4;
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  int64_t src_off[kStage];
#pragma unroll
  for (int u = 0; u < kStage; ++u) {
    const int col = wave_u + 4 * u;
    src_off[u] = col < cnt ? (int64_t)pair_src[beg + col] * np : -1;
  }
  // the next chunk is fetched in two halves of kStage / 2 columns per wave
  constexpr int kHalf = kStage / 2;
  auto load_half = [&](int kc, int h, double (&xr)[kHalf]) {
    const int k = kc + lane;
#pragma unroll
    for (int u = 0; u < kHalf; ++u) {
      const int64_t o = src_off[h * kHalf + u];
      xr[u] = (o >= 0 && k < np) ? X[o + k] : 0.0;
    }
  };
  auto store_half = [&](double* xb, int h, const double (&xr)[kHalf]) {
#pragma unroll
    for (int u = 0; u < kHalf; ++u) xb[lane * kXs + wave_u + 4 * (h * kHalf + u)] = xr[u];
  };
  // matrices are zero-padded to ld rows and kd columns; row blocks past the end and
  // prefetches past the last column are clamped to valid addresses (and never used)
  auto load_a = [&](int r0, int k, double (&a)[RB]) {
    const double* col = Tc + (int64_t)min(k, kd - 1) * ld + li;
#pragma unroll
    for (int i = 0; i < RB; ++i) a[i] = col[min(r0 + wave_u + 4 * i, nrb - 1) * 16];
  };
  for (int r0 = 0; r0 < nrb; r0 += 4 * RB) {
    d4_t acc[RB][CB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[i][cb] = (d4_t){0.0, 0.0, 0.0, 0.0};
    double xr[kHalf];
    __syncthreads();  // the previous row pass has finished reading both buffers
    load_half(0, 0, xr);
    store_half(xs[0], 0, xr);
    load_half(0, 1, xr);
    store_half(xs[0], 1, xr);
    // matrix fragments of the next kPf64 K-steps are in flight while a step's MFMAs run
    double a[kPf64][RB];
#pragma unroll
    for (int d = 0; d < kPf64; ++d) load_a(r0, 4 * d + lk, a[d]);
    __syncthreads();
    int cur = 0;
    auto steps = [&](int kc, int g0, int g1) {
      const double* xb = xs[cur];
#pragma unroll 1
      for (int g = g0; g < g1; g += kPf64) {
#pragma unroll
        for (int d = 0; d < kPf64; ++d) {
          const int st = g + d;
          double b[4];
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) b[cb] = xb[(4 * st + lk) * kXs + cb * 16 + li];
#pragma unroll
          for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
              acc[i][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[cb], a[d][i], acc[i][cb], 0, 0, 0);
          load_a(r0, kc + 4 * (st + kPf64) + lk, a[d]);
        }
      }
    };
    // all kKc/4 steps of every chunk (past np both operands are zero); the next chunk is
    // fetched into the other buffer meanwhile
    for (int kc = 0; kc < np; kc += kKc, cur ^= 1) {
      const bool more = kc + kKc < np;
      if (more) load_half(kc + kKc, 0, xr);
      steps(kc, 0, kKc / 8);
      if (more) {
        store_half(xs[cur ^ 1], 0, xr);
        load_half(kc + kKc, 1, xr);
      }
      steps(kc, kKc / 8, kKc / 4);
      if (more) store_half(xs[cur ^ 1], 1, xr);
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int rb = r0 + wave + 4 * i;
      if (rb >= nrb) continue;
      const int row = rb * 16 + li;
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // transposed product: register r of lane l holds (pair l/16 + 4r, row l%16), so
          // 16 lanes add 16 consecutive coefficients of one destination
          const int col = cb * 16 + lk + 4 * r;
          if (col < cnt && row < np) {
            if constexpr (to_slots)
              Y[(int64_t)(beg + col) * np + row] = acc[i][cb][r];
            else
              unsafeAtomicAdd(&Y[(int64_t)pair_dst[beg + col] * np + row], acc[i][cb][r]);
          }
        }
    }
  }
}

// FP32 matrix-core translations (v_mfma_f32_16x16x4f32).  Same tiling as k_translate.
// The matrices are balanced: T^ = diag(1 / s_out) T diag(1 / s_in), with s = N_n^m or
// 1 / N_n^m (N_n^m = sqrt((n+m)! (n-m)!)) by the kind of expansion, so that inputs
// x^ = s_in x, outputs and entries are O(1) at every order up to p = 20; the kernel scales
// each input as it is staged and each output before it is added to the FP64 expansions.
// T^ is stored as the FP32 pair T_hi + T_lo and each staged input as x_hi + x_lo.
//   MODE 0 (uncorrected): T_hi x_hi over every column, FP32 accumulation.
//   MODE 1 (split): the first kLead columns (degrees n <= 3, which carry most of the
//     magnitude of every output, since the expansions decay with the degree) are contracted
//     exactly on the FP64 matrix cores; over the rest each K-step forms
//     T_hi x_lo + T_lo x_hi + T_hi x_hi from zero on the FP32 matrix cores and adds it into
//     FP64 registers, so only the rounding inside one step remains.
//   MODE 2 (leading degrees): the first kLead columns in FP64 as in MODE 1, the rest
//     T_hi x_hi with FP32 accumulation.
typedef float f4_t __attribute__((ext_vector_type(4)));
constexpr int kLead = kLeadCols;  // leading packed coefficients contracted in FP64 (MODE 1, 2)

template <int KIND, int CB, int MODE, int RB = 4>
__global__ __launch_bounds__(256, MODE == 2 && CB == 2 && RB == 4 ? 4 : 1) void k_translate32(int np, const int* __restrict__ tile_cls,
                                                     const int* __restrict__ tile_beg,
                                                     const int* __restrict__ tile_cnt,
                                                     const int* __restrict__ pair_src,
                                                     const int* __restrict__ pair_dst,
                                                     const float* __restrict__ Thi,
                                                     const float* __restrict__ Tlo,
                                                     const double* __restrict__ Tlead,
                                                     const double* __restrict__ s_in,
                                                     const double* __restrict__ s_out,
                                                     const double* __restrict__ X,
                                                     double* __restrict__ Y, int ntile,
                                                     int per_xcd) {
  constexpr bool to_slots = KIND == 3;
  constexpr bool kLeadOn = MODE != 0;
  constexpr int kXs = 16 * CB + 1;  // padded LDS row
  __shared__ float2 xs[2][kKc * kXs];  // double-buffered [k][col] = (hi, lo)
  __shared__ double xl64[kLeadOn ? kLead * kXs : 1];  // leading inputs in FP64 [k][col]
  const int t = per_xcd ? (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds)
                        : (int)blockIdx.x;
  if (t >= ntile) return;
  const int cls = tile_cls[t], beg = tile_beg[t], cnt = tile_cnt[t];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ld = trans_ld(np), kd = trans_kd(np);
  const int64_t moff = (int64_t)cls * ld * kd;
  const int nrb = ld >> 4;
  static_assert(kKc == 64, "staging maps one lane to one k of a chunk");
  // matrix prefetch depth in K-steps: the split mode holds FP64 accumulators, so it
  // prefetches less to keep two waves per SIMD
  constexpr int kPf = MODE == 1 ? 2 : kPf32;
  static_assert(kLead % (4 * kPf) == 0 && kLead / 4 <= kKc / 8,
                "the FP32 steps of the first chunk start at a prefetch group of its first half");
  constexpr int kStage = 16 * CB / 4;
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  int64_t src_off[kStage];
#pragma unroll
  for (int u = 0; u < kStage; ++u) {
    const int col = wave_u + 4 * u;
    src_off[u] = col < cnt ? (int64_t)pair_src[beg + col] * np : -1;
  }
  constexpr int kHalf = kStage / 2;
  // inputs of column k are scaled by s_in[k] as they are loaded (zero past np)
  auto load_half = [&](int kc, int h, double (&xr)[kHalf]) {
    const int k = kc + lane;
    const double sc = k < np ? s_in[k] : 0.0;
#pragma unroll
    for (int u = 0; u < kHalf; ++u) {
      const int64_t o = src_off[h * kHalf + u];
      xr[u] = (o >= 0 && k < np) ? X[o + k] * sc : 0.0;
    }
  };
  auto store_half = [&](float2* xb, int h, const double (&xr)[kHalf], bool lead) {
#pragma unroll
    for (int u = 0; u < kHalf; ++u) {
      const int col = wave_u + 4 * (h * kHalf + u);
      const float hi = (float)xr[u];
      const float lo = (float)(xr[u] - (double)hi);
      xb[lane * kXs + col] = make_float2(hi, lo);
      if (kLeadOn && lead && lane < kLead) xl64[lane * kXs + col] = xr[u];
    }
  };
  auto load_a = [&](int r0, int k, float (&ah)[RB], float (&al)[RB]) {
    const int64_t col = moff + (int64_t)min(k, kd - 1) * ld + li;
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int64_t off = col + min(r0 + wave_u + 4 * i, nrb - 1) * 16;
      ah[i] = Thi[off];
      al[i] = MODE == 1 ? Tlo[off] : 0.0f;
    }
  };
  constexpr int k0 = kLeadOn ? kLead : 0;  // first column on the FP32 matrix cores
  for (int r0 = 0; r0 < nrb; r0 += 4 * RB) {
    f4_t acc[RB][CB];      // FP32 accumulation (MODE 0, 2)
    double acc64[RB][CB][MODE == 1 ? 4 : 1];  // FP64 accumulation of the steps (MODE 1)
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        acc[i][cb] = (f4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < (MODE == 1 ? 4 : 1); ++r) acc64[i][cb][r] = 0.0;
      }
    double xr[kHalf];
    __syncthreads();  // the previous row pass has finished reading every buffer
    load_half(0, 0, xr);
    store_half(xs[0], 0, xr, r0 == 0);
    load_half(0, 1, xr);
    store_half(xs[0], 1, xr, r0 == 0);
    float ah[kPf][RB], al[kPf][RB];
#pragma unroll
    for (int d = 0; d < kPf; ++d) load_a(r0, k0 + 4 * d + lk, ah[d], al[d]);
    __syncthreads();
    int cur = 0;
    auto steps = [&](int kc, int g0, int g1) {
      const float2* xb = xs[cur];
#pragma unroll 1
      for (int g = g0; g < g1; g += kPf) {
#pragma unroll
        for (int d = 0; d < kPf; ++d) {
          const int st = g + d;
          float2 b[4];
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) b[cb] = xb[(4 * st + lk) * kXs + cb * 16 + li];
#pragma unroll
          for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
              if (MODE == 1) {
                f4_t c = (f4_t){0.f, 0.f, 0.f, 0.f};
                c = __builtin_amdgcn_mfma_f32_16x16x4f32(b[cb].y, ah[d][i], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x4f32(b[cb].x, al[d][i], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x4f32(b[cb].x, ah[d][i], c, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) acc64[i][cb][r] += (double)c[r];
              } else {
                acc[i][cb] =
                    __builtin_amdgcn_mfma_f32_16x16x4f32(b[cb].x, ah[d][i], acc[i][cb], 0, 0, 0);
              }
            }
          load_a(r0, kc + 4 * (st + kPf) + lk, ah[d], al[d]);
        }
      }
    };
    for (int kc = 0; kc < np; kc += kKc, cur ^= 1) {
      const bool more = kc + kKc < np;
      if (more) load_half(kc + kKc, 0, xr);
      steps(kc, kc == 0 ? k0 / 4 : 0, kKc / 8);
      if (more) {
        store_half(xs[cur ^ 1], 0, xr, false);
        load_half(kc + kKc, 1, xr);
      }
      steps(kc, kKc / 8, kKc / 4);
      if (more) store_half(xs[cur ^ 1], 1, xr, false);
      __syncthreads();
    }
    // The leading columns on the FP64 matrix cores, one row block at a time, starting from
    // the FP32 part's result.  Inputs are fed in the pair order pi(a + 4b) = 4a + b, so
    // that register r of lane l holds pair 4 (l/16) + r, the place of the FP32
    // accumulator layout: (pair 4 (l/16) + r, row l%16) of the transposed product.
    const int pli = 4 * (li & 3) + (li >> 2);
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int rb = r0 + wave_u + 4 * i;
      if (rb >= nrb) continue;  // wave-uniform
      const int row = rb * 16 + li;
      const double so = row < np ? s_out[row] : 0.0;
      double a[kLeadOn ? kLead / 4 : 1];
      if (kLeadOn) {
#pragma unroll
        for (int st = 0; st < kLead / 4; ++st)
          a[st] = Tlead[((int64_t)cls * kLead + 4 * st + lk) * ld + rb * 16 + li];
      }
      d4_t v[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          v[cb][r] = MODE == 1 ? acc64[i][cb][MODE == 1 ? r : 0] : (double)acc[i][cb][r];
      if (kLeadOn) {
#pragma unroll
        for (int st = 0; st < kLead / 4; ++st)
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            v[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                xl64[(4 * st + lk) * kXs + cb * 16 + pli], a[st], v[cb], 0, 0, 0);
      }
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = cb * 16 + 4 * lk + r;
          if (col < cnt && row < np) {
            if constexpr (to_slots)
              Y[(int64_t)(beg + col) * np + row] = v[cb][r] * so;
            else
              unsafeAtomicAdd(&Y[(int64_t)pair_dst[beg + col] * np + row], v[cb][r] * so);
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------------------------
// P2QBXL: one thread per (center, source slice); sources staged through LDS.
// ------------------------------------------------------------------------------------

// 1/sqrt(x) for x > 0: hardware estimate refined by two Newton-Raphson steps
// y <- y (3 - x y^2) / 2, each of which squares the relative error.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x, y * y, 1.5);
  y = y * fma(-0.5 * x, y * y, 1.5);
  return y;
}

template <int Q>
__device__ __forceinline__ void p2qbxl_single(double dx, double dy, double dz, double qq,
                                              double (&acc)[(Q + 1) * (Q + 1)]) {
  // l_n^m += q J_n^m(s - c), J = conj(I): columns of fixed order m, increasing degree n
  const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
  const double ir = rsqrt_nr(r2);
  const double ir2 = ir * ir;
  const double zr = dz * ir2;
  double zk[Q + 2];  // (2k - 1) z / r^2
#pragma unroll
  for (int k = 1; k <= Q + 1; ++k) zk[k] = (2.0 * k - 1.0) * zr;
  const double xr = dx * ir2, yr = dy * ir2;
  double dr = qq * ir, di = 0.0;
#pragma unroll
  for (int m = 0; m <= Q; ++m) {
    if (m > 0) {  // J_m^m = -(2m-1)(x - i y)/r^2 J_{m-1}^{m-1}
      const double fr = -(2.0 * m - 1.0) * xr, fi = (2.0 * m - 1.0) * yr;
      const double nr = fma(dr, fr, -di * fi), ni = fma(dr, fi, di * fr);
      dr = nr;
      di = ni;
    }
    acc[cpk_re(m, m)] += dr;
    if (m) acc[cpk_im(m, m)] += di;
    double p1r = dr, p1i = di, p2r = 0.0, p2i = 0.0;
#pragma unroll
    for (int n = m + 1; n <= Q; ++n) {
      const double c2 = (double)((n - 1) * (n - 1) - m * m) * ir2;
      const double cr = fma(zk[n], p1r, -c2 * p2r);
      acc[cpk_re(n, m)] += cr;
      p2r = p1r;
      p1r = cr;
      if (m) {
        const double ci = fma(zk[n], p1i, -c2 * p2i);
        acc[cpk_im(n, m)] += ci;
        p2i = p1i;
        p1i = ci;
      }
    }
  }
}

template <int Q, int ND>
__device__ __forceinline__ void p2qbxl_double(double dx, double dy, double dz,
                                              const double (&qz)[ND], const double (&qxh)[ND],
                                              const double (&qyh)[ND],
                                              double (&acc)[ND][(Q + 1) * (Q + 1)]) {
  // l_n^m += -qz J_{n+1}^m + qa J_{n+1}^{m+1} - conj(qa) J_{n+1}^{m-1}, qa = (qx + i qy)/2,
  // scattered from each J_N^M (N = n+1 <= Q+1) into the outputs it feeds, as FMA chains;
  // the ND densities share the generated J.
  const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
  const double ir = rsqrt_nr(r2);
  const double ir2 = ir * ir;
  const double zr = dz * ir2;
  double zk[Q + 3];
#pragma unroll
  for (int k = 1; k <= Q + 1; ++k) zk[k] = (2.0 * k - 1.0) * zr;
  const double xr = dx * ir2, yr = dy * ir2;
  double dr = ir, di = 0.0;
#pragma unroll
  for (int M = 0; M <= Q + 1; ++M) {
    if (M > 0) {
      const double fr = -(2.0 * M - 1.0) * xr, fi = (2.0 * M - 1.0) * yr;
      const double nr = fma(dr, fr, -di * fi), ni = fma(dr, fi, di * fr);
      dr = nr;
      di = ni;
    }
    double p1r = 0.0, p1i = 0.0, p2r = 0.0, p2i = 0.0;
#pragma unroll
    for (int N = M; N <= Q + 1; ++N) {
      double jr, ji;
      if (N == M) {
        jr = dr;
        ji = di;
      } else {
        const double c2 = (double)((N - 1) * (N - 1) - M * M) * ir2;
        jr = fma(zk[N], p1r, -c2 * p2r);
        ji = M ? fma(zk[N], p1i, -c2 * p2i) : 0.0;
      }
      if (N >= 1) {
        const int n = N - 1;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          double* a = acc[d];
          if (M <= n) {  // -qz J_N^M -> l_n^M
            a[cpk_re(n, M)] = fma(-qz[d], jr, a[cpk_re(n, M)]);
            if (M) a[cpk_im(n, M)] = fma(-qz[d], ji, a[cpk_im(n, M)]);
          }
          if (M == 1) {  // qa J^1 + conj(qa J^1) -> l_n^0
            a[cpk_re(n, 0)] = fma(2.0 * qxh[d], jr, fma(-2.0 * qyh[d], ji, a[cpk_re(n, 0)]));
          } else if (M >= 2 && M - 1 <= n) {  // qa J_N^M -> l_n^{M-1}
            a[cpk_re(n, M - 1)] = fma(qxh[d], jr, fma(-qyh[d], ji, a[cpk_re(n, M - 1)]));
            a[cpk_im(n, M - 1)] = fma(qxh[d], ji, fma(qyh[d], jr, a[cpk_im(n, M - 1)]));
          }
          if (M + 1 <= n) {  // -conj(qa) J_N^M -> l_n^{M+1}
            a[cpk_re(n, M + 1)] = fma(-qxh[d], jr, fma(-qyh[d], ji, a[cpk_re(n, M + 1)]));
            a[cpk_im(n, M + 1)] = fma(-qxh[d], ji, fma(qyh[d], jr, a[cpk_im(n, M + 1)]));
          }
        }
      }
      if (N == M) {
        p1r = jr;
        p1i = ji;
      } else {
        p2r = p1r;
        p2i = p1i;
        p1r = jr;
        p1i = ji;
      }
    }
  }
}

// One 64-lane wavefront per item of at most 64 centers of one target box.  With nc
// centers the wave splits into S = 64 / nc source slices (lane = center + nc * slice), so
// at least 60 of the 64 lanes are busy for every nc.  The box's near sources (U, W-close,
// X-close, flattened) are staged through LDS 64 at a time, the next batch being fetched
// into registers while the current one is evaluated; slices are summed through LDS.
// ND densities (1 or 2; 2 for the double layer only) share each pair's solid harmonics:
// density d reads its strengths at qs + d qstride and adds into Lq + d lqstride.
template <int Q, int KERN, int ND>
__global__ __launch_bounds__(64) void k_p2qbxl(const int* __restrict__ it_box,
                                               const int* __restrict__ it_c0,
                                               const int* __restrict__ it_nc,
                                               const int64_t* __restrict__ near_ptr,
                                               const int* __restrict__ near_idx,
                                               SrcSoA src, const double* __restrict__ qs,
                                               int64_t qstride,
                                               const double* __restrict__ cx,
                                               const double* __restrict__ cy,
                                               const double* __restrict__ cz,
                                               double* __restrict__ Lq, int64_t nctr,
                                               int64_t lqstride) {
  static_assert(ND == 1 || KERN != 0, "the single layer evaluates one density per pass");
  constexpr int NQ = (Q + 1) * (Q + 1);
  constexpr int NW = KERN ? 3 : 1;  // strength factors per source and density
  constexpr int NF = 3 + NW * ND;
  constexpr int kRed = 8;
  __shared__ double ss[NF * 64];
  __shared__ double red[kRed * 64];
  const int item = blockIdx.x;
  const int b = it_box[item];
  const int c0 = it_c0[item], nc = it_nc[item];
  const int S = 64 / nc;
  const int lane = threadIdx.x;
  const int ci = lane % nc, sl = lane / nc;
  const bool active = sl < S;
  const int64_t c = (int64_t)c0 + ci;
  const double xc = cx[c], yc = cy[c], zc = cz[c];
  double acc[ND][NQ];
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int i = 0; i < NQ; ++i) acc[d][i] = 0.0;
  const int64_t fb = near_ptr[b], fe = near_ptr[b + 1];
  double pf[NF];
  auto fetch = [&](int64_t f0) {
    const int64_t f = f0 + lane;
    if (f < fe) {
      const int64_t sidx = near_idx[f];
      pf[0] = src.x[sidx];
      pf[1] = src.y[sidx];
      pf[2] = src.z[sidx];
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        const double qq = qs[d * qstride + sidx];
        if constexpr (KERN != 0) {
          pf[3 + 3 * d] = qq * src.nz[sidx];
          pf[4 + 3 * d] = 0.5 * qq * src.nx[sidx];
          pf[5 + 3 * d] = 0.5 * qq * src.ny[sidx];
        } else {
          pf[3 + d] = qq;
        }
      }
    }
  };
  fetch(fb);
  for (int64_t f0 = fb; f0 < fe; f0 += 64) {
    const int n = (int)min((int64_t)64, fe - f0);
    __syncthreads();
    if (lane < n) {
#pragma unroll
      for (int v = 0; v < NF; ++v) ss[v * 64 + lane] = pf[v];
    }
    __syncthreads();
    if (f0 + 64 < fe) fetch(f0 + 64);
    if (active) {
      for (int j = sl; j < n; j += S) {
        const double dx = ss[j] - xc, dy = ss[64 + j] - yc, dz = ss[128 + j] - zc;
        if constexpr (KERN != 0) {
          double qz[ND], qxh[ND], qyh[ND];
#pragma unroll
          for (int d = 0; d < ND; ++d) {
            qz[d] = ss[(3 + 3 * d) * 64 + j];
            qxh[d] = ss[(4 + 3 * d) * 64 + j];
            qyh[d] = ss[(5 + 3 * d) * 64 + j];
          }
          p2qbxl_double<Q, ND>(dx, dy, dz, qz, qxh, qyh, acc);
        } else {
          p2qbxl_single<Q>(dx, dy, dz, ss[192 + j], acc[0]);
        }
      }
    }
  }
  if (S == 1) {
    if (active)
#pragma unroll
      for (int d = 0; d < ND; ++d)
#pragma unroll
        for (int i = 0; i < NQ; ++i) Lq[d * lqstride + (int64_t)i * nctr + c] += acc[d][i];
    return;
  }
  // sum the S slices of each center through LDS, kRed coefficients at a time
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int base = 0; base < NQ; base += kRed) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kRed; ++k)
        if (base + k < NQ) red[k * 64 + lane] = active ? acc[d][base + k] : 0.0;
      __syncthreads();
      if (sl == 0) {
        for (int k = 0; k < kRed && base + k < NQ; ++k) {
          double sum = 0.0;
          for (int t = 0; t < S; ++t) sum += red[k * 64 + t * nc + ci];
          Lq[d * lqstride + (int64_t)(base + k) * nctr + c] += sum;
        }
      }
    }
}

// ------------------------------------------------------------------------------------
// M2QBXL and L2QBXL: one lane per center in each wave of an item.  The box expansion is
// rescaled to its physical form and expanded to all signed orders in a zero-padded LDS table
// of complex pairs; the solid harmonics of the center offset are generated column by column
// (fixed order M, increasing degree N; the orders are dealt to the waves) and each value is
// scattered into the order-Q outputs it feeds.  Table addresses are a per-(M, N) base plus a
// compile-time offset per output (j, k); entries outside |m| <= n <= P read zeros, so the
// inner body is branch-free apart from one uniform degree check per j.
// ------------------------------------------------------------------------------------

// M2QBXL: l_j^k(c) = sum_{n,m} [(-1)^n mu_n^m] [(-1)^N J_N^{m+k}(c - x_d)], N = n + j
// (mu unscaled multipole, J = conj(I)); padded table rows n + Q, columns m + MOFF.
template <int Q, int PT>
struct M2qTab {
  static constexpr int MOFF = PT + 2 * Q;
  static constexpr int W = 2 * PT + 3 * Q + 1;
  static constexpr int ROWS = PT + 2 * Q + 1;
};

// L2QBXL: l_j^k(c) = sum_{n,m} l_n^m R_{n-j}^{m-k}(c - x_b) (l unscaled box local);
// padded table rows n, columns m + MOFF.
template <int Q>
struct L2qTab {
  static constexpr int MOFF = kPmax;
  static constexpr int W = 2 * kPmax + Q + 1;
  static constexpr int ROWS = kPmax + Q + 1;
};

// Fill the nonzero part (n <= P, |m| <= n) of a padded table from a real-packed scaled
// expansion e, multiplying degree n by scale(n).  c^-m = (-1)^m conj(c^m).
template <class F>
__device__ __forceinline__ void fill_padded(const double* __restrict__ e, int P, double2* tab,
                                            int row0, int W, int moff, F scale) {
  const int np = (P + 1) * (P + 1);
  double* t = reinterpret_cast<double*>(tab);
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    int n = (int)sqrt((double)i);
    while (n * n > i) --n;
    while ((n + 1) * (n + 1) <= i) ++n;
    const int off = i - n * n;
    const double v = e[i] * scale(n);
    const int row = (row0 + n) * W + moff;
    if (off == 0) {
      t[2 * row] = v;
      t[2 * row + 1] = 0.0;
    } else {
      const int m = (off + 1) >> 1;
      const double sg = (m & 1) ? -1.0 : 1.0;
      if (off & 1) {  // real part
        t[2 * (row + m)] = v;
        t[2 * (row - m)] = sg * v;
      } else {  // imaginary part
        t[2 * (row + m) + 1] = v;
        t[2 * (row - m) + 1] = -sg * v;
      }
    }
  }
}

template <int Q>
__device__ __forceinline__ void cmac(double (&acc)[(Q + 1) * (Q + 1)], int j, int k, double2 a,
                                     double br, double bi) {
  acc[cpk_re(j, k)] = fma(a.x, br, fma(-a.y, bi, acc[cpk_re(j, k)]));
  if (k) acc[cpk_im(j, k)] = fma(a.x, bi, fma(a.y, br, acc[cpk_im(j, k)]));
}

// Waves per M2QBXL and L2QBXL item.  The padded expansion table is shared by the item's
// waves, which split the order loop and combine their sums at the end: with one wave per
// item, the 20-23 KB table of a 64-thread block held occupancy near 1.5 waves per SIMD.
// From q = 9 on the sums alone need most of a wave's registers, and one wave per item is
// kept.  Up to q = 5 the registers are capped for 3 (M2QBXL) and 4 (L2QBXL) waves per SIMD,
// at the cost of 2 spilled VGPRs.
constexpr int qbxl_waves(int q) { return q <= 8 ? 4 : 1; }
// L2QBXL splits the output rows over its waves, so each keeps only its rows' sums, at every
// q.  Eight waves would not raise the occupancy at q = 8 (85 against 97 VGPRs: 5 waves per
// SIMD either way), since every wave also carries the harmonic recurrences.
constexpr int l2qbxl_waves(int) { return 4; }

// Wave that takes order mu: snake order over the NW waves, so that each gets the same
// number of (order, degree) steps when the work of an order falls linearly with mu.
template <int NW>
__device__ __forceinline__ int order_owner(int mu) {
  const int r = mu / NW, w = mu % NW;
  return (r & 1) ? NW - 1 - w : w;
}

// Sum the NQ per-lane sums of the NW waves into wave 0 through the LDS array buf (of at
// least 64 doubles, no longer read by the caller), up to bytes / 512 coefficients at a time.
template <int NQ, int NW>
__device__ __forceinline__ void sum_waves(double (&acc)[NQ], double* buf, int bytes) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ch = bytes / (64 * (int)sizeof(double));
  for (int i0 = 0; i0 < NQ; i0 += ch)
    for (int w = 1; w < NW; ++w) {
      __syncthreads();
      if (wave == w)
#pragma unroll
        for (int i = 0; i < NQ; ++i)
          if (i >= i0 && i < i0 + ch) buf[(i - i0) * 64 + lane] = acc[i];
      __syncthreads();
      if (wave == 0)
#pragma unroll
        for (int i = 0; i < NQ; ++i)
          if (i >= i0 && i < i0 + ch) acc[i] += buf[(i - i0) * 64 + lane];
    }
}

// Item i: centers [it_c0, it_c0 + it_nc) of one target box and the List 3 far boxes
// wf_box[it_w0 .. it_w1); long lists are split over several items, so the outputs are
// added atomically.
template <int Q, int PT, int NW = qbxl_waves(Q)>
__global__ __launch_bounds__(64 * NW, Q <= 5 ? 3 : 1) void k_m2qbxl(int P, const int* __restrict__ it_c0,
                                               const int* __restrict__ it_nc,
                                               const int* __restrict__ it_w0,
                                               const int* __restrict__ it_w1,
                                               const int* __restrict__ wf_box,
                                               const double* __restrict__ bctr,
                                               const double* __restrict__ bh,
                                               const double* __restrict__ M,
                                               const double* __restrict__ cx,
                                               const double* __restrict__ cy,
                                               const double* __restrict__ cz,
                                               double* __restrict__ Lq, int64_t nctr) {
  using TB = M2qTab<Q, PT>;
  constexpr int NQ = (Q + 1) * (Q + 1);
  __shared__ double2 tab[TB::ROWS * TB::W];
  for (int i = threadIdx.x; i < TB::ROWS * TB::W; i += blockDim.x) tab[i] = make_double2(0.0, 0.0);
  const int item = blockIdx.x;
  const int c0 = it_c0[item], nc = it_nc[item];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool active = lane < nc;
  const int64_t c = (int64_t)c0 + (active ? lane : 0);
  const double xc = cx[c], yc = cy[c], zc = cz[c];
  const int np = (P + 1) * (P + 1);
  const int NT = P + Q;
  double acc[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) acc[i] = 0.0;
  for (int w = it_w0[item]; w < it_w1[item]; ++w) {
    const int d = wf_box[w];
    const double a = bh[d];
    __syncthreads();
    fill_padded(M + (int64_t)d * np, P, tab, Q, TB::W, TB::MOFF,
                [a](int n) { return (n & 1) ? -pow(a, (double)n) : pow(a, (double)n); });
    __syncthreads();
    const double vx = xc - bctr[3 * d], vy = yc - bctr[3 * d + 1], vz = zc - bctr[3 * d + 2];
    const double ir2 = 1.0 / (vx * vx + vy * vy + vz * vz), zr = vz * ir2;
    // J'_N^M = (-1)^N conj(I_N^M)(v), generated for fixed M with increasing N
    double dr = sqrt(ir2), di = 0.0;
    for (int Mo = 0; Mo <= NT; ++Mo) {
      if (Mo > 0) {  // the diagonal is carried by every wave
        const double f = (2.0 * Mo - 1.0) * ir2;
        const double fr = f * vx, fi = -f * vy;
        const double nr = dr * fr - di * fi, ni = dr * fi + di * fr;
        dr = nr;
        di = ni;
      }
      if (order_owner<NW>(Mo) != wave) continue;  // uniform over the wave
      const double sgn = (Mo & 1) ? -1.0 : 1.0;
      double p1r = 0, p1i = 0, p2r = 0, p2i = 0;
      for (int N = Mo; N <= NT; ++N) {
        double jr, ji;
        if (N == Mo) {
          jr = dr;
          ji = di;
        } else {
          const double c1 = (2.0 * N - 1.0) * zr;
          const double c2 = (double)((N - 1) * (N - 1) - Mo * Mo) * ir2;
          jr = -c1 * p1r - c2 * p2r;
          ji = -c1 * p1i - c2 * p2i;
          p2r = p1r;
          p2i = p1i;
        }
        p1r = jr;
        p1i = ji;
        const double jnr = sgn * jr, jni = -sgn * ji;  // J'^{-M} = (-1)^M conj(J'^M)
        const double2* t1 = tab + (N * TB::W + Mo + TB::MOFF);
        const double2* t2 = tab + (N * TB::W - Mo + TB::MOFF);
#pragma unroll
        for (int j = 0; j <= Q; ++j) {
          const int n = N - j;
          if (n < 0 || n > P) continue;  // uniform
          if (Mo - j <= n) {
#pragma unroll
            for (int k = 0; k <= j; ++k) cmac<Q>(acc, j, k, t1[(Q - j) * TB::W - k], jr, ji);
          }
          if (Mo > 0 && Mo <= n) {
#pragma unroll
            for (int k = 0; k <= j; ++k) cmac<Q>(acc, j, k, t2[(Q - j) * TB::W - k], jnr, jni);
          }
        }
      }
    }
  }
  sum_waves<NQ, NW>(acc, reinterpret_cast<double*>(tab), (int)sizeof(tab));
  if (wave == 0 && active)
#pragma unroll
    for (int i = 0; i < NQ; ++i) unsafeAtomicAdd(&Lq[(int64_t)i * nctr + c], acc[i]);
}

// f(integral_constant<int, I>) for I = B .. E-1, each with I a constant expression
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Stage 8 output rows per wave.  The NW waves of an item split the output degrees j
// (each wave keeps the sums of its own rows only), balanced by longest-processing-time on
// the row's work (2j + 1)(P - j + 1)^2, at P = 15 for q <= 5 and P = 20 above.
template <int Q, int NW>
struct L2qRows {
  static constexpr int owner(int j) {
    const int P = Q <= 5 ? 15 : 20;
    long load[NW > 0 ? NW : 1] = {};
    int own[Q + 1] = {};
    bool done[Q + 1] = {};
    for (int step = 0; step <= Q; ++step) {
      int best = -1;
      long bw = -1;
      for (int jj = 0; jj <= Q; ++jj) {
        const long w = (long)(2 * jj + 1) * (P - jj + 1) * (P - jj + 1);
        if (!done[jj] && w > bw) {
          bw = w;
          best = jj;
        }
      }
      int g = 0;
      for (int h = 1; h < NW; ++h)
        if (load[h] < load[g]) g = h;
      own[best] = g;
      load[g] += bw;
      done[best] = true;
    }
    return own[j];
  }
};

// PAIR: the item is two consecutive entries of at most 32 centers each (of two boxes); the
// lower half of every wave serves the first, the upper half the second, each with its own
// table, so the order loop stays uniform over the wave.
// The waves split the output rows (L2qRows): every wave generates all harmonics of the
// center offset and adds them into its own rows' sums only, so a wave holds a quarter of
// the sums and no sums are combined across waves.
template <int Q, int NW = l2qbxl_waves(Q), bool PAIR = false>
__global__ __launch_bounds__(64 * NW, Q <= 5 ? (PAIR ? 3 : 4) : 1) void k_l2qbxl(int P, const int* __restrict__ it_box,
                                                           const int* __restrict__ it_c0,
                                                           const int* __restrict__ it_nc,
                                                           const double* __restrict__ bctr,
                                                           const double* __restrict__ bh,
                                                           const double* __restrict__ L,
                                                           const double* __restrict__ cx,
                                                           const double* __restrict__ cy,
                                                           const double* __restrict__ cz,
                                                           double* __restrict__ Lq,
                                                           int64_t nctr) {
  using TB = L2qTab<Q>;
  constexpr int NQ = (Q + 1) * (Q + 1);
  constexpr int NTAB = PAIR ? 2 : 1;
  constexpr int TSZ = TB::ROWS * TB::W;
  __shared__ double2 tab[NTAB * TSZ];
  __shared__ double invtab[kInvTab * kInvTab];
  for (int i = threadIdx.x; i < NTAB * TSZ; i += blockDim.x) tab[i] = make_double2(0.0, 0.0);
  fill_invtab(invtab);
  const int item = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sub = PAIR ? lane >> 5 : 0;        // entry of the pair this lane serves
  const int li = PAIR ? lane & 31 : lane;      // its center within the entry
  const int e = PAIR ? 2 * item + sub : item;
  const int b = it_box[e];
  const int c0 = it_c0[e], nc = it_nc[e];
  const bool active = li < nc;
  const int64_t c = (int64_t)c0 + (active ? li : 0);
  const int np = (P + 1) * (P + 1);
  __syncthreads();
  for (int k = 0; k < NTAB; ++k) {
    const int bk = it_box[PAIR ? 2 * item + k : item];
    const double a = bh[bk];
    fill_padded(L + (int64_t)bk * np, P, tab + k * TSZ, 0, TB::W, TB::MOFF,
                [a](int n) { return pow(a, -(double)(n + 1)); });
  }
  __syncthreads();
  const double2* tb = tab + sub * TSZ;  // this lane's table
  const double vx = cx[c] - bctr[3 * b], vy = cy[c] - bctr[3 * b + 1], vz = cz[c] - bctr[3 * b + 2];
  const double r2 = vx * vx + vy * vy + vz * vz;
  auto rows = [&](auto wtag) {
    constexpr int WV = decltype(wtag)::value;
    double acc[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) acc[i] = 0.0;
    double dr = 1.0, di = 0.0;
    for (int mu = 0; mu <= P; ++mu) {
      if (mu > 0) {
        const double f = -0.5 / mu;
        const double nr = f * (dr * vx - di * vy), ni = f * (dr * vy + di * vx);
        dr = nr;
        di = ni;
      }
      const double sgn = (mu & 1) ? -1.0 : 1.0;
      double p1r = 0, p1i = 0, p2r = 0, p2i = 0;
      for (int N = mu; N <= P; ++N) {
        double rr, ri;
        if (N == mu) {
          rr = dr;
          ri = di;
        } else {
          const double tt = invtab[N * kInvTab + mu];
          const double c1 = (2.0 * N - 1.0) * vz;
          rr = (c1 * p1r - r2 * p2r) * tt;
          ri = (c1 * p1i - r2 * p2i) * tt;
          p2r = p1r;
          p2i = p1i;
        }
        p1r = rr;
        p1i = ri;
        const double rnr = sgn * rr, rni = -sgn * ri;  // R^{-mu} = (-1)^mu conj(R^mu)
        const double2* t1 = tb + (N * TB::W + mu + TB::MOFF);
        const double2* t2 = tb + (N * TB::W - mu + TB::MOFF);
        static_for<0, Q + 1>([&](auto jtag) {
          constexpr int j = decltype(jtag)::value;
          if constexpr (L2qRows<Q, NW>::owner(j) == WV) {
            const int n = N + j;
            if (n <= P) {  // uniform
              if (mu <= n) {
#pragma unroll
                for (int k = 0; k <= j; ++k) cmac<Q>(acc, j, k, t1[j * TB::W + k], rr, ri);
              }
              if (mu > 0 && mu - j <= n) {
#pragma unroll
                for (int k = 0; k <= j; ++k) cmac<Q>(acc, j, k, t2[j * TB::W + k], rnr, rni);
              }
            }
          }
        });
      }
    }
    if (!active) return;
    static_for<0, Q + 1>([&](auto jtag) {
      constexpr int j = decltype(jtag)::value;
      if constexpr (L2qRows<Q, NW>::owner(j) == WV) {
#pragma unroll
        for (int i = j * j; i < (j + 1) * (j + 1); ++i) Lq[(int64_t)i * nctr + c] += acc[i];
      }
    });
  };
  static_assert(NW >= 1 && NW <= 8, "up to eight waves per item");
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  static_for<0, NW>([&](auto wtag) {
    if (wv == decltype(wtag)::value) rows(wtag);
  });
}

// ------------------------------------------------------------------------------------
// QBXL2P: one thread per target.
// ------------------------------------------------------------------------------------

template <int Q>
__global__ __launch_bounds__(256) void k_qbxl2p(int64_t ntgt, const int64_t* __restrict__ tgt_ctr,
                                                const double* __restrict__ tx,
                                                const double* __restrict__ ty,
                                                const double* __restrict__ tz,
                                                const double* __restrict__ cx,
                                                const double* __restrict__ cy,
                                                const double* __restrict__ cz,
                                                const double* __restrict__ Lq, int64_t nctr,
                                                const int64_t* __restrict__ out_idx,
                                                double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntgt) return;
  const int64_t c = tgt_ctr[t];
  const double ux = tx[t] - cx[c], uy = ty[t] - cy[c], uz = tz[t] - cz[c];
  const double r2 = ux * ux + uy * uy + uz * uz;
  double phi = 0.0;
  double dr = 1.0, di = 0.0;
#pragma unroll
  for (int m = 0; m <= Q; ++m) {
    if (m > 0) {
      const double f = -0.5 / m;
      const double nr = f * (dr * ux - di * uy), ni = f * (dr * uy + di * ux);
      dr = nr;
      di = ni;
    }
    const double wgt = m ? 2.0 : 1.0;
    double p1r = dr, p1i = di, p2r = 0.0, p2i = 0.0;
    phi += wgt * (Lq[(int64_t)cpk_re(m, m) * nctr + c] * dr -
                  (m ? Lq[(int64_t)cpk_im(m, m) * nctr + c] * di : 0.0));
#pragma unroll
    for (int n = m + 1; n <= Q; ++n) {
      double rr, ri;
      if (n == m + 1) {
        rr = uz * p1r;
        ri = uz * p1i;
      } else {
        const double inv = 1.0 / (double)(n * n - m * m);
        const double c1 = (2.0 * n - 1.0) * uz;
        rr = (c1 * p1r - r2 * p2r) * inv;
        ri = (c1 * p1i - r2 * p2i) * inv;
      }
      phi += wgt * (Lq[(int64_t)cpk_re(n, m) * nctr + c] * rr -
                    (m ? Lq[(int64_t)cpk_im(n, m) * nctr + c] * ri : 0.0));
      p2r = p1r;
      p2i = p1i;
      p1r = rr;
      p1i = ri;
    }
  }
  out[out_idx[t]] = phi * kInv4Pi;
}

// Stage 9 for the adjoint double layer S': the derivative of the QBX local along the
// target's unit normal nu,
//   phi'(t) = (1/4pi) Re sum_{n >= 1} sum_{|m| <= n} l_n^m (nu . grad) R_n^m (t - c),
//   (nu . grad) R_n^m = nu_z R_{n-1}^m + (nu_x - i nu_y)/2 R_{n-1}^{m+1}
//                       - (nu_x + i nu_y)/2 R_{n-1}^{m-1}   (zero where |order| > degree),
// with l^-m = (-1)^m conj(l^m) and R^-m = (-1)^m conj(R^m).
template <int Q>
__global__ __launch_bounds__(256) void k_qbxl2p_grad(
    int64_t ntgt, const int64_t* __restrict__ tgt_ctr, const double* __restrict__ tx,
    const double* __restrict__ ty, const double* __restrict__ tz, const double* __restrict__ tnx,
    const double* __restrict__ tny, const double* __restrict__ tnz, const double* __restrict__ cx,
    const double* __restrict__ cy, const double* __restrict__ cz, const double* __restrict__ Lq,
    int64_t nctr, const int64_t* __restrict__ out_idx, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntgt) return;
  const int64_t c = tgt_ctr[t];
  const double ux = tx[t] - cx[c], uy = ty[t] - cy[c], uz = tz[t] - cz[c];
  const double r2 = ux * ux + uy * uy + uz * uz;
  constexpr int K = Q > 0 ? Q : 1;  // degrees 0..Q-1 of R are needed
  double Rr[K * (K + 1) / 2], Ri[K * (K + 1) / 2];
  double dr = 1.0, di = 0.0;
#pragma unroll
  for (int m = 0; m < K; ++m) {
    if (m > 0) {  // R_m^m = -(x + i y)/(2m) R_{m-1}^{m-1}
      const double f = -0.5 / m;
      const double nr = f * (dr * ux - di * uy), ni = f * (dr * uy + di * ux);
      dr = nr;
      di = ni;
    }
    double p1r = dr, p1i = di, p2r = 0.0, p2i = 0.0;
    Rr[m * (m + 1) / 2 + m] = dr;
    Ri[m * (m + 1) / 2 + m] = di;
#pragma unroll
    for (int n = m + 1; n < K; ++n) {
      const double inv = 1.0 / (double)(n * n - m * m);
      const double c1 = (2.0 * n - 1.0) * uz;
      const double rr = (c1 * p1r - r2 * p2r) * inv, ri = (c1 * p1i - r2 * p2i) * inv;
      Rr[n * (n + 1) / 2 + m] = rr;
      Ri[n * (n + 1) / 2 + m] = ri;
      p2r = p1r;
      p2i = p1i;
      p1r = rr;
      p1i = ri;
    }
  }
  auto R = [&](int k, int j, double& re, double& im) {
    const int aj = j < 0 ? -j : j;
    if (aj > k) {
      re = im = 0.0;
      return;
    }
    re = Rr[k * (k + 1) / 2 + aj];
    im = Ri[k * (k + 1) / 2 + aj];
    if (j < 0) {  // R^-j = (-1)^j conj(R^j)
      const double sg = (aj & 1) ? -1.0 : 1.0;
      re *= sg;
      im *= -sg;
    }
  };
  const double ax = 0.5 * tnx[t], ay = 0.5 * tny[t], nz = tnz[t];
  double sum = 0.0;
#pragma unroll
  for (int n = 1; n <= Q; ++n) {
#pragma unroll
    for (int m = -n; m <= n; ++m) {
      const int am = m < 0 ? -m : m;
      double lr = Lq[(int64_t)cpk_re(n, am) * nctr + c];
      double li = am ? Lq[(int64_t)cpk_im(n, am) * nctr + c] : 0.0;
      if (m < 0) {  // l^-m = (-1)^m conj(l^m)
        const double sg = (am & 1) ? -1.0 : 1.0;
        lr *= sg;
        li *= -sg;
      }
      double r0r, r0i, rpr, rpi, rmr, rmi;
      R(n - 1, m, r0r, r0i);
      R(n - 1, m + 1, rpr, rpi);
      R(n - 1, m - 1, rmr, rmi);
      // D = nu_z R^m + (ax - i ay) R^(m+1) - (ax + i ay) R^(m-1)
      const double Dr = nz * r0r + (ax * rpr + ay * rpi) - (ax * rmr - ay * rmi);
      const double Di = nz * r0i + (ax * rpi - ay * rpr) - (ax * rmi + ay * rmr);
      sum += lr * Dr - li * Di;
    }
  }
  out[out_idx[t]] = sum * kInv4Pi;
}

// ------------------------------------------------------------------------------------
// dispatch helpers over the compile-time QBX order
// ------------------------------------------------------------------------------------

template <template <int> class F, int Qv = 0>
struct QDispatch {
  template <class... A>
  static void run(int q, A&&... a) {
    if (q == Qv)
      F<Qv>::go(a...);
    else if constexpr (Qv < kQmax)
      QDispatch<F, Qv + 1>::run(q, a...);
  }
};

inline dim3 grid1d(int64_t n, int bs) { return dim3((unsigned)((n + bs - 1) / bs)); }

template <int Q>
struct P2qbxlGo {
  static void go(hipStream_t s, int kernel, int nd, int nitem, const int* it_box,
                 const int* it_c0, const int* it_nc, const int64_t* np_, const int* ni,
                 SrcSoA src, const double* qs, int64_t qstride, const double* cx,
                 const double* cy, const double* cz, double* Lq, int64_t nctr,
                 int64_t lqstride) {
    if constexpr (Q <= kNd2Qmax) {
      if (nd == 2 && kernel) {
        k_p2qbxl<Q, 1, 2><<<nitem, 64, 0, s>>>(it_box, it_c0, it_nc, np_, ni, src, qs, qstride,
                                               cx, cy, cz, Lq, nctr, lqstride);
        return;
      }
    }
    if (kernel)
      k_p2qbxl<Q, 1, 1><<<nitem, 64, 0, s>>>(it_box, it_c0, it_nc, np_, ni, src, qs, qstride, cx,
                                             cy, cz, Lq, nctr, lqstride);
    else
      k_p2qbxl<Q, 0, 1><<<nitem, 64, 0, s>>>(it_box, it_c0, it_nc, np_, ni, src, qs, qstride, cx,
                                             cy, cz, Lq, nctr, lqstride);
  }
};

template <int Q>
struct M2qbxlGo {
  static void go(hipStream_t s, int p, int nitem, const int* it_c0, const int* it_nc,
                 const int* it_w0, const int* it_w1, const int* wf_box, const double* bctr,
                 const double* bh, const double* M, const double* cx, const double* cy,
                 const double* cz, double* Lq, int64_t nctr) {
    // smallest compiled table bound covering p
    if (p <= 8)
      k_m2qbxl<Q, 8><<<nitem, 64 * qbxl_waves(Q), 0, s>>>(p, it_c0, it_nc, it_w0, it_w1, wf_box, bctr, bh, M,
                                          cx, cy, cz, Lq, nctr);
    else if (p <= 12)
      k_m2qbxl<Q, 12><<<nitem, 64 * qbxl_waves(Q), 0, s>>>(p, it_c0, it_nc, it_w0, it_w1, wf_box, bctr, bh, M,
                                           cx, cy, cz, Lq, nctr);
    else if (p <= 16)
      k_m2qbxl<Q, 16><<<nitem, 64 * qbxl_waves(Q), 0, s>>>(p, it_c0, it_nc, it_w0, it_w1, wf_box, bctr, bh, M,
                                           cx, cy, cz, Lq, nctr);
    else
      k_m2qbxl<Q, kPmax><<<nitem, 64 * qbxl_waves(Q), 0, s>>>(p, it_c0, it_nc, it_w0, it_w1, wf_box, bctr, bh,
                                              M, cx, cy, cz, Lq, nctr);
  }
};

template <int Q>
struct L2qbxlGo {
  static void go(hipStream_t s, int p, int nitem, const int* it_box, const int* it_c0,
                 const int* it_nc, const double* bctr, const double* bh, const double* L,
                 const double* cx, const double* cy, const double* cz, double* Lq,
                 int64_t nctr) {
    k_l2qbxl<Q><<<nitem, 64 * l2qbxl_waves(Q), 0, s>>>(p, it_box, it_c0, it_nc, bctr, bh, L, cx,
                                                    cy, cz, Lq, nctr);
  }
};

template <int Q>
struct L2qbxlPairGo {
  static void go(hipStream_t s, int p, int nitem, const int* it_box, const int* it_c0,
                 const int* it_nc, const double* bctr, const double* bh, const double* L,
                 const double* cx, const double* cy, const double* cz, double* Lq,
                 int64_t nctr) {
    k_l2qbxl<Q, l2qbxl_waves(Q), true><<<nitem, 64 * l2qbxl_waves(Q), 0, s>>>(
        p, it_box, it_c0, it_nc, bctr, bh, L, cx, cy, cz, Lq, nctr);
  }
};

template <int Q>
struct Qbxl2pGradGo {
  static void go(hipStream_t s, int64_t ntgt, const int64_t* tgt_ctr, const double* tx,
                 const double* ty, const double* tz, const double* tnx, const double* tny,
                 const double* tnz, const double* cx, const double* cy, const double* cz,
                 const double* Lq, int64_t nctr, const int64_t* out_idx, double* out) {
    k_qbxl2p_grad<Q><<<grid1d(ntgt, 256), 256, 0, s>>>(ntgt, tgt_ctr, tx, ty, tz, tnx, tny, tnz,
                                                       cx, cy, cz, Lq, nctr, out_idx, out);
  }
};

template <int Q>
struct Qbxl2pGo {
  static void go(hipStream_t s, int64_t ntgt, const int64_t* tgt_ctr, const double* tx,
                 const double* ty, const double* tz, const double* cx, const double* cy,
                 const double* cz, const double* Lq, int64_t nctr, const int64_t* out_idx,
                 double* out) {
    k_qbxl2p<Q><<<grid1d(ntgt, 256), 256, 0, s>>>(ntgt, tgt_ctr, tx, ty, tz, cx, cy, cz, Lq,
                                                  nctr, out_idx, out);
  }
};

}  // namespace

void launch_fill(hipStream_t s, double* p, int64_t n, double v) {
  if (n <= 0) return;
  int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  k_fill<<<(unsigned)blocks, 256, 0, s>>>(p, n, v);
}

void launch_strength(hipStream_t s, int64_t n, const int64_t* order, const double* w,
                     const double* density, double* q) {
  if (n <= 0) return;
  k_strength<<<grid1d(n, 256), 256, 0, s>>>(n, order, w, density, q);
}

template <int CB, int MODE>
void launch_translate32(hipStream_t s, dim3 grid, int kind, int np, int ntile, const int* tile_cls,
                        const int* tile_beg, const int* tile_cnt, const int* pair_src,
                        const int* pair_dst, const TransMats& T, const double* X, double* Y,
                        int per_xcd) {
  auto k = kind == 0   ? k_translate32<0, CB, MODE>
           : kind == 1 ? k_translate32<1, CB, MODE>
           : kind == 2 ? k_translate32<2, CB, MODE>
                       : k_translate32<3, CB, MODE>;
  // one row round of 28 row blocks for p = 16..20, uncorrected mode with 32-pair tiles only:
  // measured on the ellipsoid, M2L 82 against 93 ms; the leading-degree mode lost (104
  // against 99 ms: 2 waves per SIMD instead of 4), and the split mode's FP64 step sums
  // would not fit
  constexpr bool kWide = CB == 2 && MODE == 0;
  const int nrb = trans_ld(np) / 16;
  if (kWide && nrb > 16 && nrb <= 28)
    k = kind == 0   ? k_translate32<0, CB, MODE, kWide ? 7 : 4>
        : kind == 1 ? k_translate32<1, CB, MODE, kWide ? 7 : 4>
        : kind == 2 ? k_translate32<2, CB, MODE, kWide ? 7 : 4>
                    : k_translate32<3, CB, MODE, kWide ? 7 : 4>;
  k<<<grid, 256, 0, s>>>(np, tile_cls, tile_beg, tile_cnt, pair_src, pair_dst, T.hi, T.lo,
                         T.lead, T.s_in, T.s_out, X, Y, ntile, per_xcd);
}

template <int CB>
void launch_translate_cb(hipStream_t s, int kind, int prec, int np, int ntile,
                         const int* tile_cls, const int* tile_beg, const int* tile_cnt,
                         const int* pair_src, const int* pair_dst, const TransMats& T,
                         const double* X, double* Y, bool xcd_order) {
  // xcd_order: blocks are dealt round-robin over the XCDs, so tile t runs on XCD t % 8
  // unless remapped; per_xcd = 1 with a grid of ntile reproduces plain order (t = block)
  const int per_xcd = xcd_order ? (ntile + kXcds - 1) / kXcds : 0;
  const dim3 grid(xcd_order ? per_xcd * kXcds : ntile);
  if (prec == 0) {
    // one row round of 28 row blocks for p = 16..20 (32-pair tiles; 64-pair tiles would need
    // twice the accumulators)
    const int nrb = trans_ld(np) / 16;
    constexpr bool kWide = CB == 2;
    auto k = kind == 0   ? k_translate<0, CB>
             : kind == 1 ? k_translate<1, CB>
             : kind == 2 ? k_translate<2, CB>
                         : k_translate<3, CB>;
    if (kWide && nrb > 16 && nrb <= 28)
      k = kind == 0   ? k_translate<0, CB, kWide ? 7 : 4>
          : kind == 1 ? k_translate<1, CB, kWide ? 7 : 4>
          : kind == 2 ? k_translate<2, CB, kWide ? 7 : 4>
                      : k_translate<3, CB, kWide ? 7 : 4>;
    k<<<grid, 256, 0, s>>>(np, tile_cls, tile_beg, tile_cnt, pair_src, pair_dst, T.t64, X, Y,
                           ntile, per_xcd);
  } else if (prec == 1) {
    launch_translate32<CB, 1>(s, grid, kind, np, ntile, tile_cls, tile_beg, tile_cnt, pair_src,
                              pair_dst, T, X, Y, per_xcd);
  } else if (prec == 2) {
    launch_translate32<CB, 0>(s, grid, kind, np, ntile, tile_cls, tile_beg, tile_cnt, pair_src,
                              pair_dst, T, X, Y, per_xcd);
  } else {
    launch_translate32<CB, 2>(s, grid, kind, np, ntile, tile_cls, tile_beg, tile_cnt, pair_src,
                              pair_dst, T, X, Y, per_xcd);
  }
}

// Ordered sum of slot results: block i adds the slots of destination dst[i], the pair
// positions pair[ptr[i] .. ptr[i+1]) in that order, into Y[dst[i]].  Each destination
// appears once, so no two blocks write the same output.
__global__ __launch_bounds__(256) void k_slot_sum(int np, const int* __restrict__ dst,
                                                  const int64_t* __restrict__ ptr,
                                                  const int* __restrict__ pair,
                                                  const double* __restrict__ S,
                                                  double* __restrict__ Y) {
  const int i = blockIdx.x;
  const int64_t b = ptr[i], e = ptr[i + 1];
  double* y = Y + (int64_t)dst[i] * np;
  for (int row = threadIdx.x; row < np; row += blockDim.x) {
    double sum = 0.0;
    for (int64_t k = b; k < e; ++k) sum += S[(int64_t)pair[k] * np + row];
    y[row] += sum;
  }
}

void launch_translate(hipStream_t s, int kind, int prec, int np, int ntile,
                      const int* tile_cls, const int* tile_beg, const int* tile_cnt,
                      const int* pair_src, const int* pair_dst, const TransMats& T,
                      const double* X, double* Y, int tile_cols, bool xcd_order,
                      bool to_slots) {
  if (ntile <= 0) return;
  if (to_slots) kind = 3;
  if (tile_cols == 32)
    launch_translate_cb<2>(s, kind, prec, np, ntile, tile_cls, tile_beg, tile_cnt, pair_src,
                           pair_dst, T, X, Y, xcd_order);
  else
    launch_translate_cb<4>(s, kind, prec, np, ntile, tile_cls, tile_beg, tile_cnt, pair_src,
                           pair_dst, T, X, Y, xcd_order);
}

void launch_slot_sum(hipStream_t s, int np, int ndst, const int* dst, const int64_t* ptr,
                     const int* pair, const double* slots, double* Y) {
  if (ndst <= 0) return;
  k_slot_sum<<<ndst, 256, 0, s>>>(np, dst, ptr, pair, slots, Y);
}

void launch_p2qbxl(hipStream_t s, int kernel, int q, int nitem, const int* it_box,
                   const int* it_c0, const int* it_nc, const int64_t* near_ptr,
                   const int* near_idx, SrcSoA src, const double* qs, const double* cx,
                   const double* cy, const double* cz, double* Lq, int64_t nctr, int nd,
                   int64_t qstride, int64_t lqstride) {
  if (nitem <= 0) return;
  QDispatch<P2qbxlGo>::run(q, s, kernel, nd == 2 ? 2 : 1, nitem, it_box, it_c0, it_nc, near_ptr,
                           near_idx, src, qs, qstride, cx, cy, cz, Lq, nctr, lqstride);
}

void launch_m2qbxl(hipStream_t s, int p, int q, int nitem, const int* it_c0,
                   const int* it_nc, const int* it_w0, const int* it_w1, const int* wf_box,
                   const double* bctr, const double* bh, const double* M, const double* cx,
                   const double* cy, const double* cz, double* Lq, int64_t nctr) {
  if (nitem <= 0) return;
  QDispatch<M2qbxlGo>::run(q, s, p, nitem, it_c0, it_nc, it_w0, it_w1, wf_box, bctr, bh, M, cx,
                           cy, cz, Lq, nctr);
}

void launch_l2qbxl(hipStream_t s, int p, int q, int nitem, const int* it_box,
                   const int* it_c0, const int* it_nc, const double* bctr, const double* bh,
                   const double* L, const double* cx, const double* cy, const double* cz,
                   double* Lq, int64_t nctr) {
  if (nitem <= 0) return;
  QDispatch<L2qbxlGo>::run(q, s, p, nitem, it_box, it_c0, it_nc, bctr, bh, L, cx, cy, cz, Lq,
                           nctr);
}

void launch_l2qbxl_pairs(hipStream_t s, int p, int q, int npair, const int* it_box,
                         const int* it_c0, const int* it_nc, const double* bctr,
                         const double* bh, const double* L, const double* cx, const double* cy,
                         const double* cz, double* Lq, int64_t nctr) {
  if (npair <= 0) return;
  QDispatch<L2qbxlPairGo>::run(q, s, p, npair, it_box, it_c0, it_nc, bctr, bh, L, cx, cy, cz,
                               Lq, nctr);
}

void launch_qbxl2p(hipStream_t s, int q, int64_t ntgt, const int64_t* tgt_ctr,
                   const double* tx, const double* ty, const double* tz, const double* cx,
                   const double* cy, const double* cz, const double* Lq, int64_t nctr,
                   const int64_t* out_idx, double* out) {
  if (ntgt <= 0) return;
  QDispatch<Qbxl2pGo>::run(q, s, ntgt, tgt_ctr, tx, ty, tz, cx, cy, cz, Lq, nctr, out_idx,
                           out);
}

void launch_qbxl2p_grad(hipStream_t s, int q, int64_t ntgt, const int64_t* tgt_ctr,
                        const double* tx, const double* ty, const double* tz, const double* tnx,
                        const double* tny, const double* tnz, const double* cx, const double* cy,
                        const double* cz, const double* Lq, int64_t nctr, const int64_t* out_idx,
                        double* out) {
  if (ntgt <= 0) return;
  QDispatch<Qbxl2pGradGo>::run(q, s, ntgt, tgt_ctr, tx, ty, tz, tnx, tny, tnz, cx, cy, cz, Lq,
                               nctr, out_idx, out);
}

}  // namespace gq
