// Launchers for the GIGAQBX device kernels (gfx950).  All arrays are device pointers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gq {

constexpr int kPmax = 20;  // highest FMM order supported by the device kernels
constexpr int kQmax = 10;  // highest QBX order supported by the device kernels
constexpr int kNd2Qmax = 5;  // highest QBX order of the two-density near-field kernel
constexpr int kTileCols = 64;  // expansions per translation tile (default; 32 also built)
constexpr int kTransKc = 64;   // K-chunk of the translation kernels

// Device layout of a translation matrix of order n_p = (p+1)^2: column-major with the
// rows padded to trans_ld and the columns to trans_kd, zeros in the padding.
__host__ __device__ inline int trans_ld(int np) { return (np + 15) / 16 * 16; }
__host__ __device__ inline int trans_kd(int np) { return (np + kTransKc - 1) / kTransKc * kTransKc; }

struct SrcSoA {
  const double *x, *y, *z, *nx, *ny, *nz;
};

// q[i] = w[i] * density[order[i]]
void launch_strength(hipStream_t s, int64_t n, const int64_t* order, const double* w,
                     const double* density, double* q);
// Oversampled quadrature: q[i] = w[i] * sum_k interp[f * n_node + k] * density[e * n_node + k]
// with (e, f) = divmod(order[i], n_quad) (source i in tree order; oversample.hip).
void launch_strength_interp(hipStream_t s, int64_t n, const int64_t* order, const double* w,
                            int n_node, int n_quad, const double* interp, const double* density,
                            double* q);
void launch_fill(hipStream_t s, double* p, int64_t n, double v);

// M2L by rotation (kernels_rot.hip), FP64, p_fmm <= 15: per class, the ntile nonzero 16 x 16
// tiles of A and B in row-tile order (row tile r, then column tile ascending), and the 2p+1
// order blocks of Z (block b holds the rows n^2 + b for n >= (b + 1) / 2 in increasing n,
// padded to 16).  Within a tile, element (row i, column k) is at [(16 (k % 4) + i) 4 + k / 4]:
// the matrix-core operand of lane 16 (k % 4) + i in k-step k / 4.
constexpr int kRotCols = 64;  // pairs per tile, 16 per wave
struct RotMats {
  const double *A, *Z, *B;
};
// The nonzero tiles of A per class that the kernel for order p assumes (-1: p > 15).
int m2l_rot_tiles(int p);
void launch_m2l_rot(hipStream_t s, int np, int ntile, const int* tile_cls, const int* tile_beg,
                    const int* tile_cnt, const int* pair_src, const int* pair_dst,
                    const RotMats& R, const double* X, double* Y, bool xcd_order,
                    bool to_slots = false);

// Target association (associate.hip).  A uniform grid of n[0] x n[1] x n[2] cells of width
// h from lo; cell (i, j, k) has linear index (k * n[1] + j) * n[0] + i.
struct AssocGrid {
  double lo[3];
  double h;
  int n[3];
};
// Points sorted by cell: cell c holds [start[c], start[c + 1]); r is the query radius of
// each point (danger radius, or center radius times 1 + tol); side and id for centers only.
struct AssocCells {
  const int64_t* start;
  const double *x, *y, *z, *r;
  const int8_t* side;
  const int64_t* id;
};
void launch_associate(hipStream_t s, int64_t nt, const double* tx, const double* ty,
                      const double* tz, const int8_t* tside, const AssocGrid& g,
                      const AssocCells& src, const AssocCells& ctr, int64_t* out);
// hit[i] = 1 iff a point of `pts` (grid g) lies within r[i] of query i (< if strict, else <=)
void launch_points_near(hipStream_t s, int64_t nq, const double* qx, const double* qy,
                        const double* qz, const double* r, int strict, const AssocGrid& g,
                        const AssocCells& pts, uint8_t* hit);

// Stage 2a: multipoles (scaled) of leaf boxes from their own sources.  Item i: box
// boxes[i], sources idx[ptr[i] .. ptr[i+1]) (tree positions).  Overwrites.  (kernels_p2x.hip)
// ordered: the block's partial sums are combined in a fixed order (reproducible results)
// instead of with LDS atomics; the same for P2L.
void launch_p2m(hipStream_t s, int kernel, int p, int nitem, const int* boxes,
                const int64_t* ptr, const int* idx, const double* bctr, const double* bh,
                SrcSoA src, const double* q, double* M, bool ordered = false);

// Stage 6b: box locals (scaled) of target boxes from the sources of their X-far boxes.
// Item i: box boxes[i], sources idx[ptr[i] .. ptr[i+1]).  Accumulates into L.
void launch_p2l(hipStream_t s, int kernel, int p, int nitem, const int* boxes,
                const int64_t* ptr, const int* idx, const double* bctr, const double* bh,
                SrcSoA src, const double* q, double* L, bool ordered = false);

// Translation matrices of one kind, column-major n_p x n_p per class: FP64 (t64), or for
// the FP32 modes the balanced matrix T^ = diag(1 / s_out) T diag(1 / s_in) as the FP32 pair
// T^ = hi + lo, its first kLead columns in FP64 (lead: [class][kLead][trans_ld] column-major)
// and the scalings s_in, s_out [n_p] (inputs are multiplied by s_in, outputs by s_out).
constexpr int kLeadCols = 16;
struct TransMats {
  const double* t64;
  const float *hi, *lo;
  const double* lead;
  const double *s_in, *s_out;
};

// Batched dense translations: for each tile t, Y[dst] += T[cls] X[src] for its pairs.
// kind: 0 M2M, 1 L2L, 2 M2L (selects a separately named instantiation).
// prec: 0 FP64 MFMA; 1 split (leading degrees on FP64 MFMA, the rest FP32 MFMA with the
// hi/lo correction products and FP64 accumulation per K-step); 2 FP32 MFMA, hi only, FP32
// accumulation; 3 leading degrees on FP64 MFMA, the rest FP32 MFMA hi only.
// tile_cols: 32 or 64, the tile width the tiles were formed with; xcd_order: map
// consecutive tiles to one XCD (else plain block order).  to_slots: instead of adding into
// Y[dst], store each pair's result to Y[(pair position) * np ..] (Y then holds one slot per
// pair of the tile set), for launch_slot_sum.
void launch_translate(hipStream_t s, int kind, int prec, int np, int ntile,
                      const int* tile_cls, const int* tile_beg, const int* tile_cnt,
                      const int* pair_src, const int* pair_dst, const TransMats& T,
                      const double* X, double* Y, int tile_cols = kTileCols,
                      bool xcd_order = true, bool to_slots = false);
// Reproducible accumulation of slot results: Y[dst[i]] += sum over k in [ptr[i], ptr[i+1])
// of slots[pair[k]], summed in that order; the dst[i] are distinct.
void launch_slot_sum(hipStream_t s, int np, int ndst, const int* dst, const int64_t* ptr,
                     const int* pair, const double* slots, double* Y);

// Stages 3, 5a, 6a: QBX locals from the near sources (U, W-close, X-close).
// Item i: target box it_box[i], centers [it_c0[i], it_c0[i]+it_nc[i]) (at most 64); the
// box's near sources are near_idx[near_ptr[b] .. near_ptr[b+1]) (tree positions).
// nd (1 or 2) densities in one pass, sharing each pair's solid harmonics: density d has
// its strengths at qs + d qstride and its locals at Lq + d lqstride.  nd = 2 is built for
// the double layer with q <= kNd2Qmax only (other calls run one density).
void launch_p2qbxl(hipStream_t s, int kernel, int q, int nitem, const int* it_box,
                   const int* it_c0, const int* it_nc, const int64_t* near_ptr,
                   const int* near_idx, SrcSoA src,
                   const double* qs, const double* cx, const double* cy, const double* cz,
                   double* Lq, int64_t nctr, int nd = 1, int64_t qstride = 0,
                   int64_t lqstride = 0);

// Stage 5b: QBX locals from W-far multipoles.  Item i: centers [it_c0, it_c0 + it_nc) and
// W-far boxes wf_box[it_w0 .. it_w1); accumulated atomically into Lq.
void launch_m2qbxl(hipStream_t s, int p, int q, int nitem, const int* it_c0,
                   const int* it_nc, const int* it_w0, const int* it_w1, const int* wf_box,
                   const double* bctr, const double* bh, const double* M, const double* cx,
                   const double* cy, const double* cz, double* Lq, int64_t nctr);

// Stage 8: QBX locals from the owning box's local.
void launch_l2qbxl(hipStream_t s, int p, int q, int nitem, const int* it_box,
                   const int* it_c0, const int* it_nc, const double* bctr, const double* bh,
                   const double* L, const double* cx, const double* cy, const double* cz,
                   double* Lq, int64_t nctr);

// Stage 8 for pairs of items: item i is entries 2i and 2i+1 of the arrays, each of at most
// 32 centers (of one box each); one wave serves both.
void launch_l2qbxl_pairs(hipStream_t s, int p, int q, int npair, const int* it_box,
                         const int* it_c0, const int* it_nc, const double* bctr,
                         const double* bh, const double* L, const double* cx, const double* cy,
                         const double* cz, double* Lq, int64_t nctr);

// Conventional targets (kernels_pt.hip), point targets in tree order, phi accumulates:
// Stages 3, 5a, 6a: direct sums from the box's near sources.  Item i: box it_box[i],
// point targets [it_t0[i], it_t0[i] + it_nt[i]) (at most 64).
void launch_p2p(hipStream_t s, int kernel, int nitem, const int* it_box, const int* it_t0,
                const int* it_nt, const int64_t* near_ptr, const int* near_idx, SrcSoA src,
                const double* qs, const double* px, const double* py, const double* pz,
                double* phi);
// Stage 5b: multipoles of List 3 far boxes wf_box[it_w0[i] .. it_w1[i]) at the item's
// targets.
void launch_m2p(hipStream_t s, int p, int nitem, const int* it_t0, const int* it_nt,
                const int* it_w0, const int* it_w1, const int* wf_box, const double* bctr,
                const double* bh, const double* M, const double* px, const double* py,
                const double* pz, double* phi);
// Stage 9: the owning box's local at each point target; writes out[out_idx[t]].
void launch_l2p(hipStream_t s, int p, int64_t npt, const int* pt_box, const double* bctr,
                const double* bh, const double* L, const double* px, const double* py,
                const double* pz, const double* phi, const int64_t* out_idx, double* out);

// Stage 9 for the adjoint double layer: derivative of the QBX local along the target
// normal (tnx, tny, tnz in target tree order).
void launch_qbxl2p_grad(hipStream_t s, int q, int64_t ntgt, const int64_t* tgt_ctr,
                        const double* tx, const double* ty, const double* tz, const double* tnx,
                        const double* tny, const double* tnz, const double* cx, const double* cy,
                        const double* cz, const double* Lq, int64_t nctr, const int64_t* out_idx,
                        double* out);

// Stage 9: potential at targets (tree order t -> output index out_idx[t]).
void launch_qbxl2p(hipStream_t s, int q, int64_t ntgt, const int64_t* tgt_ctr,
                   const double* tx, const double* ty, const double* tz, const double* cx,
                   const double* cy, const double* cz, const double* Lq, int64_t nctr,
                   const int64_t* out_idx, double* out);

}  // namespace gq
