/*
 * gigaqbx.h -- C ABI of the MI355X (gfx950) GIGAQBX library: FMM-accelerated
 * quadrature by expansion (QBX) for the 3D Laplace single- and double-layer potentials.
 *
 * Method: Wala & Kloeckner, "A fast algorithm for quadrature by expansion in three
 * dimensions" (arXiv:1805.06106).  The library evaluates Algorithm 5 (Stages 1-9) for
 * targets that are all associated with QBX centers:
 *
 *   potential(t) = sum_{n <= p_qbx} sum_{|m| <= n} L_n^m(c) |t - c|^n Y_n^m(t - c)
 *
 * where c is the center associated with target t and L(c) approximates the QBX local
 * coefficients of the layer potential (Section 2.1, QBX coefficient integral, discretized
 * by the quadrature sum over source nodes with weights w_j):
 *
 *   single layer S:  L_n^m(c) = sum_j w_j mu_j  1/(2n+1) |s_j - c|^-(n+1) Y_n^-m(s_j - c)
 *   double layer D:  same with the factor n_j . grad_{s_j} applied (kernel dG/dn_y,
 *                    G(x, y) = 1 / (4 pi |x - y|), n_j the source normal)
 *
 * accelerated by the GIGAQBX FMM of order p_fmm with target confinement factor t_f.
 *
 * Conventions for every entry point:
 *  - Host arrays are read during the call and copied; the caller keeps ownership.
 *  - Device arrays (density, potential) are caller-owned HIP device allocations; work is
 *    enqueued on `hip_stream` (NULL = default stream) in stream order.
 *  - Points are AoS, xyz interleaved: p[3*i + k].
 *  - Functions return a gq_status; on error nothing is written to caller outputs and
 *    gq_last_error() (thread-local) describes the failure.  No exceptions cross the ABI.
 */
#ifndef GIGAQBX_H
#define GIGAQBX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GQ_OK = 0,
  GQ_EINVAL = 1,       /* invalid argument */
  GQ_ENOMEM = 2,       /* device or host allocation failed */
  GQ_EDEVICE = 3,      /* HIP runtime error */
  GQ_EUNSUPPORTED = 4  /* valid but outside what this build supports (e.g. p_fmm > 20) */
} gq_status;

/* GQ_KERNEL_S: single layer S; GQ_KERNEL_D: double layer D (kernel dG/dn_y);
   GQ_KERNEL_SP: adjoint double layer S' = dS/dn_t, the derivative of the single layer
   along the target's unit normal (the Neumann operator): the QBX coefficients are S's and
   Stage 9 differentiates the local expansion (targets with a QBX center only; the target
   normals are given by gq_set_target_normals). */
typedef enum { GQ_KERNEL_S = 0, GQ_KERNEL_D = 1, GQ_KERNEL_SP = 2 } gq_kernel;
/* Arithmetic of the dense translations (M2M, M2L, L2L; Stages 2, 4, 7).  Every other
   stage, the expansions in memory and the final potential are FP64 in all modes.  The FP32
   modes work on balanced matrices: each degree n, order m coefficient is scaled by
   N_n^m = sqrt((n+m)! (n-m)!) (multipoles) or 1 / N_n^m (locals), the Schmidt
   semi-normalization of the solid harmonics, so that coefficients and matrix entries stay
   O(1) and inside FP32's range up to p_fmm = 20.
   GQ_FP64        FP64 matrix cores.
   GQ_FP32_SPLIT  split precision: the leading 16 packed coefficients of every input
                  (degrees n <= 3, which carry most of each output's magnitude because the
                  expansions decay with the degree) are contracted on the FP64 matrix cores;
                  the rest on the FP32 matrix cores as T_hi x_hi + T_hi x_lo + T_lo x_hi
                  (T = T_hi + T_lo, x = x_hi + x_lo), each K-step of 4 columns summed in
                  FP32 from zero and added into FP64 accumulators.
   GQ_FP32        uncorrected: T_hi x_hi over every column, FP32 accumulation over the
                  whole contraction.
   GQ_FP32_LEAD   the leading 16 coefficients on the FP64 matrix cores as in GQ_FP32_SPLIT,
                  the rest T_hi x_hi with FP32 accumulation (no correction products). */
typedef enum { GQ_FP64 = 0, GQ_FP32_SPLIT = 1, GQ_FP32 = 2, GQ_FP32_LEAD = 3 } gq_precision;

/* gq_params.flags */
#define GQ_FLAG_HOST_ONLY (1u << 0) /* plan on the host only: no device memory, no apply */
#define GQ_FLAG_TIMING (1u << 1)    /* record per-stage HIP events in gq_apply (gq_stats) */
/* Run gq_apply as one HIP graph: the first call with a given (density, potential) pair
   captures every kernel of the apply on a stream of the plan's own and later calls with
   the same pair replay it with one launch on the caller's stream (a new pair is captured
   anew).  Exclusive with GQ_FLAG_TIMING. */
#define GQ_FLAG_GRAPH (1u << 2)
/* At plan creation, time the Stage 4 (M2L) launch for tile widths 64 and 32 and for
   XCD-aware or plain tile order on the plan's own tiles, and keep the fastest (reported in
   gq_stats_t).  Without it: XCD-aware order, width 32 (also for the rotation M2L). */
#define GQ_FLAG_AUTOTUNE (1u << 3)
/* Reproducible applies: every gq_apply of the plan returns the same bits for the same
   density, and so does any plan built from the same inputs and parameters (the M2L tile
   shape the autotuner picks does not matter).  The translations (M2M, M2L, L2L) store each
   pair's result to a slot of its own and sum the slots of a destination in a fixed order
   instead of adding atomically; P2M and P2L combine their partial sums in a fixed order;
   List 3 far boxes are not split over several M2QBXL items.
   Costs one slot of (p_fmm+1)^2 doubles per M2L pair of device memory (11 GB for 5.5M
   pairs at p_fmm = 15) and the extra pass over it.  Without the flag, results of two
   applies agree to rounding (about 1e-15 relative) but not bit for bit.  Batch members
   must all have it or all lack it; the batch plan inherits it. */
#define GQ_FLAG_DETERMINISTIC (1u << 4)
/* Choose the tree at plan creation: build and time complete candidate plans (one warm-up
   and two timed applies of a unit density each, on hip_stream) with nmax at 1/2, 3/4, 1
   and 3/2 of gq_params.nmax, then, when wfar_direct_max is nonzero, Remark 4's threshold
   at 1/2 and 2 times its value with the best nmax, and keep the fastest.  The parameters
   kept are in the nmax and wfar_direct_max fields of the statistics; plan_seconds includes
   the search.  Candidates over max_device_bytes are skipped (GQ_ENOMEM if none fits); the
   search also holds a density and a potential buffer of its own.  Not with
   GQ_FLAG_HOST_ONLY. */
#define GQ_FLAG_AUTOTUNE_TREE (1u << 5)
/* Which interaction lists contribute (testing aid).  0 in bits 8..13 means all. */
#define GQ_LIST_U (1u << 8)       /* List 1 (direct)            Stage 3 */
#define GQ_LIST_V (1u << 9)       /* List 2 (M2L, then L2L)     Stages 4, 7, 8 */
#define GQ_LIST_WCLOSE (1u << 10) /* List 3 close (direct)      Stage 5a */
#define GQ_LIST_WFAR (1u << 11)   /* List 3 far (M2QBXL)        Stage 5b */
#define GQ_LIST_XCLOSE (1u << 12) /* List 4 close (direct)      Stage 6a */
#define GQ_LIST_XFAR (1u << 13)   /* List 4 far (P2L, then L2L) Stages 6b, 7, 8 */

typedef struct {
  int p_qbx;         /* QBX order, 0 <= p_qbx <= p_fmm, p_qbx <= 10 */
  int p_fmm;         /* FMM order, p_fmm <= 20 */
  int nmax;          /* max particles (sources+centers+targets) per box before a split, >= 1 */
  double tcf;        /* target confinement factor t_f, 0 <= t_f < 2 sqrt(3) - 2 (Theorem 1) */
  int kernel;        /* gq_kernel */
  int precision;     /* gq_precision */
  int n_densities;   /* densities evaluated per gq_apply, >= 1 */
  unsigned flags;    /* GQ_FLAG_* | GQ_LIST_* */
  /* Remark 4 of Section 5.2.4: a List 3 far box whose subtree holds at most this many
     sources is evaluated directly instead (its source leaves join List 3 close).  Exact
     replacement of an approximated interaction by a direct one; 0 disables it. */
  int wfar_direct_max;
  /* Shape of the target confinement region (Section 5.2.2): 0 the ball of radius
     sqrt(3)|b|(1 + t_f) of this method; 1 the box of half-width |b|(1 + t_f) of the
     earlier two-dimensional algorithm, kept for the cost comparison of Section 6 (Theorem 1
     is stated for the ball). */
  int tcr_norm;
  /* Level restriction (the remark on List 3 complexity in Section 5): 1 refines the tree
     after Stage 1 until leaves that touch differ by at most one level, splitting the
     coarser leaf of each offending pair by the usual rule (a leaf where nothing can move
     stays); 0 (default) keeps the adaptive tree as built. */
  int level_restrict;
  /* Stage 4 (M2L) arithmetic: 0 (default) one dense matrix per offset class; 1 the same
     operator factored as rotate, translate along z, rotate back (T = B Z A; the rotation-
     based translations of Appendix C's cost model), run as three sparse tile products on
     the FP64 matrix cores: 0.42 of the dense flops at p_fmm = 15, and faster on this chip.
     The factors are fitted on the host and reproduce the dense matrix to about 1e-11 of
     each row's largest entry.  1 needs GQ_FP64 and p_fmm <= 15 (else GQ_EUNSUPPORTED). */
  int m2l_rotation;
  /* Cap on the device memory a plan may hold (geometry, work lists, translation matrices,
     expansions), in bytes; 0 means no cap.  A plan that would exceed it is not created:
     gq_plan_create (or gq_batch_create, which applies the first member's cap) returns
     GQ_ENOMEM, frees what it had allocated and leaves *out untouched.  Later calls that
     add device data to a plan (gq_set_source_interp, gq_set_target_normals) are held to
     the same cap.  gq_stats reports the bytes a plan holds.  Must be >= 0. */
  int64_t max_device_bytes;
} gq_params;

typedef struct gq_plan gq_plan; /* opaque */

/* Statistics of a plan (and of the last timed apply). */
typedef struct {
  int64_t n_sources, n_centers, n_targets;
  int64_t n_boxes, n_levels, n_target_boxes, n_suspended_centers;
  int64_t list_entries[6];  /* box entries of U, V, Wclose, Wfar, Xclose, Xfar */
  /* interaction counts: U, Wclose, Xclose: (source, center) pairs; V: (box, box) pairs;
     Wfar: (box, center) pairs; Xfar: (source, box) pairs */
  int64_t pairs[6];
  int64_t m2l_classes;      /* distinct M2L offsets in use (at most 1206) */
  double plan_seconds;      /* host tree + lists + matrices + upload */
  /* With GQ_FLAG_TIMING: stage times (ms, HIP events on the stream that runs the stage;
     see gq_set_overlap) summed over all
     gq_apply calls (and densities) since the previous gq_stats call, and their count:
     0 strength, 1 P2M, 2 M2M, 3 M2L, 4 P2L, 5 L2L, 6 P2QBXL, 7 M2QBXL, 8 L2QBXL,
     9 QBXL2P, 10 fill, 11 total */
  double stage_ms[12];
  int64_t timed_applies;
  int32_t m2l_tile_cols;    /* M2L tile width in use (64 or 32) */
  int32_t m2l_xcd_order;    /* 1: XCD-aware M2L tile order, 0: plain */
  int64_t n_point_targets;  /* conventional targets (tgt_center = -1) */
  /* The operation-count model of Section 6 (Table 7) over the plan's interaction lists,
     with p = p_fmm and q = p_qbx: per list U, V, Wclose, Wfar, Xclose, Xfar the sum over
     entries of q^2 n_s n_t, p^3, q^2 n_s n_t, p^3 n_t, q^2 n_s n_t and p^2 n_s (n_s sources
     of the source box, n_t centers of the target box), then the total of the six. */
  double modeled_flops[7];
  int64_t device_bytes;     /* device memory held by the plan (its workspace) */
  int32_t nmax;             /* the tree's nmax and Remark 4 threshold in use (the given */
  int32_t wfar_direct_max;  /* values, or those GQ_FLAG_AUTOTUNE_TREE kept) */
} gq_stats_t;

/*
 * Build a plan (Algorithm 5 Stage 1 plus interaction lists, translation operators and
 * device-resident geometry).
 *   n_src, src_xyz[3*n_src], src_w[n_src]   source quadrature nodes and final weights
 *                                           (area element included)
 *   src_normal[3*n_src]                     unit normals; required for GQ_KERNEL_D, may be
 *                                           NULL for GQ_KERNEL_S
 *   n_ctr, ctr_xyz[3*n_ctr], ctr_radius[n_ctr]  QBX centers c = x +- r n (Section 2.2)
 *   n_tgt, tgt_xyz[3*n_tgt], tgt_center[n_tgt]  targets and their associated center index;
 *                                           tgt_center = -1 makes a conventional target:
 *                                           the plain layer potential at the point,
 *                                           evaluated by the FMM of Algorithm 5 (direct
 *                                           sums over the near lists, List 3 far
 *                                           multipoles, and the box local; no QBX), for
 *                                           points off the surface (a target on a source
 *                                           node gives inf)
 * Errors: GQ_EINVAL for negative counts, non-finite input, p_qbx > p_fmm, radius <= 0,
 * center index out of range (below -1 or >= n_ctr), missing or non-unit normals (|1-|n|| > 1e-6) for D, t_f out
 * of range; GQ_EUNSUPPORTED for orders beyond the compiled limits.  *out is set only on
 * success; release with gq_plan_destroy.
 */
gq_status gq_plan_create(const gq_params* params, int64_t n_src, const double* src_xyz,
                         const double* src_w, const double* src_normal, int64_t n_ctr,
                         const double* ctr_xyz, const double* ctr_radius, int64_t n_tgt,
                         const double* tgt_xyz, const int64_t* tgt_center, void* hip_stream,
                         gq_plan** out);

/*
 * Evaluate the layer potential (Algorithm 5 Stages 2-9) for params.n_densities densities.
 *   density   device, [n_densities][n_src] (row d is density d at the input source order)
 *   potential device, [n_densities][n_tgt], OVERWRITTEN (input target order); may be
 *             NULL when n_tgt = 0
 * The plan owns its workspace; concurrent applies of one plan must be serialized by the
 * caller (they share it).  Non-finite densities propagate to the output.
 */
gq_status gq_apply(gq_plan* plan, const double* density, double* potential, void* hip_stream);

/* Copy plan statistics.  With GQ_FLAG_TIMING this waits for the timed applies, sums
   their stage times into out->stage_ms and starts a new timing window. */
gq_status gq_stats(gq_plan* plan, gq_stats_t* out);

/*
 * Concurrent near and far field inside one apply (default off: on = 0).  The stages of
 * Algorithm 5 that build the box expansions (Stages 2, 4, 6b and 7: P2M, M2M, M2L, P2L,
 * L2L) read only the strengths and write only M and L, and the near field (Stages 3, 5a and
 * 6a) writes only the center locals, so the far-field chain runs on a stream owned by the
 * plan, forked from the apply stream by an event after the expansions are cleared and
 * joined back by an event before Stage 5b.  The apply is still ordered as a whole on the
 * caller's stream; the plan's stream has the default priority.  on = 0 runs every stage in
 * order on the apply stream.  It is off by default because on gfx950 the near-field
 * kernel's waves fill every SIMD's registers, so the far-field workgroups wait for the near
 * field to drain and the two streams gave no gain.  With GQ_FLAG_TIMING the far-field stage
 * times are taken on
 * the plan's stream, so with on = 1 the stage times overlap and may sum to more than the
 * whole apply.  A captured graph (GQ_FLAG_GRAPH) is recaptured at the next apply after a
 * change.  Errors: GQ_EINVAL for a NULL plan or on outside {0, 1}.
 */
gq_status gq_set_overlap(gq_plan* plan, int on);

/*
 * Target normals for GQ_KERNEL_SP: tgt_normal[3*n_tgt] unit vectors (host, input target
 * order; copied).  Required before the first gq_apply of an S' plan; may be called again
 * to change them.  Errors: GQ_EINVAL for a host-only or batch plan (a batch takes its
 * members' normals), non-finite or non-unit normals.
 */
gq_status gq_set_target_normals(gq_plan* plan, const double* tgt_normal);

/*
 * Oversampled source quadrature (Section 3, the stage-2 quadrature discretization: the
 * density lives on the nodes of a unisolvent discretization and the layer potential is
 * computed with a finer quadrature on the same elements).  After this call the densities
 * given to gq_apply are node values, [n_densities][n_elem * n_node] (element-major), and
 * the apply's first step computes the quadrature strengths of each source from its
 * element's node values:
 *   q_{e*n_quad + j} = w_{e*n_quad + j} * sum_k interp[j*n_node + k] * density[e*n_node + k]
 * The plan's sources must be the quadrature nodes in element-major order, so
 * n_src = n_elem * n_quad.  interp: host, [n_quad][n_node] row-major (copied);
 * 1 <= n_node <= 64, 1 <= n_quad, n_quad * n_node <= 2^20.  May be called again to change
 * the matrix; a captured graph of the plan is recaptured at the next apply.
 * Errors: GQ_EINVAL for a host-only plan, sizes that do not match the plan's sources or
 * exceed the limits, or non-finite entries; GQ_EUNSUPPORTED for a batch plan.
 */
gq_status gq_set_source_interp(gq_plan* plan, int64_t n_elem, int n_node, int n_quad,
                               const double* interp);

/*
 * gq_points_near without device allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, result and errors as gq_points_near; every device buffer of the query (cell
 * starts, sorted points, queries, radii, flags) lives in one fixed scratch array of 32 MiB
 * per GPU, held until the process ends.  The grid is limited to 2^20 cells (wider cells
 * only add candidates).  A query whose buffers exceed the scratch (about
 * 24 n_p + 33 n_q bytes plus the cell starts) returns GQ_EINVAL with outputs untouched.
 * Calls share the scratch of their GPU: calls that overlap in time on one GPU (from several
 * host threads) race and must be serialized by the caller; a call returns only when its
 * result is on the host.
 */
gq_status gq_points_near_noalloc(int64_t n_q, const double* q_xyz, const double* radius,
                                 int strict, int64_t n_p, const double* p_xyz, uint8_t* hit,
                                 void* hip_stream);

/* Target association results (gq_associate_targets) besides a center index. */
#define GQ_TARGET_FAR (-1)        /* no source endangers it: a conventional target */
#define GQ_TARGET_UNMATCHED (-2)  /* endangered, but no admissible center is close enough */

/*
 * Proximity query for geometry processing (the area queries of Algorithms 1 and 2, Section
 * 3): hit[i] = 1 if some point p_j lies within radius[i] of query q_i, else 0; with
 * strict != 0 the test is |q_i - p_j| < radius[i], else <=.  Squared distances are compared
 * in FP64 without fused multiply-adds, ((dx*dx + dy*dy) + dz*dz) against (r*r).
 *   q_xyz[3*n_q], radius[n_q] (finite, >= 0), p_xyz[3*n_p]: host; hit[n_q]: host output.
 * The queries run on the device over a uniform cell grid built on the host; the call
 * allocates and frees its own device memory and returns when the result is on the host.
 * Errors: GQ_EINVAL for NULL arrays with nonzero counts, non-finite coordinates, negative
 * or non-finite radii.
 */
gq_status gq_points_near(int64_t n_q, const double* q_xyz, const double* radius, int strict,
                         int64_t n_p, const double* p_xyz, uint8_t* hit, void* hip_stream);

/*
 * Associate targets with QBX centers (Algorithm 3, with the side preference of Section 3).
 * A target t is endangered if some source s has |t - s| <= danger[s] (the danger zone of
 * a source is half its element's size).  An endangered target is associated with the
 * closest center c with |t - c| <= ctr_radius[c] * (1 + tol) whose side matches: when
 * tgt_side[t] != 0, only centers with ctr_side[c] == tgt_side[t] qualify.  Equal
 * distances go to the lower center index.  Distances are compared squared, in FP64,
 * without fused multiply-adds: ((dx*dx + dy*dy) + dz*dz) <= (r*r).
 *   src_xyz[3*n_src], src_danger[n_src]        host, danger radii >= 0
 *   ctr_xyz[3*n_ctr], ctr_radius[n_ctr]        host, radii > 0
 *   ctr_side[n_ctr]   host, +1 / -1 per center (which side of the surface it lies on);
 *                     may be NULL when tgt_side is NULL
 *   tgt_xyz[3*n_tgt]  host
 *   tgt_side[n_tgt]   host, +1 / -1 / 0 (no preference); NULL means all 0
 *   tol               >= 0
 *   tgt_center[n_tgt] host output: a center index, GQ_TARGET_FAR or GQ_TARGET_UNMATCHED;
 *                     it can be passed to gq_plan_create once no entry is
 *                     GQ_TARGET_UNMATCHED (GQ_TARGET_FAR is its conventional-target mark)
 * The queries run on the device (one thread per target over a uniform cell grid built on
 * the host); the call allocates and frees its own device memory and returns when the
 * result is on the host.  Errors: GQ_EINVAL for NULL arrays with nonzero counts,
 * non-finite coordinates or radii, negative radii or tolerance, side values outside
 * {-1, 0, +1} (ctr_side: {-1, +1}), or tgt_side without ctr_side.
 */
gq_status gq_associate_targets(int64_t n_src, const double* src_xyz, const double* src_danger,
                               int64_t n_ctr, const double* ctr_xyz, const double* ctr_radius,
                               const int8_t* ctr_side, int64_t n_tgt, const double* tgt_xyz,
                               const int8_t* tgt_side, double tol, int64_t* tgt_center,
                               void* hip_stream);

/*
 * Merge plans into one batch plan (the many-surface form of Algorithm 5): each stage then
 * runs as one launch over every member's work, and the members' M2L pairs share the
 * offset-class matrices, so tiles fill across surfaces.
 *   plans[n_plans]  members; they must share p_qbx, p_fmm, kernel, precision and
 *                   n_densities and must not be host-only.  Their geometry and work lists
 *                   are copied: members may be destroyed or used on their own afterwards.
 *   flags           GQ_FLAG_TIMING or GQ_FLAG_GRAPH (or 0) for the batch plan.
 * The batch plan is applied with gq_apply and released with gq_plan_destroy.  Its density
 * is [n_densities][sum of member n_src] and its potential [n_densities][sum of member
 * n_tgt], members concatenated in the order given (member k's sources of density d at
 * d * sum_n_src + (n_src of members before k)).  Errors: GQ_EINVAL for mismatched or
 * host-only members, a member listed twice, or bad flags; GQ_EUNSUPPORTED beyond 2^31
 * boxes, sources or centers.
 */
gq_status gq_batch_create(int n_plans, gq_plan* const* plans, unsigned flags, void* hip_stream,
                          gq_plan** out);

/* Release a plan (NULL is ignored).  Synchronizes with outstanding device work. */
void gq_plan_destroy(gq_plan* plan);

/* Thread-local description of the last error ("" if none). */
const char* gq_last_error(void);

/*
 * Host-side export of the tree (for inspection and testing; works with
 * GQ_FLAG_HOST_ONLY).  Boxes are numbered breadth-first with children in octant order
 * (bit 0: x upper half, bit 1: y, bit 2: z).  Any pointer may be NULL.
 *   box_center[3*n_boxes], box_h[n_boxes] (half-width), level[n_boxes], parent[n_boxes]
 *   (-1 for the root), ctr_owner[n_ctr] owning box of each input center.
 */
gq_status gq_tree_export(const gq_plan* plan, double* box_center, double* box_h,
                         int32_t* level, int32_t* parent, int64_t* ctr_owner);

/*
 * Host-side export of one interaction list as CSR over boxes.
 *   list: 0 U (List 1), 1 V (List 2), 2 W-close, 3 W-far, 4 X-close, 5 X-far
 *   ptr[n_boxes+1] (may be NULL), items[*n_items] (may be NULL); *n_items receives the
 *   entry count.  Lists exist for target boxes (U, W-close, W-far, X-close) and for target
 *   and target-ancestor boxes (V, X-far; X-close also for ancestors).
 */
gq_status gq_list_export(const gq_plan* plan, int list, int64_t* ptr, int32_t* items,
                         int64_t* n_items);

/*
 * Download the QBX local coefficients of the last gq_apply for its last density
 * (n_densities - 1; density 0 for a one-density plan), after Stage 8:
 * host_out[n_ctr * (p_qbx+1)^2], input center order, in the library's internal real-packed
 * solid-harmonic form l_n^m = sum_j q_j conj(I_n^m)(s_j - c), with
 * I_n^m(v) = (n-m)! P_n^m(cos theta) e^{i m phi} / r^(n+1) (Condon-Shortley phase in P_n^m),
 * so that the potential is (1/4 pi) sum_n [l_n^0 R_n^0 + 2 Re sum_{m>0} l_n^m R_n^m](t - c)
 * with R_n^m(v) = r^n P_n^m(cos theta) e^{i m phi} / (n+m)!.  Synchronizes the plan's last stream.
 */
gq_status gq_qbx_locals(gq_plan* plan, double* host_out);

/*
 * Host computation of one dense translation matrix (column-major, (p+1)^2 square):
 *   kind 0: M2M child octant a -> parent;  kind 1: L2L parent -> child octant a;
 *   kind 2: M2L for integer offset (a, b, c) = (x_target - x_source) / (box width);
 *   kinds 3, 4, 5: the factors A, Z, B of that M2L (kind 2 = B Z A): A rotates multipoles
 *   so that the offset points along +z, Z translates along z, B rotates locals back.
 * Scaled real-packed form; for testing.
 */
gq_status gq_translation_matrix(int kind, int p, int a, int b, int c, double* out);

#ifdef __cplusplus
}
#endif

#endif /* GIGAQBX_H */
