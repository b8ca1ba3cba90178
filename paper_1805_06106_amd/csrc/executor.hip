// Plan construction and the Algorithm 5 evaluation pipeline behind the C ABI.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/gigaqbx.h"
#include "kernels.hpp"
#include "planner.hpp"
#include "query.hpp"

namespace {

thread_local std::string g_err;

gq_status fail(gq_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define GQ_HIP(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(e_ == hipErrorOutOfMemory ? GQ_ENOMEM : GQ_EDEVICE,                      \
                  std::string(#call) + ": " + hipGetErrorString(e_));                      \
  } while (0)

// A batch of dense translations: tiles of up to kTileCols pairs of one matrix class.
struct TileSet {
  std::vector<int> cls, beg, cnt, src, dst;
  int ntile() const { return (int)cls.size(); }
};

// pairs (cls, src, dst) -> tiles of at most `width` pairs, grouped by class
void make_tiles(std::vector<std::array<int, 3>> pairs, TileSet& ts, int width = gq::kTileCols) {
  std::stable_sort(pairs.begin(), pairs.end(),
                   [](const std::array<int, 3>& a, const std::array<int, 3>& b) { return a[0] < b[0]; });
  size_t i = 0;
  while (i < pairs.size()) {
    size_t j = i;
    while (j < pairs.size() && pairs[j][0] == pairs[i][0] && j - i < (size_t)width) ++j;
    ts.cls.push_back(pairs[i][0]);
    ts.beg.push_back((int)ts.src.size());
    ts.cnt.push_back((int)(j - i));
    for (size_t k = i; k < j; ++k) {
      ts.src.push_back(pairs[k][1]);
      ts.dst.push_back(pairs[k][2]);
    }
    i = j;
  }
}

// M2L tile width of a plan that is not autotuned: the autotuner's choice on the urchin,
// 32 pairs (FP64 7.6 against 8.4 ms for 64, FP32 5.2 against 6.1 ms; the split kernel
// holds its FP64 accumulators in registers, which 64-pair tiles would double); the
// rotation kernel has its own width.
int default_m2l_cols(const gq_params& prm) {
  if (prm.m2l_rotation) return gq::kRotCols;
  return 32;
}

// M2M and L2L tile width, by the same rule as M2L: the level passes have few tiles at the
// coarse levels, where narrower tiles give more workgroups.
int level_cols(const gq_params&) { return 32; }

}  // namespace

// Timing events of one density pass: 0..11 close consecutive stages on the apply stream
// (or, for the far-field chain, on the stream that runs it); 12 opens the near field and 13
// the first stage after the join, so that neither interval counts the other stream's work.
constexpr int kEvents = 14;

struct gq_plan {
  gq_params prm{};
  int np = 0, nq = 0;
  int64_t n_src = 0, n_ctr = 0, n_tgt = 0;
  gq::Tree tree;
  gq::Lists lists;
  gq_stats_t stats{};
  hipStream_t last_stream = nullptr;

  // host work description
  std::vector<int> p2m_boxes;
  std::vector<int64_t> p2m_ptr;  // item -> sources p2m_idx[ptr[i] .. ptr[i+1])
  std::vector<int> p2m_idx;
  std::vector<TileSet> m2m_levels;  // index: child level
  TileSet m2l;
  std::vector<TileSet> l2l_levels;  // index: child level
  std::vector<int> p2l_box;
  std::vector<int64_t> p2l_ptr;
  std::vector<int> p2l_idx;
  std::vector<int64_t> near_ptr;  // box-indexed CSR into near_idx
  std::vector<int> near_idx;      // near sources (tree positions) of each target box
  std::vector<int> k3_box, k3_c0, k3_nc;
  std::vector<int> wf_box;
  std::vector<int> k5_c0, k5_nc, k5_w0, k5_w1;
  std::vector<int> k8_box, k8_c0, k8_nc;  // single items, then pairs (pair_center_items)
  int k8_nsingle = 0, k8_npair = 0;
  // conventional targets (no QBX center), in tree order grouped by owning box
  int64_t n_pt = 0, n_qt = 0;             // point targets, QBX targets
  std::vector<int64_t> pt_count_box;      // per box: point targets owned
  std::vector<int64_t> pt_first_box;      // per box: its first point target
  std::vector<int64_t> h_pt_in;           // tree position -> input target index
  std::vector<int> h_pt_box;              // tree position -> owning box
  std::vector<int> pp_box, pp_t0, pp_nt;  // direct-sum items
  std::vector<int> pm_t0, pm_nt, pm_w0, pm_w1;  // multipole-evaluation items
  std::vector<int> cls_keys;           // M2L class index -> offset key
  int m2l_cols = gq::kTileCols;        // M2L tile width (32 or 64)
  int lvl_cols = gq::kTileCols;        // M2M and L2L tile width (32 or 64)
  bool m2l_xcd = true;                 // XCD-aware M2L tile order
  std::vector<int64_t> h_tgt_ctr, h_tgt_out;  // host copies of tgt_ctr / tgt_out
  bool is_batch = false;               // made by gq_batch_create
  // oversampled source quadrature: densities are node values of n_elem elements
  int64_t n_elem = 0;
  int n_node = 0, n_quad = 0;

  // device memory
  std::vector<void*> allocs;
  int64_t dev_bytes = 0;  // bytes in allocs
  double *sx = nullptr, *sy = nullptr, *sz = nullptr, *snx = nullptr, *sny = nullptr,
         *snz = nullptr, *sw = nullptr;
  int64_t* src_order = nullptr;
  double *cx = nullptr, *cy = nullptr, *cz = nullptr;
  double *tx = nullptr, *ty = nullptr, *tz = nullptr;
  int64_t *tgt_ctr = nullptr, *tgt_out = nullptr;
  double *bctr = nullptr, *bh = nullptr;
  int64_t *src_start = nullptr, *src_count = nullptr;
  int* d_p2m_boxes = nullptr;
  int64_t* d_p2m_ptr = nullptr;
  int* d_p2m_idx = nullptr;
  std::vector<std::array<int*, 5>> d_m2m, d_l2l;
  std::array<int*, 5> d_m2l{};
  int *d_p2l_box = nullptr;
  int64_t* d_p2l_ptr = nullptr;
  int* d_p2l_idx = nullptr;
  int64_t* d_near_ptr = nullptr;
  int* d_near_idx = nullptr;
  int *d_k3_box = nullptr, *d_k3_c0 = nullptr, *d_k3_nc = nullptr;
  int* d_wf_box = nullptr;
  int *d_k5_c0 = nullptr, *d_k5_nc = nullptr, *d_k5_w0 = nullptr, *d_k5_w1 = nullptr;
  int *d_k8_box = nullptr, *d_k8_c0 = nullptr, *d_k8_nc = nullptr;
  double *px = nullptr, *py = nullptr, *pz = nullptr, *phi = nullptr;
  double *tnx = nullptr, *tny = nullptr, *tnz = nullptr;  // S': QBX target normals
  int* d_pt_box = nullptr;
  int64_t* d_pt_out = nullptr;
  int *d_pp_box = nullptr, *d_pp_t0 = nullptr, *d_pp_nt = nullptr;
  int *d_pm_t0 = nullptr, *d_pm_nt = nullptr, *d_pm_w0 = nullptr, *d_pm_w1 = nullptr;
  double *T_m2m = nullptr, *T_l2l = nullptr, *T_m2l = nullptr;
  // M2L by rotation: per-class tiles of A, B and order blocks of Z
  double *R_A = nullptr, *R_Z = nullptr, *R_B = nullptr;
  gq::RotMats rot{};
  float *T32_m2m[2] = {nullptr, nullptr}, *T32_l2l[2] = {nullptr, nullptr},
        *T32_m2l[2] = {nullptr, nullptr};  // (hi, lo)
  // FP32 modes: leading FP64 columns of the balanced matrices and the balancing N, 1 / N
  double *Tlead_m2m = nullptr, *Tlead_l2l = nullptr, *Tlead_m2l = nullptr;
  double *d_norm = nullptr, *d_inorm = nullptr;
  gq::TransMats tm_m2m{}, tm_l2l{}, tm_m2l{};
  double *q = nullptr, *M = nullptr, *L = nullptr, *Lq = nullptr;
  double* interp = nullptr;  // [n_quad][n_node], set by gq_set_source_interp
  // GQ_FLAG_DETERMINISTIC: every translation stores its result to a slot of its own (one
  // per pair, np doubles each, shared by all tile sets) and an ordered sum per destination
  // adds them in pair order
  struct SlotSum {
    int ndst = 0;
    int* dst = nullptr;
    int64_t* ptr = nullptr;
    int* pair = nullptr;
  };
  bool det = false;
  double* slots = nullptr;
  // densities per near-field pass (1 or 2): with 2, q and Lq hold two densities each
  int nbuf = 1;
  SlotSum ss_m2l;
  std::vector<SlotSum> ss_m2m, ss_l2l;  // index: child level
  // GQ_FLAG_GRAPH: the passes of one apply captured once per (density, potential) pair
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  const double* graph_density = nullptr;
  double* graph_potential = nullptr;
  int64_t graph_launches = 0;
  // near field and far field on two streams: the far-field chain (P2M, M2M, M2L, P2L,
  // L2L) runs on `side`, forked from the apply stream after the fills and joined back before
  // the first stage that reads M or L into the center locals
  bool overlap = false;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // per-stage timing: one event set per density pass, summed by gq_stats()
  std::vector<std::array<hipEvent_t, kEvents>> ev_sets;
  size_t ev_used = 0;
  int64_t timed_applies = 0;

  ~gq_plan() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (side) (void)hipStreamDestroy(side);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    for (auto& set : ev_sets)
      for (auto& e : set) (void)hipEventDestroy(e);
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace {

// Densities that share one near-field pass: two for the double layer up to p_qbx =
// kNd2Qmax when the plan has more than one density.  Measured on one MI355X: the urchin's
// near field for two densities took 25.5 ms in one pass against 32.6 ms in two (D, q = 5);
// the single layer lost (217 against 193 ms, S, q = 8: the pass's two sets of sums leave too
// few registers for the harmonics), so it keeps one density per pass.
int near_field_densities(const gq_params& prm) {
  return prm.n_densities >= 2 && prm.kernel == GQ_KERNEL_D && prm.p_qbx <= gq::kNd2Qmax ? 2
                                                                                        : 1;
}

// Every device allocation of a plan goes through here: the workspace cap is enforced and
// the held bytes counted.
gq_status plan_malloc(gq_plan* P, void** d, size_t bytes) {
  if (P->prm.max_device_bytes > 0 &&
      P->dev_bytes + (int64_t)bytes > P->prm.max_device_bytes)
    return fail(GQ_ENOMEM, "the plan needs more device memory than its cap of " +
                               std::to_string(P->prm.max_device_bytes) + " bytes");
  GQ_HIP(hipMalloc(d, bytes));
  P->allocs.push_back(*d);
  P->dev_bytes += (int64_t)bytes;
  return GQ_OK;
}

template <class T>
gq_status upload(gq_plan* P, const std::vector<T>& h, T** d, hipStream_t s) {
  *d = nullptr;
  if (h.empty()) return GQ_OK;
  gq_status st = plan_malloc(P, (void**)d, h.size() * sizeof(T));
  if (st != GQ_OK) return st;
  GQ_HIP(hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return GQ_OK;
}

template <class T>
gq_status alloc(gq_plan* P, size_t n, T** d) {
  *d = nullptr;
  if (n == 0) return GQ_OK;
  return plan_malloc(P, (void**)d, n * sizeof(T));
}

#define GQ_TRY(x)                  \
  do {                             \
    gq_status st_ = (x);           \
    if (st_ != GQ_OK) return st_;  \
  } while (0)

bool finite3(const double* p, int64_t n) {
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

void merge_ranges(std::vector<std::pair<int64_t, int64_t>>& r) {
  std::sort(r.begin(), r.end());
  std::vector<std::pair<int64_t, int64_t>> out;
  for (auto& x : r) {
    if (x.second == 0) continue;
    if (!out.empty() && out.back().first + out.back().second == x.first)
      out.back().second += x.second;
    else
      out.push_back(x);
  }
  r.swap(out);
}

void center_items(const gq::Tree& T, int b, int chunk, std::vector<int>& box,
                  std::vector<int>& c0, std::vector<int>& nc) {
  int64_t s = T.ctr_start[b], n = T.ctr_count[b];
  for (int64_t o = 0; o < n; o += chunk) {
    box.push_back(b);
    c0.push_back((int)(s + o));
    nc.push_back((int)std::min<int64_t>(chunk, n - o));
  }
}

// Near-field items.  An item of r <= 64 centers runs one wave with S = 64 / r source slices,
// so r * S of its 64 lanes work and the wave makes n / S passes over the box's n near
// sources.  Cutting a box's centers into plain 64-chunks leaves the last chunk with up to
// half its lanes idle (r = 33 gives S = 1); instead the remainder is split into chunks that
// fill the lanes (37 = 32 + 5: S = 2 and 12), chosen by a small dynamic program that
// minimizes the passes sum(1 / S) plus a per-item charge of 1/64 for staging the sources
// once more.
const std::array<std::vector<int>, 64>& near_chunk_table() {
  static const std::array<std::vector<int>, 64> table = [] {
    std::array<double, 64> best{};
    std::array<int, 64> first{};
    for (int r = 1; r < 64; ++r) {
      best[r] = 1e30;
      for (int k = 1; k <= r; ++k) {
        const double c = 1.0 / (64 / k) + 1.0 / 64 + best[r - k];
        if (c < best[r] - 1e-12) {
          best[r] = c;
          first[r] = k;
        }
      }
    }
    std::array<std::vector<int>, 64> t;
    for (int r = 1; r < 64; ++r)
      for (int q = r; q > 0; q -= first[q]) t[r].push_back(first[q]);
    return t;
  }();
  return table;
}

void near_center_items(const gq::Tree& T, int b, std::vector<int>& box, std::vector<int>& c0,
                       std::vector<int>& nc) {
  int64_t s = T.ctr_start[b], n = T.ctr_count[b];
  auto push = [&](int64_t o, int k) {
    box.push_back(b);
    c0.push_back((int)(s + o));
    nc.push_back(k);
  };
  int64_t o = 0;
  for (; o + 64 <= n; o += 64) push(o, 64);
  for (int k : near_chunk_table()[n - o]) {
    push(o, k);
    o += k;
  }
}

// Stage 8 items of at most 32 centers go two to a wave, one per half-wave: the arrays hold
// the single items first, then the pairs as consecutive entries.  Rebuilds the order from
// any input order (a batch re-pairs its members' items).
void pair_center_items(gq_plan* P) {
  std::vector<int> box, c0, nc, sb, sc, sn;
  for (size_t i = 0; i < P->k8_box.size(); ++i) {
    auto& b = P->k8_nc[i] <= 32 ? sb : box;
    auto& c = P->k8_nc[i] <= 32 ? sc : c0;
    auto& n = P->k8_nc[i] <= 32 ? sn : nc;
    b.push_back(P->k8_box[i]);
    c.push_back(P->k8_c0[i]);
    n.push_back(P->k8_nc[i]);
  }
  if (sb.size() % 2) {  // the odd one out runs as a single item
    box.push_back(sb.back());
    c0.push_back(sc.back());
    nc.push_back(sn.back());
    sb.pop_back();
    sc.pop_back();
    sn.pop_back();
  }
  P->k8_nsingle = (int)box.size();
  P->k8_npair = (int)(sb.size() / 2);
  box.insert(box.end(), sb.begin(), sb.end());
  c0.insert(c0.end(), sc.begin(), sc.end());
  nc.insert(nc.end(), sn.begin(), sn.end());
  P->k8_box.swap(box);
  P->k8_c0.swap(c0);
  P->k8_nc.swap(nc);
}

// Near-field items, most expensive first (passes over the near sources times slice length),
// so that the longest workgroups start early.
void sort_near_items(gq_plan* P) {
  const size_t n = P->k3_box.size();
  std::vector<size_t> ord(n);
  std::vector<int64_t> cost(n);
  for (size_t i = 0; i < n; ++i) {
    ord[i] = i;
    const int b = P->k3_box[i];
    const int64_t slices = 64 / P->k3_nc[i];
    cost[i] = (P->near_ptr[b + 1] - P->near_ptr[b] + slices - 1) / slices;
  }
  std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
  std::vector<int> bx(n), c0(n), nc(n);
  for (size_t i = 0; i < n; ++i) {
    bx[i] = P->k3_box[ord[i]];
    c0[i] = P->k3_c0[ord[i]];
    nc[i] = P->k3_nc[ord[i]];
  }
  P->k3_box.swap(bx);
  P->k3_c0.swap(c0);
  P->k3_nc.swap(nc);
}

gq_status build_work(gq_plan* P) {
  const gq::Tree& T = P->tree;
  const gq::Lists& Ls = P->lists;
  const int nb = T.nboxes;
  unsigned mask = (P->prm.flags >> 8) & 63u;
  if (mask == 0) mask = 63u;
  auto on = [&](unsigned bit) { return (mask & (bit >> 8)) != 0; };

  // Stage 2a
  P->p2m_ptr.push_back(0);
  for (int b = 0; b < nb; ++b)
    if (T.is_leaf(b) && T.src_count[b] > 0) {
      P->p2m_boxes.push_back(b);
      for (int64_t k = 0; k < T.src_count[b]; ++k) P->p2m_idx.push_back((int)(T.src_start[b] + k));
      P->p2m_ptr.push_back((int64_t)P->p2m_idx.size());
    }
  // Stage 2b, per child level (deepest first when launched)
  P->m2m_levels.assign(T.nlevels, TileSet());
  {
    std::vector<std::vector<std::array<int, 3>>> per(T.nlevels);
    for (int b = 0; b < nb; ++b) {
      int pb = T.parent[b];
      if (pb < 0 || T.sub_src[b] == 0) continue;
      int oct = -1;
      for (int o = 0; o < 8; ++o)
        if (T.child[pb][o] == b) oct = o;
      per[T.level[b]].push_back({oct, b, pb});
    }
    P->lvl_cols = level_cols(P->prm);
    for (int l = 0; l < T.nlevels; ++l) make_tiles(per[l], P->m2m_levels[l], P->lvl_cols);
  }
  // Stage 4
  std::map<int, int> cls_index;
  std::vector<int>& cls_keys = P->cls_keys;
  if (on(GQ_LIST_V)) {
    std::vector<std::array<int, 3>> pairs;
    for (int b = 0; b < nb; ++b) {
      const auto& V = Ls.lst[gq::L_V];
      for (int64_t k = V.ptr[b]; k < V.ptr[b + 1]; ++k) {
        int d = V.items[k];
        int o[3];
        for (int a = 0; a < 3; ++a) {
          double off = (T.center[3 * b + a] - T.center[3 * d + a]) / (2.0 * T.h[b]);
          o[a] = (int)std::lround(off);
        }
        int key = (o[0] + 5) * 121 + (o[1] + 5) * 11 + (o[2] + 5);
        auto it = cls_index.find(key);
        int ci;
        if (it == cls_index.end()) {
          ci = (int)cls_keys.size();
          cls_index[key] = ci;
          cls_keys.push_back(key);
        } else {
          ci = it->second;
        }
        pairs.push_back({ci, d, b});
      }
    }
    P->m2l_cols = default_m2l_cols(P->prm);
    make_tiles(pairs, P->m2l, P->m2l_cols);
  }
  // Stage 6b
  if (on(GQ_LIST_XFAR)) {
    const auto& X = Ls.lst[gq::L_XFAR];
    P->p2l_ptr.push_back(0);
    for (int b = 0; b < nb; ++b) {
      if (X.size(b) == 0) continue;
      std::vector<std::pair<int64_t, int64_t>> r;
      for (int64_t k = X.ptr[b]; k < X.ptr[b + 1]; ++k) {
        int d = X.items[k];
        r.push_back({T.src_start[d], T.src_count[d]});
      }
      merge_ranges(r);
      P->p2l_box.push_back(b);
      for (auto& x : r)
        for (int64_t k = 0; k < x.second; ++k) P->p2l_idx.push_back((int)(x.first + k));
      P->p2l_ptr.push_back((int64_t)P->p2l_idx.size());
    }
  }
  // Stage 7, per child level
  P->l2l_levels.assign(T.nlevels, TileSet());
  {
    std::vector<std::vector<std::array<int, 3>>> per(T.nlevels);
    for (int b = 0; b < nb; ++b) {
      int pb = T.parent[b];
      if (pb < 0 || !Ls.is_owner[b]) continue;
      int oct = -1;
      for (int o = 0; o < 8; ++o)
        if (T.child[pb][o] == b) oct = o;
      per[T.level[b]].push_back({oct, pb, b});
    }
    P->lvl_cols = level_cols(P->prm);
    for (int l = 0; l < T.nlevels; ++l) make_tiles(per[l], P->l2l_levels[l], P->lvl_cols);
  }
  // Stages 3, 5a, 6a (near sources), 5b (W-far), 8
  P->near_ptr.assign(nb + 1, 0);
  for (int b = 0; b < nb; ++b) {
    if (Ls.is_target[b]) {
      std::vector<std::pair<int64_t, int64_t>> r;
      const int ids[3] = {gq::L_U, gq::L_WCLOSE, gq::L_XCLOSE};
      const unsigned bits[3] = {GQ_LIST_U, GQ_LIST_WCLOSE, GQ_LIST_XCLOSE};
      for (int l = 0; l < 3; ++l) {
        if (!on(bits[l])) continue;
        const auto& Lst = Ls.lst[ids[l]];
        for (int64_t k = Lst.ptr[b]; k < Lst.ptr[b + 1]; ++k) {
          int d = Lst.items[k];
          r.push_back({T.src_start[d], T.src_count[d]});
        }
      }
      merge_ranges(r);
      for (auto& x : r)
        for (int64_t k = 0; k < x.second; ++k) P->near_idx.push_back((int)(x.first + k));
      if (!r.empty()) near_center_items(T, b, P->k3_box, P->k3_c0, P->k3_nc);
      const int64_t npt_b = P->pt_count_box.empty() ? 0 : P->pt_count_box[b];
      if (npt_b > 0 && !r.empty())
        for (int64_t o = 0; o < npt_b; o += 64) {
          P->pp_box.push_back(b);
          P->pp_t0.push_back((int)(P->pt_first_box[b] + o));
          P->pp_nt.push_back((int)std::min<int64_t>(64, npt_b - o));
        }
      if (on(GQ_LIST_WFAR)) {
        const auto& W = Ls.lst[gq::L_WFAR];
        const int w0 = (int)P->wf_box.size();
        for (int64_t k = W.ptr[b]; k < W.ptr[b + 1]; ++k) P->wf_box.push_back(W.items[k]);
        const int w1 = (int)P->wf_box.size();
        // (center chunk of <= 64) x (W-far chunk of <= kWfarChunk boxes) items; a
        // deterministic plan keeps a center's whole list in one item, so that its single
        // atomic add lands on a value fixed by the stages before it
        const int kWfarChunk = (P->prm.flags & GQ_FLAG_DETERMINISTIC) ? (1 << 30) : 4;
        for (int64_t o = 0; o < T.ctr_count[b]; o += 64)
          for (int ws = w0; ws < w1; ws += kWfarChunk) {
            P->k5_c0.push_back((int)(T.ctr_start[b] + o));
            P->k5_nc.push_back((int)std::min<int64_t>(64, T.ctr_count[b] - o));
            P->k5_w0.push_back(ws);
            P->k5_w1.push_back(std::min(w1, ws + kWfarChunk));
          }
        if (w1 > w0)
          for (int64_t o = 0; o < npt_b; o += 64) {
            P->pm_t0.push_back((int)(P->pt_first_box[b] + o));
            P->pm_nt.push_back((int)std::min<int64_t>(64, npt_b - o));
            P->pm_w0.push_back(w0);
            P->pm_w1.push_back(w1);
          }
      }
      center_items(T, b, 64, P->k8_box, P->k8_c0, P->k8_nc);
    }
    P->near_ptr[b + 1] = (int64_t)P->near_idx.size();
  }
  sort_near_items(P);
  pair_center_items(P);
  P->stats.m2l_classes = (int64_t)cls_keys.size();
  // statistics
  gq_stats_t& S = P->stats;
  S.n_boxes = nb;
  S.n_levels = T.nlevels;
  for (int b = 0; b < nb; ++b) {
    if (Ls.is_target[b]) {
      S.n_target_boxes++;
      if (!T.is_leaf(b)) S.n_suspended_centers += T.ctr_count[b];
    }
    for (int l = 0; l < gq::L_NLISTS; ++l) {
      const auto& Lst = Ls.lst[l];
      int64_t ne = Lst.size(b);
      bool used = (l == gq::L_V || l == gq::L_XFAR) ? Ls.is_owner[b] : Ls.is_target[b];
      if (!used) continue;
      S.list_entries[l] += ne;
      int64_t nsrc = 0;
      for (int64_t k = Lst.ptr[b]; k < Lst.ptr[b + 1]; ++k) nsrc += T.src_count[Lst.items[k]];
      if (l == gq::L_U || l == gq::L_WCLOSE || l == gq::L_XCLOSE) S.pairs[l] += nsrc * T.ctr_count[b];
      if (l == gq::L_V) S.pairs[l] += ne;
      if (l == gq::L_WFAR) S.pairs[l] += ne * T.ctr_count[b];
      if (l == gq::L_XFAR) S.pairs[l] += nsrc;
    }
  }
  return GQ_OK;
}

// M2L by rotation: the factors A, Z, B of every class (host threads over classes), cut
// into the device tiles: the nonzero 16 x 16 tiles of the block-diagonal A and B (the same
// positions for every class, which the kernel knows at compile time) and the order blocks
// of Z.
gq_status upload_rotation(gq_plan* P, hipStream_t s) {
  const int p = P->prm.p_fmm, np = P->np;
  if (p > 15) return fail(GQ_EUNSUPPORTED, "M2L by rotation needs p_fmm <= 15");
  const int ntr = (np + 15) / 16;
  // tile positions of a matrix that is block diagonal by degree
  std::vector<int> row_beg(ntr + 1, 0), tile_c;
  for (int r = 0; r < ntr; ++r) {
    row_beg[r] = (int)tile_c.size();
    for (int c = 0; c < ntr; ++c) {
      bool nz = false;
      for (int n = 0; n <= p && !nz; ++n) {
        const int lo = n * n, hi = (n + 1) * (n + 1) - 1;
        nz = lo <= 16 * r + 15 && hi >= 16 * r && lo <= 16 * c + 15 && hi >= 16 * c;
      }
      if (nz) tile_c.push_back(c);
    }
  }
  row_beg[ntr] = (int)tile_c.size();
  const int ntile = (int)tile_c.size();
  const int kt = gq::m2l_rot_tiles(p);
  if (kt >= 0 && kt != ntile)
    return fail(GQ_EUNSUPPORTED, "rotation tile shape differs from the kernel's");
  // order blocks: m = 0 (real parts), then (m, real), (m, imaginary) for m = 1..p
  const int nblk = 2 * p + 1;
  std::vector<int> rowmap((size_t)nblk * 16, -1);
  for (int b = 0; b < nblk; ++b) {
    const int m = (b + 1) / 2, im = b > 0 && (b % 2 == 0);
    for (int n = m; n <= p; ++n) rowmap[b * 16 + n - m] = n * n + (m ? 2 * m - 1 + im : 0);
  }
  const size_t ncls = P->cls_keys.size();
  std::vector<double> hA(ncls * ntile * 256, 0.0), hB(ncls * ntile * 256, 0.0),
      hZ(ncls * nblk * 256, 0.0);
  auto work = [&](size_t c0, size_t c1) {
    std::vector<double> A((size_t)np * np), Z((size_t)np * np), B((size_t)np * np);
    for (size_t c = c0; c < c1; ++c) {
      const int key = P->cls_keys[c];
      gq::m2l_rotation_factors(p, key / 121 - 5, (key / 11) % 11 - 5, key % 11 - 5, A.data(),
                               Z.data(), B.data());
      for (int r = 0; r < ntr; ++r)
        for (int t = row_beg[r]; t < row_beg[r + 1]; ++t)
          for (int k = 0; k < 16; ++k)
            for (int i = 0; i < 16; ++i) {
              const int row = 16 * r + i, col = 16 * tile_c[t] + k;
              if (row >= np || col >= np) continue;
              // lane-major: lane 16 (k % 4) + i, k-step k / 4
              const size_t at = (c * ntile + t) * 256 + (16 * (k % 4) + i) * 4 + k / 4;
              hA[at] = A[(size_t)col * np + row];
              hB[at] = B[(size_t)col * np + row];
            }
      for (int b = 0; b < nblk; ++b)
        for (int k = 0; k < 16; ++k)
          for (int i = 0; i < 16; ++i) {
            const int row = rowmap[b * 16 + i], col = rowmap[b * 16 + k];
            if (row >= 0 && col >= 0)
              hZ[(c * nblk + b) * 256 + (16 * (k % 4) + i) * 4 + k / 4] = Z[(size_t)col * np + row];
          }
    }
  };
  const size_t nth = std::max<size_t>(1, std::min<size_t>(8, ncls / 16));
  std::vector<std::thread> th;
  for (size_t k = 0; k < nth; ++k)
    th.emplace_back(work, ncls * k / nth, ncls * (k + 1) / nth);
  for (auto& x : th) x.join();
  GQ_TRY(upload(P, hA, &P->R_A, s));
  GQ_TRY(upload(P, hZ, &P->R_Z, s));
  GQ_TRY(upload(P, hB, &P->R_B, s));
  GQ_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
  P->rot = gq::RotMats{P->R_A, P->R_Z, P->R_B};
  return GQ_OK;
}

// Translation matrices for the plan's classes and the upload of every work list.
gq_status upload_work(gq_plan* P) {
  if (P->prm.flags & GQ_FLAG_HOST_ONLY) return GQ_OK;
  const gq::Tree& T = P->tree;
  const std::vector<int>& cls_keys = P->cls_keys;
  // translation matrices
  const int p = P->prm.p_fmm, np = P->np;
  std::vector<double> Tm((size_t)8 * np * np), Tl((size_t)8 * np * np);
  for (int o = 0; o < 8; ++o) {
    gq::m2m_matrix(p, o, Tm.data() + (size_t)o * np * np);
    gq::l2l_matrix(p, o, Tl.data() + (size_t)o * np * np);
  }
  const bool rot = P->prm.m2l_rotation != 0;
  std::vector<double> Tv(rot ? 0 : (size_t)cls_keys.size() * np * np);
  if (!rot)
    for (size_t c = 0; c < cls_keys.size(); ++c) {
      int key = cls_keys[c];
      gq::m2l_matrix(p, key / 121 - 5, (key / 11) % 11 - 5, key % 11 - 5, Tv.data() + c * np * np);
    }

  hipStream_t s = P->last_stream;
  // device layout: padded column-major (trans_ld rows, trans_kd columns, zero padding)
  auto pad = [&](std::vector<double>& T) {
    const int ld = gq::trans_ld(np), kd = gq::trans_kd(np);
    const size_t nm = T.size() / ((size_t)np * np);
    std::vector<double> out(nm * ld * kd, 0.0);
    for (size_t m = 0; m < nm; ++m)
      for (int c = 0; c < np; ++c)
        for (int r = 0; r < np; ++r)
          out[m * ld * kd + (size_t)c * ld + r] = T[m * np * np + (size_t)c * np + r];
    T.swap(out);
  };
  pad(Tm);
  pad(Tl);
  pad(Tv);
  if (P->prm.precision == GQ_FP64) {
    GQ_TRY(upload(P, Tm, &P->T_m2m, s));
    GQ_TRY(upload(P, Tl, &P->T_l2l, s));
    GQ_TRY(upload(P, Tv, &P->T_m2l, s));
  } else {
    // Balanced FP32 forms T^ = diag(1 / s_out) T diag(1 / s_in) (N = sqrt((n+m)! (n-m)!);
    // multipoles in, s_in = N; locals in, 1 / N; multipoles out, s_out = 1 / N; locals
    // out, N), split as T^ = hi + lo with hi = fl32(T^), lo = fl32(T^ - hi); the first
    // kLeadCols columns are also kept in FP64 for the modes that contract them exactly.
    std::vector<double> N(np), Ni(np);
    gq::expansion_norms(p, N.data());
    for (int i = 0; i < np; ++i) Ni[i] = 1.0 / N[i];
    GQ_TRY(upload(P, N, &P->d_norm, s));
    GQ_TRY(upload(P, Ni, &P->d_inorm, s));
    const int prec = P->prm.precision;
    const bool lead = prec == GQ_FP32_SPLIT || prec == GQ_FP32_LEAD;
    const int ld = gq::trans_ld(np), kd = gq::trans_kd(np), nl = gq::kLeadCols;
    auto split = [&](const std::vector<double>& T64, const std::vector<double>& sin,
                     const std::vector<double>& sout, float** d, double** dl) -> gq_status {
      const size_t nm = T64.size() / ((size_t)ld * kd);
      std::vector<float> hi(T64.size()), lo(prec == GQ_FP32_SPLIT ? T64.size() : 0);
      std::vector<double> lh(lead ? nm * nl * ld : 0, 0.0);
      for (size_t m = 0; m < nm; ++m)
        for (int c = 0; c < kd; ++c)
          for (int r = 0; r < ld; ++r) {
            const size_t i = m * ld * kd + (size_t)c * ld + r;
            const double v = (c < np && r < np) ? T64[i] / (sout[r] * sin[c]) : 0.0;
            hi[i] = (float)v;
            if (!lo.empty()) lo[i] = (float)(v - (double)hi[i]);
            if (lead && c < nl) lh[(m * nl + c) * ld + r] = v;
          }
      GQ_TRY(upload(P, hi, &d[0], s));
      GQ_TRY(upload(P, lo, &d[1], s));
      GQ_TRY(upload(P, lh, dl, s));
      GQ_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
      return GQ_OK;
    };
    GQ_TRY(split(Tm, N, Ni, P->T32_m2m, &P->Tlead_m2m));
    GQ_TRY(split(Tl, Ni, N, P->T32_l2l, &P->Tlead_l2l));
    GQ_TRY(split(Tv, N, N, P->T32_m2l, &P->Tlead_m2l));
  }
  P->tm_m2m = {P->T_m2m, P->T32_m2m[0], P->T32_m2m[1], P->Tlead_m2m, P->d_norm, P->d_inorm};
  P->tm_l2l = {P->T_l2l, P->T32_l2l[0], P->T32_l2l[1], P->Tlead_l2l, P->d_inorm, P->d_norm};
  P->tm_m2l = {P->T_m2l, P->T32_m2l[0], P->T32_m2l[1], P->Tlead_m2l, P->d_norm, P->d_norm};
  if (rot) GQ_TRY(upload_rotation(P, s));
  GQ_TRY(upload(P, P->p2m_boxes, &P->d_p2m_boxes, s));
  GQ_TRY(upload(P, P->p2m_ptr, &P->d_p2m_ptr, s));
  GQ_TRY(upload(P, P->p2m_idx, &P->d_p2m_idx, s));
  auto up_tiles = [&](const TileSet& t, std::array<int*, 5>& d) -> gq_status {
    GQ_TRY(upload(P, t.cls, &d[0], s));
    GQ_TRY(upload(P, t.beg, &d[1], s));
    GQ_TRY(upload(P, t.cnt, &d[2], s));
    GQ_TRY(upload(P, t.src, &d[3], s));
    GQ_TRY(upload(P, t.dst, &d[4], s));
    return GQ_OK;
  };
  P->d_m2m.assign(T.nlevels, {});
  P->d_l2l.assign(T.nlevels, {});
  for (int l = 0; l < T.nlevels; ++l) {
    GQ_TRY(up_tiles(P->m2m_levels[l], P->d_m2m[l]));
    GQ_TRY(up_tiles(P->l2l_levels[l], P->d_l2l[l]));
  }
  GQ_TRY(up_tiles(P->m2l, P->d_m2l));
  GQ_TRY(upload(P, P->p2l_box, &P->d_p2l_box, s));
  GQ_TRY(upload(P, P->p2l_ptr, &P->d_p2l_ptr, s));
  GQ_TRY(upload(P, P->p2l_idx, &P->d_p2l_idx, s));
  GQ_TRY(upload(P, P->near_ptr, &P->d_near_ptr, s));
  GQ_TRY(upload(P, P->near_idx, &P->d_near_idx, s));
  GQ_TRY(upload(P, P->k3_box, &P->d_k3_box, s));
  GQ_TRY(upload(P, P->k3_c0, &P->d_k3_c0, s));
  GQ_TRY(upload(P, P->k3_nc, &P->d_k3_nc, s));
  GQ_TRY(upload(P, P->wf_box, &P->d_wf_box, s));
  GQ_TRY(upload(P, P->k5_c0, &P->d_k5_c0, s));
  GQ_TRY(upload(P, P->k5_nc, &P->d_k5_nc, s));
  GQ_TRY(upload(P, P->k5_w0, &P->d_k5_w0, s));
  GQ_TRY(upload(P, P->k5_w1, &P->d_k5_w1, s));
  GQ_TRY(upload(P, P->k8_box, &P->d_k8_box, s));
  GQ_TRY(upload(P, P->k8_c0, &P->d_k8_c0, s));
  GQ_TRY(upload(P, P->k8_nc, &P->d_k8_nc, s));
  GQ_TRY(upload(P, P->pp_box, &P->d_pp_box, s));
  GQ_TRY(upload(P, P->pp_t0, &P->d_pp_t0, s));
  GQ_TRY(upload(P, P->pp_nt, &P->d_pp_nt, s));
  GQ_TRY(upload(P, P->pm_t0, &P->d_pm_t0, s));
  GQ_TRY(upload(P, P->pm_nt, &P->d_pm_nt, s));
  GQ_TRY(upload(P, P->pm_w0, &P->d_pm_w0, s));
  GQ_TRY(upload(P, P->pm_w1, &P->d_pm_w1, s));
  GQ_HIP(hipStreamSynchronize(s));  // the matrices above are host temporaries
  return GQ_OK;
}


// GQ_FLAG_DETERMINISTIC: for every tile set, its destinations and the positions of their
// pairs in ascending order, and one slot buffer for the largest tile set.  Pair positions
// follow the class order of make_tiles (a stable sort), whatever the tile width, so the
// sums are the same for every tile shape the autotuner may pick.  Called once the M2L
// tiles are final.
gq_status upload_slot_sums(gq_plan* P) {
  if (!(P->prm.flags & GQ_FLAG_DETERMINISTIC) || (P->prm.flags & GQ_FLAG_HOST_ONLY))
    return GQ_OK;
  hipStream_t s = P->last_stream;
  int64_t most = 0;
  std::vector<std::vector<int>> keep_i;  // host copies alive until the uploads complete
  std::vector<std::vector<int64_t>> keep_p;
  auto one = [&](const TileSet& t, gq_plan::SlotSum& out) -> gq_status {
    const int n = (int)t.dst.size();
    most = std::max<int64_t>(most, n);
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return t.dst[a] < t.dst[b]; });
    std::vector<int> dst;
    std::vector<int64_t> ptr;
    for (int i = 0; i < n; ++i)
      if (i == 0 || t.dst[ord[i]] != t.dst[ord[i - 1]]) {
        dst.push_back(t.dst[ord[i]]);
        ptr.push_back(i);
      }
    ptr.push_back(n);
    out.ndst = (int)dst.size();
    GQ_TRY(upload(P, dst, &out.dst, s));
    GQ_TRY(upload(P, ptr, &out.ptr, s));
    GQ_TRY(upload(P, ord, &out.pair, s));
    keep_i.push_back(std::move(dst));
    keep_i.push_back(std::move(ord));
    keep_p.push_back(std::move(ptr));
    return GQ_OK;
  };
  const int nl = P->tree.nlevels;
  P->ss_m2m.assign(nl, {});
  P->ss_l2l.assign(nl, {});
  for (int l = 0; l < nl; ++l) {
    GQ_TRY(one(P->m2m_levels[l], P->ss_m2m[l]));
    GQ_TRY(one(P->l2l_levels[l], P->ss_l2l[l]));
  }
  GQ_TRY(one(P->m2l, P->ss_m2l));
  GQ_TRY(alloc(P, (size_t)most * P->np, &P->slots));
  GQ_HIP(hipStreamSynchronize(s));
  P->det = true;
  return GQ_OK;
}

// ------------------------------------------------------------------------------------
// Batches: several plans merged into one plan whose stages each run as one launch over
// every member's work.  Box, source, center and target indices of member k are shifted by
// the member totals before it; M2L tiles are re-formed over the union of the members'
// offset classes, so members share translation matrices and fill tiles together.
// ------------------------------------------------------------------------------------

template <class T>
void append_shifted(std::vector<T>& dst, const std::vector<T>& src, T shift) {
  for (const T& v : src) dst.push_back(v + shift);
}

// ptr: CSR offsets (size n+1) of member items appended after `base` existing items
void append_ptr(std::vector<int64_t>& dst, const std::vector<int64_t>& src, int64_t base) {
  for (size_t i = 1; i < src.size(); ++i) dst.push_back(base + src[i]);
}

void tiles_to_pairs(const TileSet& t, int shift, const std::vector<int>* cls_map,
                    std::vector<std::array<int, 3>>& out) {
  for (int i = 0; i < t.ntile(); ++i) {
    const int c = cls_map ? (*cls_map)[t.cls[i]] : t.cls[i];
    for (int j = t.beg[i]; j < t.beg[i] + t.cnt[i]; ++j)
      out.push_back({c, t.src[j] + shift, t.dst[j] + shift});
  }
}

gq_status merge_plans(gq_plan* B, gq_plan* const* plans, int n) {
  gq::Tree& TB = B->tree;
  int nlev = 0;
  for (int k = 0; k < n; ++k) nlev = std::max(nlev, plans[k]->tree.nlevels);
  TB.nlevels = nlev;
  std::vector<std::vector<std::array<int, 3>>> m2m(nlev), l2l(nlev);
  std::vector<std::array<int, 3>> m2l;
  std::map<int, int> cls_index;
  B->p2m_ptr.push_back(0);
  B->p2l_ptr.push_back(0);
  B->near_ptr.push_back(0);
  int64_t boff = 0, soff = 0, coff = 0, toff = 0, poff = 0;
  int woff = 0;
  gq_stats_t& S = B->stats;
  for (int k = 0; k < n; ++k) {
    const gq_plan* P = plans[k];
    const gq::Tree& T = P->tree;
    const int bo = (int)boff, co = (int)coff;
    TB.center.insert(TB.center.end(), T.center.begin(), T.center.end());
    TB.h.insert(TB.h.end(), T.h.begin(), T.h.end());
    append_shifted(TB.src_order, T.src_order, soff);  // index into the concatenated density
    append_shifted(B->h_tgt_ctr, P->h_tgt_ctr, coff);
    append_shifted(B->h_tgt_out, P->h_tgt_out, toff);
    // Stage 2a and 6b source ranges
    append_ptr(B->p2m_ptr, P->p2m_ptr, (int64_t)B->p2m_idx.size());
    append_shifted(B->p2m_boxes, P->p2m_boxes, bo);
    append_shifted(B->p2m_idx, P->p2m_idx, (int)soff);
    append_ptr(B->p2l_ptr, P->p2l_ptr, (int64_t)B->p2l_idx.size());
    append_shifted(B->p2l_box, P->p2l_box, bo);
    append_shifted(B->p2l_idx, P->p2l_idx, (int)soff);
    // translations: M2M/L2L by level, M2L by offset class
    for (int l = 0; l < T.nlevels; ++l) {
      tiles_to_pairs(P->m2m_levels[l], bo, nullptr, m2m[l]);
      tiles_to_pairs(P->l2l_levels[l], bo, nullptr, l2l[l]);
    }
    std::vector<int> cmap(P->cls_keys.size());
    for (size_t c = 0; c < P->cls_keys.size(); ++c) {
      auto it = cls_index.find(P->cls_keys[c]);
      if (it == cls_index.end()) {
        it = cls_index.emplace(P->cls_keys[c], (int)B->cls_keys.size()).first;
        B->cls_keys.push_back(P->cls_keys[c]);
      }
      cmap[c] = it->second;
    }
    tiles_to_pairs(P->m2l, bo, &cmap, m2l);
    // near field, W-far, L2QBXL items
    append_ptr(B->near_ptr, P->near_ptr, (int64_t)B->near_idx.size());
    append_shifted(B->near_idx, P->near_idx, (int)soff);
    append_shifted(B->k3_box, P->k3_box, bo);
    append_shifted(B->k3_c0, P->k3_c0, co);
    B->k3_nc.insert(B->k3_nc.end(), P->k3_nc.begin(), P->k3_nc.end());
    append_shifted(B->wf_box, P->wf_box, bo);
    append_shifted(B->k5_c0, P->k5_c0, co);
    B->k5_nc.insert(B->k5_nc.end(), P->k5_nc.begin(), P->k5_nc.end());
    append_shifted(B->k5_w0, P->k5_w0, woff);
    append_shifted(B->k5_w1, P->k5_w1, woff);
    append_shifted(B->k8_box, P->k8_box, bo);
    append_shifted(B->k8_c0, P->k8_c0, co);
    B->k8_nc.insert(B->k8_nc.end(), P->k8_nc.begin(), P->k8_nc.end());
    // conventional targets
    append_shifted(B->h_pt_in, P->h_pt_in, toff);  // output index in the batch
    append_shifted(B->h_pt_box, P->h_pt_box, bo);
    append_shifted(B->pp_box, P->pp_box, bo);
    append_shifted(B->pp_t0, P->pp_t0, (int)poff);
    B->pp_nt.insert(B->pp_nt.end(), P->pp_nt.begin(), P->pp_nt.end());
    append_shifted(B->pm_t0, P->pm_t0, (int)poff);
    B->pm_nt.insert(B->pm_nt.end(), P->pm_nt.begin(), P->pm_nt.end());
    append_shifted(B->pm_w0, P->pm_w0, woff);
    append_shifted(B->pm_w1, P->pm_w1, woff);
    // statistics
    const gq_stats_t& Q = P->stats;
    S.n_sources += Q.n_sources;
    S.n_centers += Q.n_centers;
    S.n_targets += Q.n_targets;
    S.n_boxes += Q.n_boxes;
    S.n_target_boxes += Q.n_target_boxes;
    S.n_suspended_centers += Q.n_suspended_centers;
    for (int l = 0; l < 6; ++l) {
      S.list_entries[l] += Q.list_entries[l];
      S.pairs[l] += Q.pairs[l];
    }
    boff += T.nboxes;
    soff += P->n_src;
    coff += P->n_ctr;
    toff += P->n_tgt;
    poff += P->n_pt;
    woff += (int)P->wf_box.size();
  }
  if (boff > INT32_MAX || soff > INT32_MAX || coff > INT32_MAX)
    return fail(GQ_EUNSUPPORTED, "batch exceeds 2^31 boxes, sources or centers");
  TB.nboxes = (int)boff;
  B->n_pt = poff;
  S.n_levels = nlev;
  S.m2l_classes = (int64_t)B->cls_keys.size();
  B->m2m_levels.assign(nlev, TileSet());
  B->l2l_levels.assign(nlev, TileSet());
  B->lvl_cols = level_cols(B->prm);
  for (int l = 0; l < nlev; ++l) {
    make_tiles(m2m[l], B->m2m_levels[l], B->lvl_cols);
    make_tiles(l2l[l], B->l2l_levels[l], B->lvl_cols);
  }
  B->m2l_cols = default_m2l_cols(B->prm);
  make_tiles(m2l, B->m2l, B->m2l_cols);
  sort_near_items(B);
  pair_center_items(B);
  return GQ_OK;
}

// Device geometry of a merged plan: member arrays copied device to device.
gq_status merge_geometry(gq_plan* B, gq_plan* const* plans, int n, hipStream_t s) {
  struct Field {
    double* gq_plan::*arr;
    int which;  // 0 sources, 1 centers, 2 targets
  };
  const Field fields[] = {{&gq_plan::sx, 0}, {&gq_plan::sy, 0}, {&gq_plan::sz, 0},
                          {&gq_plan::snx, 0}, {&gq_plan::sny, 0}, {&gq_plan::snz, 0},
                          {&gq_plan::sw, 0}, {&gq_plan::cx, 1}, {&gq_plan::cy, 1},
                          {&gq_plan::cz, 1}, {&gq_plan::tx, 2}, {&gq_plan::ty, 2},
                          {&gq_plan::tz, 2}};
  for (const Field& f : fields) {
    // targets: the QBX targets only (point targets are copied below)
    const int64_t total = f.which == 0 ? B->n_src : f.which == 1 ? B->n_ctr : B->n_qt;
    GQ_TRY(alloc(B, (size_t)total, &(B->*f.arr)));
    int64_t off = 0;
    for (int k = 0; k < n; ++k) {
      const gq_plan* P = plans[k];
      const int64_t m = f.which == 0 ? P->n_src : f.which == 1 ? P->n_ctr : P->n_qt;
      if (m > 0)
        GQ_HIP(hipMemcpyAsync(B->*f.arr + off, P->*f.arr, (size_t)m * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
      off += m;
    }
  }
  const gq::Tree& T = B->tree;
  if (B->prm.kernel == GQ_KERNEL_SP && B->n_qt > 0) {
    double* gq_plan::*nf[3] = {&gq_plan::tnx, &gq_plan::tny, &gq_plan::tnz};
    for (auto f : nf) {
      GQ_TRY(alloc(B, (size_t)B->n_qt, &(B->*f)));
      int64_t off = 0;
      for (int k = 0; k < n; ++k) {
        if (plans[k]->n_qt > 0 && !(plans[k]->*f))
          return fail(GQ_EINVAL, "S' batch member without target normals");
        if (plans[k]->n_qt > 0)
          GQ_HIP(hipMemcpyAsync(B->*f + off, plans[k]->*f, (size_t)plans[k]->n_qt * sizeof(double),
                                hipMemcpyDeviceToDevice, s));
        off += plans[k]->n_qt;
      }
    }
  }
  if (B->n_pt > 0) {
    double* gq_plan::*pf[3] = {&gq_plan::px, &gq_plan::py, &gq_plan::pz};
    for (auto f : pf) {
      GQ_TRY(alloc(B, (size_t)B->n_pt, &(B->*f)));
      int64_t off = 0;
      for (int k = 0; k < n; ++k) {
        if (plans[k]->n_pt > 0)
          GQ_HIP(hipMemcpyAsync(B->*f + off, plans[k]->*f, (size_t)plans[k]->n_pt * sizeof(double),
                                hipMemcpyDeviceToDevice, s));
        off += plans[k]->n_pt;
      }
    }
    GQ_TRY(upload(B, B->h_pt_box, &B->d_pt_box, s));
    GQ_TRY(upload(B, B->h_pt_in, &B->d_pt_out, s));
    GQ_TRY(alloc(B, (size_t)B->n_pt, &B->phi));
  }
  GQ_TRY(upload(B, T.src_order, &B->src_order, s));
  GQ_TRY(upload(B, B->h_tgt_ctr, &B->tgt_ctr, s));
  GQ_TRY(upload(B, B->h_tgt_out, &B->tgt_out, s));
  GQ_TRY(upload(B, T.center, &B->bctr, s));
  GQ_TRY(upload(B, T.h, &B->bh, s));
  B->nbuf = near_field_densities(B->prm);
  GQ_TRY(alloc(B, (size_t)B->n_src * B->nbuf, &B->q));
  GQ_TRY(alloc(B, (size_t)T.nboxes * B->np, &B->M));
  GQ_TRY(alloc(B, (size_t)T.nboxes * B->np, &B->L));
  GQ_TRY(alloc(B, (size_t)B->n_ctr * B->nq * B->nbuf, &B->Lq));
  GQ_HIP(hipStreamSynchronize(s));
  return GQ_OK;
}

// GQ_FLAG_AUTOTUNE: time the M2L launch (Stage 4) on this plan's own tiles for tile widths
// 64 and 32 and for XCD-aware or plain tile order, and keep the fastest.  The timed
// launches read zeroed multipoles; the box locals are cleared by every apply.
gq_status autotune_m2l(gq_plan* P, hipStream_t s) {
  if (P->m2l.ntile() == 0 || P->prm.m2l_rotation) return GQ_OK;  // one rotation kernel shape
  std::vector<std::array<int, 3>> pairs;
  tiles_to_pairs(P->m2l, 0, nullptr, pairs);
  struct Cand {
    TileSet ts;
    std::array<int*, 5> d{};
  } cand[2];
  const int widths[2] = {64, 32};
  for (int w = 0; w < 2; ++w) {
    make_tiles(pairs, cand[w].ts, widths[w]);
    const TileSet& t = cand[w].ts;
    GQ_TRY(upload(P, t.cls, &cand[w].d[0], s));
    GQ_TRY(upload(P, t.beg, &cand[w].d[1], s));
    GQ_TRY(upload(P, t.cnt, &cand[w].d[2], s));
    GQ_TRY(upload(P, t.src, &cand[w].d[3], s));
    GQ_TRY(upload(P, t.dst, &cand[w].d[4], s));
  }
  gq::launch_fill(s, P->M, (int64_t)P->tree.nboxes * P->np, 0.0);
  gq::launch_fill(s, P->L, (int64_t)P->tree.nboxes * P->np, 0.0);
  hipEvent_t e0, e1;
  GQ_HIP(hipEventCreate(&e0));
  GQ_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int bw = 0;
  bool bx = true;
  gq_status st = GQ_OK;
  for (int w = 0; w < 2 && st == GQ_OK; ++w)
    for (int x = 0; x < 2; ++x) {
      const bool xcd = x == 0;
      auto run = [&]() {
        const auto& d = cand[w].d;
        gq::launch_translate(s, 2, P->prm.precision, P->np, cand[w].ts.ntile(), d[0], d[1], d[2],
                             d[3], d[4], P->tm_m2l, P->M, P->L, widths[w], xcd);
      };
      run();  // warm-up
      hipError_t e = hipEventRecord(e0, s);
      for (int r = 0; r < 3; ++r) run();
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        st = fail(GQ_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
        break;
      }
      if (ms < best) {
        best = ms;
        bw = w;
        bx = xcd;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != GQ_OK) return st;
  P->m2l = cand[bw].ts;
  P->d_m2l = cand[bw].d;
  P->m2l_cols = widths[bw];
  P->m2l_xcd = bx;
  return GQ_OK;
}

// Uniform cell grid over [lo, hi] whose cells are at least `reach` wide (slightly more, so
// that a point within reach of a query lies in the 27 cells around the query's cell even
// after rounding), with at most max_cells cells.
gq::AssocGrid make_grid(const double lo[3], const double hi[3], double reach,
                        int64_t max_cells = (int64_t)1 << 24) {
  const double extent = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
  gq::AssocGrid g{};
  g.h = reach * (1.0 + 1e-9) + extent * 1e-12;
  if (!(g.h > 0)) g.h = 1.0;
  for (;;) {
    int64_t cells = 1;
    for (int a = 0; a < 3; ++a) {
      g.lo[a] = lo[a];
      g.n[a] = (int)std::min<double>(std::floor((hi[a] - lo[a]) / g.h) + 1.0, 1 << 24);
      cells *= g.n[a];
    }
    if (cells <= max_cells) break;
    g.h *= 1.25;  // wider cells only add candidates; reach is unchanged
  }
  return g;
}

int64_t grid_cell(const gq::AssocGrid& g, const double* p) {
  int64_t c[3];
  for (int a = 0; a < 3; ++a) {
    int64_t i = (int64_t)std::floor((p[a] - g.lo[a]) / g.h);
    c[a] = i < 0 ? 0 : (i >= g.n[a] ? g.n[a] - 1 : i);
  }
  return (c[2] * g.n[1] + c[1]) * g.n[0] + c[0];
}

}  // namespace

namespace gq {

gq_status set_error(gq_status st, const std::string& msg) { return fail(st, msg); }

gq_status near_prepare(int64_t n_q, const double* q_xyz, const double* radius, int64_t n_p,
                       const double* p_xyz, uint8_t* hit, int64_t max_cells, NearQuery& Q,
                       bool& done) {
  done = false;
  if (n_q < 0 || n_p < 0) return fail(GQ_EINVAL, "negative count");
  if ((n_q && (!q_xyz || !radius || !hit)) || (n_p && !p_xyz))
    return fail(GQ_EINVAL, "NULL array with a nonzero count");
  if (!finite3(q_xyz, n_q) || !finite3(p_xyz, n_p)) return fail(GQ_EINVAL, "non-finite coordinate");
  double rmax = 0.0;
  for (int64_t i = 0; i < n_q; ++i) {
    if (!std::isfinite(radius[i]) || radius[i] < 0)
      return fail(GQ_EINVAL, "radii must be finite and >= 0");
    rmax = std::max(rmax, radius[i]);
  }
  if (n_q + n_p >= ((int64_t)1 << 31)) return fail(GQ_EUNSUPPORTED, "more than 2^31 points");
  if (n_q == 0) {
    done = true;
    return GQ_OK;
  }
  if (n_p == 0) {
    std::fill(hit, hit + n_q, (uint8_t)0);
    done = true;
    return GQ_OK;
  }
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) lo[a] = hi[a] = q_xyz[a];
  for (const double* pp : {q_xyz, p_xyz}) {
    const int64_t n = pp == q_xyz ? n_q : n_p;
    for (int64_t i = 0; i < n; ++i)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], pp[3 * i + a]);
        hi[a] = std::max(hi[a], pp[3 * i + a]);
      }
  }
  Q.g = make_grid(lo, hi, rmax, max_cells);
  const gq::AssocGrid& g = Q.g;
  const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
  Q.start.assign(ncell + 1, 0);
  std::vector<int64_t> cell(n_p);
  for (int64_t i = 0; i < n_p; ++i) {
    cell[i] = grid_cell(g, p_xyz + 3 * i);
    Q.start[cell[i] + 1] += 1;
  }
  for (int64_t c = 0; c < ncell; ++c) Q.start[c + 1] += Q.start[c];
  std::vector<int64_t> fill(Q.start.begin(), Q.start.end() - 1);
  Q.px.resize(n_p);
  Q.py.resize(n_p);
  Q.pz.resize(n_p);
  for (int64_t i = 0; i < n_p; ++i) {
    const int64_t k = fill[cell[i]]++;
    Q.px[k] = p_xyz[3 * i];
    Q.py[k] = p_xyz[3 * i + 1];
    Q.pz[k] = p_xyz[3 * i + 2];
  }
  Q.qx.resize(n_q);
  Q.qy.resize(n_q);
  Q.qz.resize(n_q);
  for (int64_t i = 0; i < n_q; ++i) {
    Q.qx[i] = q_xyz[3 * i];
    Q.qy[i] = q_xyz[3 * i + 1];
    Q.qz[i] = q_xyz[3 * i + 2];
  }
  return GQ_OK;
}

}  // namespace gq

extern "C" {

const char* gq_last_error(void) { return g_err.c_str(); }

// One plan with the given parameters (gq_plan_create without GQ_FLAG_AUTOTUNE_TREE).
static gq_status create_plan(const gq_params* prm, int64_t n_src, const double* src_xyz,
                             const double* src_w, const double* src_normal, int64_t n_ctr,
                             const double* ctr_xyz, const double* ctr_radius, int64_t n_tgt,
                             const double* tgt_xyz, const int64_t* tgt_center,
                             void* hip_stream, gq_plan** out) {
  g_err.clear();
  auto t0 = std::chrono::steady_clock::now();
  if (!prm || !out) return fail(GQ_EINVAL, "params and out must not be NULL");
  if (n_src < 0 || n_ctr < 0 || n_tgt < 0) return fail(GQ_EINVAL, "negative count");
  if (n_src == 0 || n_ctr == 0) return fail(GQ_EINVAL, "need at least one source and one center");
  if ((n_src && (!src_xyz || !src_w)) || (n_ctr && (!ctr_xyz || !ctr_radius)) ||
      (n_tgt && (!tgt_xyz || !tgt_center)))
    return fail(GQ_EINVAL, "NULL input array");
  if (prm->p_qbx < 0 || prm->p_fmm < 0) return fail(GQ_EINVAL, "negative order");
  if (prm->p_qbx > prm->p_fmm) return fail(GQ_EINVAL, "p_qbx must not exceed p_fmm");
  if (prm->p_fmm > gq::kPmax || prm->p_qbx > gq::kQmax)
    return fail(GQ_EUNSUPPORTED, "order beyond this build's limits (p_fmm <= 20, p_qbx <= 10)");
  if (prm->nmax < 1) return fail(GQ_EINVAL, "nmax must be >= 1");
  if (!(prm->tcf >= 0.0 && prm->tcf < 2.0 * std::sqrt(3.0) - 2.0))
    return fail(GQ_EINVAL, "target confinement factor outside [0, 2 sqrt(3) - 2)");
  if (prm->kernel != GQ_KERNEL_S && prm->kernel != GQ_KERNEL_D && prm->kernel != GQ_KERNEL_SP)
    return fail(GQ_EINVAL, "unknown kernel");
  if (prm->precision != GQ_FP64 && prm->precision != GQ_FP32_SPLIT && prm->precision != GQ_FP32 &&
      prm->precision != GQ_FP32_LEAD)
    return fail(GQ_EINVAL, "unknown precision");
  if (prm->n_densities < 1) return fail(GQ_EINVAL, "n_densities must be >= 1");
  if (prm->wfar_direct_max < 0) return fail(GQ_EINVAL, "wfar_direct_max must be >= 0");
  if (prm->tcr_norm != 0 && prm->tcr_norm != 1) return fail(GQ_EINVAL, "tcr_norm must be 0 or 1");
  if (prm->level_restrict != 0 && prm->level_restrict != 1)
    return fail(GQ_EINVAL, "level_restrict must be 0 or 1");
  if (prm->m2l_rotation != 0 && prm->m2l_rotation != 1)
    return fail(GQ_EINVAL, "m2l_rotation must be 0 or 1");
  if (prm->max_device_bytes < 0) return fail(GQ_EINVAL, "max_device_bytes must be >= 0");
  if (prm->m2l_rotation && (prm->precision != GQ_FP64 || prm->p_fmm > 15))
    return fail(GQ_EUNSUPPORTED, "M2L by rotation needs GQ_FP64 and p_fmm <= 15");
  if ((prm->flags & GQ_FLAG_TIMING) && (prm->flags & GQ_FLAG_GRAPH))
    return fail(GQ_EINVAL, "GQ_FLAG_TIMING and GQ_FLAG_GRAPH are exclusive");
  if ((prm->flags & GQ_FLAG_AUTOTUNE_TREE) && (prm->flags & GQ_FLAG_HOST_ONLY))
    return fail(GQ_EINVAL, "GQ_FLAG_AUTOTUNE_TREE needs a device plan, not a host-only one");
  if (prm->kernel == GQ_KERNEL_D && !src_normal) return fail(GQ_EINVAL, "double layer needs normals");
  if (!finite3(src_xyz, n_src) || !finite3(ctr_xyz, n_ctr) || !finite3(tgt_xyz, n_tgt))
    return fail(GQ_EINVAL, "non-finite coordinates");
  for (int64_t i = 0; i < n_src; ++i)
    if (!std::isfinite(src_w[i])) return fail(GQ_EINVAL, "non-finite weight");
  for (int64_t i = 0; i < n_ctr; ++i)
    if (!(ctr_radius[i] > 0.0) || !std::isfinite(ctr_radius[i]))
      return fail(GQ_EINVAL, "center radius must be positive and finite");
  for (int64_t i = 0; i < n_tgt; ++i)
    if (tgt_center[i] < -1 || tgt_center[i] >= n_ctr) return fail(GQ_EINVAL, "tgt_center out of range");
  if (src_normal) {
    if (!finite3(src_normal, n_src)) return fail(GQ_EINVAL, "non-finite normal");
    for (int64_t i = 0; i < n_src; ++i) {
      const double* nn = src_normal + 3 * i;
      double l = std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
      if (std::fabs(l - 1.0) > 1e-6) return fail(GQ_EINVAL, "normals must have unit length");
    }
  }
  gq_plan* P = new (std::nothrow) gq_plan();
  if (!P) return fail(GQ_ENOMEM, "host allocation failed");
  P->prm = *prm;
  P->np = gq::ncoef(prm->p_fmm);
  P->nq = gq::ncoef(prm->p_qbx);
  P->n_src = n_src;
  P->n_ctr = n_ctr;
  P->n_tgt = n_tgt;
  P->last_stream = (hipStream_t)hip_stream;
  gq::TreeParams tp;
  tp.nmax = prm->nmax;
  tp.tcf = prm->tcf;
  tp.tcr_linf = prm->tcr_norm == 1;
  tp.level_restrict = prm->level_restrict == 1;
  std::string msg = gq::build_tree(tp, n_src, src_xyz, n_ctr, ctr_xyz, ctr_radius, n_tgt,
                                   tgt_xyz, P->tree);
  if (!msg.empty()) {
    delete P;
    return fail(GQ_EINVAL, msg);
  }
  {
    // conventional targets (tgt_center < 0), grouped by the box that owns them
    const gq::Tree& T0 = P->tree;
    P->pt_count_box.assign(T0.nboxes, 0);
    P->pt_first_box.assign(T0.nboxes, 0);
    for (int b : T0.preorder) {
      P->pt_first_box[b] = (int64_t)P->h_pt_in.size();
      for (int64_t k = T0.tgt_start[b]; k < T0.tgt_start[b] + T0.tgt_count[b]; ++k) {
        const int64_t j = T0.tgt_order[k];
        if (tgt_center[j] >= 0) continue;
        P->h_pt_in.push_back(j);
        P->h_pt_box.push_back(b);
        P->pt_count_box[b] += 1;
      }
    }
    P->n_pt = (int64_t)P->h_pt_in.size();
    P->n_qt = n_tgt - P->n_pt;
    if (P->n_pt > 0 && prm->kernel == GQ_KERNEL_SP) {
      delete P;
      return fail(GQ_EUNSUPPORTED, "S' is evaluated at QBX targets only (tgt_center >= 0)");
    }
    if (P->n_pt > INT32_MAX) {
      delete P;
      return fail(GQ_EUNSUPPORTED, "more than 2^31 point targets");
    }
  }
  gq::build_lists(P->tree, prm->tcf, prm->wfar_direct_max, P->lists, tp.tcr_linf,
                  &P->pt_count_box);
  P->stats.n_sources = n_src;
  P->stats.n_centers = n_ctr;
  P->stats.n_targets = n_tgt;
  gq_status st = build_work(P);
  if (st == GQ_OK) st = upload_work(P);
  if (st != GQ_OK) {
    delete P;
    return st;
  }
  if (!(prm->flags & GQ_FLAG_HOST_ONLY)) {
    const gq::Tree& T = P->tree;
    hipStream_t s = P->last_stream;
    // particles in tree order
    std::vector<double> a(n_src), b(n_src), c(n_src), na(n_src, 0.0), nb(n_src, 0.0),
        nc(n_src, 0.0), w(n_src);
    for (int64_t i = 0; i < n_src; ++i) {
      int64_t j = T.src_order[i];
      a[i] = src_xyz[3 * j];
      b[i] = src_xyz[3 * j + 1];
      c[i] = src_xyz[3 * j + 2];
      w[i] = src_w[j];
      if (src_normal) {
        na[i] = src_normal[3 * j];
        nb[i] = src_normal[3 * j + 1];
        nc[i] = src_normal[3 * j + 2];
      }
    }
    auto go = [&]() -> gq_status {
      GQ_TRY(upload(P, a, &P->sx, s));
      GQ_TRY(upload(P, b, &P->sy, s));
      GQ_TRY(upload(P, c, &P->sz, s));
      GQ_TRY(upload(P, na, &P->snx, s));
      GQ_TRY(upload(P, nb, &P->sny, s));
      GQ_TRY(upload(P, nc, &P->snz, s));
      GQ_TRY(upload(P, w, &P->sw, s));
      GQ_TRY(upload(P, T.src_order, &P->src_order, s));
      std::vector<double> x(n_ctr), y(n_ctr), z(n_ctr);
      std::vector<int64_t> pos(n_ctr);
      for (int64_t i = 0; i < n_ctr; ++i) {
        int64_t j = T.ctr_order[i];
        pos[j] = i;
        x[i] = ctr_xyz[3 * j];
        y[i] = ctr_xyz[3 * j + 1];
        z[i] = ctr_xyz[3 * j + 2];
      }
      GQ_TRY(upload(P, x, &P->cx, s));
      GQ_TRY(upload(P, y, &P->cy, s));
      GQ_TRY(upload(P, z, &P->cz, s));
      // targets sorted by the tree position of their center
      // QBX targets, sorted by the tree position of their center
      std::vector<int64_t> tord;
      tord.reserve(P->n_qt);
      for (int64_t i = 0; i < n_tgt; ++i)
        if (tgt_center[i] >= 0) tord.push_back(i);
      std::stable_sort(tord.begin(), tord.end(), [&](int64_t u, int64_t v) {
        return pos[tgt_center[u]] < pos[tgt_center[v]];
      });
      const int64_t nq = (int64_t)tord.size();
      std::vector<double> tx(nq), ty(nq), tz(nq);
      std::vector<int64_t> tc(nq);
      for (int64_t i = 0; i < nq; ++i) {
        int64_t j = tord[i];
        tx[i] = tgt_xyz[3 * j];
        ty[i] = tgt_xyz[3 * j + 1];
        tz[i] = tgt_xyz[3 * j + 2];
        tc[i] = pos[tgt_center[j]];
      }
      GQ_TRY(upload(P, tx, &P->tx, s));
      GQ_TRY(upload(P, ty, &P->ty, s));
      GQ_TRY(upload(P, tz, &P->tz, s));
      GQ_TRY(upload(P, tc, &P->tgt_ctr, s));
      GQ_TRY(upload(P, tord, &P->tgt_out, s));
      P->h_tgt_ctr.swap(tc);
      P->h_tgt_out.swap(tord);
      // conventional targets
      if (P->n_pt > 0) {
        std::vector<double> a(P->n_pt), b(P->n_pt), c(P->n_pt);
        for (int64_t i = 0; i < P->n_pt; ++i) {
          const int64_t j = P->h_pt_in[i];
          a[i] = tgt_xyz[3 * j];
          b[i] = tgt_xyz[3 * j + 1];
          c[i] = tgt_xyz[3 * j + 2];
        }
        GQ_TRY(upload(P, a, &P->px, s));
        GQ_TRY(upload(P, b, &P->py, s));
        GQ_TRY(upload(P, c, &P->pz, s));
        GQ_TRY(upload(P, P->h_pt_box, &P->d_pt_box, s));
        GQ_TRY(upload(P, P->h_pt_in, &P->d_pt_out, s));
        GQ_TRY(alloc(P, (size_t)P->n_pt, &P->phi));
      }
      GQ_TRY(upload(P, T.center, &P->bctr, s));
      GQ_TRY(upload(P, T.h, &P->bh, s));
      GQ_TRY(upload(P, T.src_start, &P->src_start, s));
      GQ_TRY(upload(P, T.src_count, &P->src_count, s));
      P->nbuf = near_field_densities(P->prm);
      GQ_TRY(alloc(P, (size_t)n_src * P->nbuf, &P->q));
      GQ_TRY(alloc(P, (size_t)T.nboxes * P->np, &P->M));
      GQ_TRY(alloc(P, (size_t)T.nboxes * P->np, &P->L));
      GQ_TRY(alloc(P, (size_t)n_ctr * P->nq * P->nbuf, &P->Lq));
      GQ_HIP(hipStreamSynchronize(s));
      return GQ_OK;
    };
    st = go();
    if (st == GQ_OK && (prm->flags & GQ_FLAG_AUTOTUNE)) st = autotune_m2l(P, s);
    if (st == GQ_OK) st = upload_slot_sums(P);
    if (st != GQ_OK) {
      delete P;
      return st;
    }
  }
  P->stats.plan_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = P;
  return GQ_OK;
}

// GQ_FLAG_AUTOTUNE_TREE: time one apply of candidate trees and keep the fastest.  nmax is
// tried at 1/2, 3/4, 1 and 3/2 of the given value, then Remark 4's threshold (when
// nonzero) at 1/2, 1 and 2 times the given value with the best nmax; the kept parameters
// are reported in gq_stats_t.  Each candidate is a complete plan, built, timed (one warm-up
// and two timed applies of a unit density on the plan's stream) and destroyed in turn.
static gq_status create_plan_tuned(const gq_params* prm, int64_t n_src, const double* src_xyz,
                                   const double* src_w, const double* src_normal,
                                   int64_t n_ctr, const double* ctr_xyz,
                                   const double* ctr_radius, int64_t n_tgt,
                                   const double* tgt_xyz, const int64_t* tgt_center,
                                   void* hip_stream, gq_plan** out) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)hip_stream;
  gq_params base = *prm;
  base.flags &= ~(GQ_FLAG_AUTOTUNE_TREE | GQ_FLAG_GRAPH | GQ_FLAG_TIMING | GQ_FLAG_AUTOTUNE);
  double* dens = nullptr;
  double* pot = nullptr;
  GQ_HIP(hipMalloc(&dens, sizeof(double) * (size_t)prm->n_densities * n_src));
  const hipError_t ep = hipMalloc(&pot, sizeof(double) * (size_t)prm->n_densities *
                                            (n_tgt > 0 ? n_tgt : 1));
  if (ep != hipSuccess) {
    (void)hipFree(dens);
    return fail(GQ_ENOMEM, std::string("autotune: ") + hipGetErrorString(ep));
  }
  gq::launch_fill(s, dens, (int64_t)prm->n_densities * n_src, 1.0);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  gq_status st = GQ_OK;
  double best_ms = 1e300;
  gq_params best = base;
  auto trial = [&](const gq_params& c) -> gq_status {
    gq_plan* P = nullptr;
    gq_status r = create_plan(&c, n_src, src_xyz, src_w, src_normal, n_ctr, ctr_xyz,
                              ctr_radius, n_tgt, tgt_xyz, tgt_center, hip_stream, &P);
    if (r == GQ_ENOMEM) return GQ_OK;  // a candidate over the workspace cap is skipped
    if (r != GQ_OK) return r;
    r = gq_apply(P, dens, pot, hip_stream);
    hipError_t e = hipSuccess;
    if (r == GQ_OK) e = hipEventRecord(e0, s);
    for (int k = 0; k < 2 && r == GQ_OK && e == hipSuccess; ++k) r = gq_apply(P, dens, pot, hip_stream);
    if (r == GQ_OK && e == hipSuccess) e = hipEventRecord(e1, s);
    if (r == GQ_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (r == GQ_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    gq_plan_destroy(P);
    if (r != GQ_OK) return r;
    if (e != hipSuccess)
      return fail(GQ_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
    return GQ_OK;
  };
  const double fn[4] = {0.5, 0.75, 1.0, 1.5};
  for (int i = 0; i < 4 && st == GQ_OK; ++i) {
    gq_params c = base;
    c.nmax = std::max(1, (int)std::lround(prm->nmax * fn[i]));
    if (i > 0 && c.nmax == (int)std::lround(prm->nmax * fn[i - 1])) continue;
    st = trial(c);
  }
  if (st == GQ_OK && prm->wfar_direct_max > 0) {
    const int nm = best.nmax;
    const int w[2] = {std::max(1, prm->wfar_direct_max / 2), 2 * prm->wfar_direct_max};
    for (int i = 0; i < 2 && st == GQ_OK; ++i) {
      gq_params c = base;
      c.nmax = nm;
      c.wfar_direct_max = w[i];
      st = trial(c);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(dens);
  (void)hipFree(pot);
  if (st != GQ_OK) return st;
  if (best_ms >= 1e300) return fail(GQ_ENOMEM, "no candidate tree fits the workspace cap");
  gq_params fin = *prm;
  fin.nmax = best.nmax;
  fin.wfar_direct_max = best.wfar_direct_max;
  fin.flags &= ~GQ_FLAG_AUTOTUNE_TREE;
  st = create_plan(&fin, n_src, src_xyz, src_w, src_normal, n_ctr, ctr_xyz, ctr_radius, n_tgt,
                   tgt_xyz, tgt_center, hip_stream, out);
  if (st != GQ_OK) return st;
  (*out)->prm.flags |= GQ_FLAG_AUTOTUNE_TREE;
  (*out)->stats.plan_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return GQ_OK;
}

gq_status gq_plan_create(const gq_params* prm, int64_t n_src, const double* src_xyz,
                         const double* src_w, const double* src_normal, int64_t n_ctr,
                         const double* ctr_xyz, const double* ctr_radius, int64_t n_tgt,
                         const double* tgt_xyz, const int64_t* tgt_center, void* hip_stream,
                         gq_plan** out) {
  if (prm && (prm->flags & GQ_FLAG_AUTOTUNE_TREE)) {
    g_err.clear();
    if (prm->flags & GQ_FLAG_HOST_ONLY)
      return fail(GQ_EINVAL, "GQ_FLAG_AUTOTUNE_TREE needs a device plan, not a host-only one");
    // the candidates' own validation reports bad inputs; only the tuner's buffer sizes are
    // checked here
    if (out && n_src > 0 && n_ctr > 0 && n_tgt >= 0 && prm->n_densities >= 1 && prm->nmax >= 1)
      return create_plan_tuned(prm, n_src, src_xyz, src_w, src_normal, n_ctr, ctr_xyz,
                               ctr_radius, n_tgt, tgt_xyz, tgt_center, hip_stream, out);
  }
  return create_plan(prm, n_src, src_xyz, src_w, src_normal, n_ctr, ctr_xyz, ctr_radius, n_tgt,
                     tgt_xyz, tgt_center, hip_stream, out);
}

}  // extern "C"

namespace {

// Enqueues every density pass of one apply on stream s (eager launches, or the launches
// being captured into a graph).
// One roctx range per stage of an apply, shown by rocprofv3 --marker-trace.  The ranges are
// host-side: they bracket the enqueue of each stage's launches, and the kernel records of the
// same trace give the device times.  Outside a profiler the calls return at once.
class StageRanges {
 public:
  void next(const char* name) {
    if (open_) roctxRangePop();
    roctxRangePushA(name);
    open_ = true;
  }
  ~StageRanges() {
    if (open_) roctxRangePop();
  }

 private:
  bool open_ = false;
};

gq_status apply_passes(gq_plan* P, const double* density, double* potential, hipStream_t s,
                       bool timing) {
  const gq::Tree& T = P->tree;
  const int p = P->prm.p_fmm, qo = P->prm.p_qbx, np = P->np;
  const int kern = P->prm.kernel == GQ_KERNEL_D ? 1 : 0;  // source side: S' uses S's
  const bool sprime = P->prm.kernel == GQ_KERNEL_SP;
  const int prec = P->prm.precision;
  gq::SrcSoA src{P->sx, P->sy, P->sz, P->snx, P->sny, P->snz};
  const bool overlap = P->overlap && P->side;
  hipEvent_t* ev = nullptr;
  auto mark = [&](int i, hipStream_t st) -> gq_status {
    if (timing) GQ_HIP(hipEventRecord(ev[i], st));
    return GQ_OK;
  };
  // one batch of dense translations, Y[dst] += T X[src]: added atomically, or (deterministic
  // plans) stored to the pair slots and summed per destination in pair order
  auto translate = [&](hipStream_t st, int kind, const TileSet& t, const std::array<int*, 5>& dd,
                       const gq::TransMats& tm, const double* X, double* Y, int cols, bool xcd,
                       const gq_plan::SlotSum* ss) {
    if (P->det) {
      gq::launch_translate(st, kind, prec, np, t.ntile(), dd[0], dd[1], dd[2], dd[3], dd[4], tm,
                           X, P->slots, cols, xcd, true);
      gq::launch_slot_sum(st, np, ss->ndst, ss->dst, ss->ptr, ss->pair, P->slots, Y);
    } else {
      gq::launch_translate(st, kind, prec, np, t.ntile(), dd[0], dd[1], dd[2], dd[3], dd[4], tm,
                           X, Y, cols, xcd);
    }
  };
  // Densities go through the near field in groups of P->nbuf (its kernel shares each
  // pair's harmonics between them); every other stage runs once per density.  One timed pass
  // per density: the group's strengths, fills and near field are timed in its first pass.
  const int nden = P->prm.n_densities;
  const int64_t nlq = P->n_ctr * P->nq;
  for (int d = 0; d < nden; ++d) {
    const int e = d % P->nbuf;                        // position in the near-field group
    const int ng = std::min(P->nbuf, nden - (d - e));  // densities of the group
    double* qd = P->q + (int64_t)e * P->n_src;        // this density's strengths
    double* Lqd = P->Lq + (int64_t)e * nlq;           // and center locals
    if (timing) {
      if (P->ev_used == P->ev_sets.size()) {
        std::array<hipEvent_t, kEvents> set{};
        for (auto& e : set) GQ_HIP(hipEventCreate(&e));
        P->ev_sets.push_back(set);
      }
      ev = P->ev_sets[P->ev_used++].data();
    }
    StageRanges rng;
    rng.next("gq: strengths");
    GQ_TRY(mark(0, s));
    for (int g = 0; e == 0 && g < ng; ++g) {
      double* qg = P->q + (int64_t)g * P->n_src;
      if (P->interp)
        gq::launch_strength_interp(s, P->n_src, P->src_order, P->sw, P->n_node, P->n_quad,
                                   P->interp, density + (int64_t)(d + g) * P->n_elem * P->n_node,
                                   qg);
      else
        gq::launch_strength(s, P->n_src, P->src_order, P->sw,
                            density + (int64_t)(d + g) * P->n_src, qg);
    }
    GQ_TRY(mark(1, s));
    rng.next("gq: clear expansions");
    gq::launch_fill(s, P->M, (int64_t)T.nboxes * np, 0.0);
    gq::launch_fill(s, P->L, (int64_t)T.nboxes * np, 0.0);
    if (e == 0) gq::launch_fill(s, P->Lq, nlq * ng, 0.0);
    if (P->n_pt > 0) gq::launch_fill(s, P->phi, P->n_pt, 0.0);
    GQ_TRY(mark(2, s));
    // far-field chain: writes only M and L, so it may run beside the near field
    hipStream_t f = s;
    if (overlap) {
      GQ_HIP(hipEventRecord(P->ev_fork, s));
      GQ_HIP(hipStreamWaitEvent(P->side, P->ev_fork, 0));
      f = P->side;
    }
    rng.next("gq: stage 2a P2M");
    gq::launch_p2m(f, kern, p, (int)P->p2m_boxes.size(), P->d_p2m_boxes, P->d_p2m_ptr,
                   P->d_p2m_idx, P->bctr, P->bh, src, qd, P->M, P->det);
    GQ_TRY(mark(3, f));
    rng.next("gq: stage 2b M2M");
    for (int l = T.nlevels - 1; l >= 1; --l)
      translate(f, 0, P->m2m_levels[l], P->d_m2m[l], P->tm_m2m, P->M, P->M, P->lvl_cols, true,
                P->det ? &P->ss_m2m[l] : nullptr);
    GQ_TRY(mark(4, f));
    rng.next("gq: stage 4 M2L");
    if (P->prm.m2l_rotation) {
      gq::launch_m2l_rot(f, np, P->m2l.ntile(), P->d_m2l[0], P->d_m2l[1], P->d_m2l[2],
                         P->d_m2l[3], P->d_m2l[4], P->rot, P->M, P->det ? P->slots : P->L,
                         P->m2l_xcd, P->det);
      if (P->det)
        gq::launch_slot_sum(f, np, P->ss_m2l.ndst, P->ss_m2l.dst, P->ss_m2l.ptr,
                            P->ss_m2l.pair, P->slots, P->L);
    } else {
      translate(f, 2, P->m2l, P->d_m2l, P->tm_m2l, P->M, P->L, P->m2l_cols, P->m2l_xcd,
                &P->ss_m2l);
    }
    GQ_TRY(mark(5, f));
    rng.next("gq: stage 6b P2L");
    gq::launch_p2l(f, kern, p, (int)P->p2l_box.size(), P->d_p2l_box, P->d_p2l_ptr,
                   P->d_p2l_idx, P->bctr, P->bh, src, qd, P->L, P->det);
    GQ_TRY(mark(6, f));
    rng.next("gq: stage 7 L2L");
    for (int l = 1; l < T.nlevels; ++l)
      translate(f, 1, P->l2l_levels[l], P->d_l2l[l], P->tm_l2l, P->L, P->L, P->lvl_cols, true,
                P->det ? &P->ss_l2l[l] : nullptr);
    GQ_TRY(mark(7, f));
    // near field: writes only Lq and the point-target potentials
    rng.next("gq: stages 3, 5a, 6a P2QBXL");
    GQ_TRY(mark(12, s));
    if (e == 0)
      gq::launch_p2qbxl(s, kern, qo, (int)P->k3_box.size(), P->d_k3_box, P->d_k3_c0,
                        P->d_k3_nc, P->d_near_ptr, P->d_near_idx, src, P->q, P->cx, P->cy,
                        P->cz, P->Lq, P->n_ctr, ng, P->n_src, nlq);
    gq::launch_p2p(s, kern, (int)P->pp_box.size(), P->d_pp_box, P->d_pp_t0, P->d_pp_nt,
                   P->d_near_ptr, P->d_near_idx, src, qd, P->px, P->py, P->pz, P->phi);
    GQ_TRY(mark(8, s));
    if (overlap) {
      GQ_HIP(hipEventRecord(P->ev_join, f));
      GQ_HIP(hipStreamWaitEvent(s, P->ev_join, 0));
    }
    GQ_TRY(mark(13, s));
    rng.next("gq: stage 5b M2QBXL");
    gq::launch_m2qbxl(s, p, qo, (int)P->k5_c0.size(), P->d_k5_c0, P->d_k5_nc, P->d_k5_w0,
                      P->d_k5_w1, P->d_wf_box, P->bctr, P->bh, P->M, P->cx, P->cy, P->cz,
                      Lqd, P->n_ctr);
    gq::launch_m2p(s, p, (int)P->pm_t0.size(), P->d_pm_t0, P->d_pm_nt, P->d_pm_w0, P->d_pm_w1,
                   P->d_wf_box, P->bctr, P->bh, P->M, P->px, P->py, P->pz, P->phi);
    GQ_TRY(mark(9, s));
    rng.next("gq: stage 8 L2QBXL");
    gq::launch_l2qbxl(s, p, qo, P->k8_nsingle, P->d_k8_box, P->d_k8_c0, P->d_k8_nc, P->bctr,
                      P->bh, P->L, P->cx, P->cy, P->cz, Lqd, P->n_ctr);
    gq::launch_l2qbxl_pairs(s, p, qo, P->k8_npair, P->d_k8_box + P->k8_nsingle,
                            P->d_k8_c0 + P->k8_nsingle, P->d_k8_nc + P->k8_nsingle, P->bctr,
                            P->bh, P->L, P->cx, P->cy, P->cz, Lqd, P->n_ctr);
    GQ_TRY(mark(10, s));
    rng.next("gq: stage 9 QBXL2P");
    if (sprime)
      gq::launch_qbxl2p_grad(s, qo, P->n_qt, P->tgt_ctr, P->tx, P->ty, P->tz, P->tnx, P->tny,
                             P->tnz, P->cx, P->cy, P->cz, Lqd, P->n_ctr, P->tgt_out,
                             potential + (int64_t)d * P->n_tgt);
    else
      gq::launch_qbxl2p(s, qo, P->n_qt, P->tgt_ctr, P->tx, P->ty, P->tz, P->cx, P->cy, P->cz,
                        Lqd, P->n_ctr, P->tgt_out, potential + (int64_t)d * P->n_tgt);
    gq::launch_l2p(s, p, P->n_pt, P->d_pt_box, P->bctr, P->bh, P->L, P->px, P->py, P->pz,
                   P->phi, P->d_pt_out, potential + (int64_t)d * P->n_tgt);
    GQ_TRY(mark(11, s));
    GQ_HIP(hipGetLastError());
  }
  return GQ_OK;
}

}  // namespace

extern "C" {

gq_status gq_apply(gq_plan* P, const double* density, double* potential, void* hip_stream) {
  g_err.clear();
  if (!P) return fail(GQ_EINVAL, "NULL plan");
  if (P->prm.flags & GQ_FLAG_HOST_ONLY) return fail(GQ_EINVAL, "plan was created host-only");
  if (!density || (!potential && P->n_tgt > 0)) return fail(GQ_EINVAL, "NULL device buffer");
  if (P->prm.kernel == GQ_KERNEL_SP && P->n_qt > 0 && !P->tnx)
    return fail(GQ_EINVAL, "S' needs the target normals (gq_set_target_normals)");
  hipStream_t s = (hipStream_t)hip_stream;
  P->last_stream = s;
  if (P->overlap && !P->side) {
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
    if (e != hipSuccess) {
      if (join) (void)hipEventDestroy(join);
      if (fork) (void)hipEventDestroy(fork);
      if (side) (void)hipStreamDestroy(side);
      return fail(GQ_EDEVICE, std::string("far-field stream: ") + hipGetErrorString(e));
    }
    P->side = side;
    P->ev_fork = fork;
    P->ev_join = join;
  }
  const bool timing = (P->prm.flags & GQ_FLAG_TIMING) != 0;
  if (!(P->prm.flags & GQ_FLAG_GRAPH)) {
    GQ_TRY(apply_passes(P, density, potential, s, timing));
    if (timing) P->timed_applies += 1;
    return GQ_OK;
  }
  // graph mode: capture on the plan's own stream, launch on the caller's
  if (!P->graph_exec || P->graph_density != density || P->graph_potential != potential) {
    if (P->graph_exec) {
      GQ_HIP(hipStreamSynchronize(s));
      GQ_HIP(hipGraphExecDestroy(P->graph_exec));
      P->graph_exec = nullptr;
    }
    if (!P->cap_stream) GQ_HIP(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    GQ_HIP(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
    gq_status st = apply_passes(P, density, potential, P->cap_stream, false);
    hipError_t e = hipStreamEndCapture(P->cap_stream, &g);
    if (st != GQ_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(GQ_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&P->graph_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(GQ_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    P->graph_density = density;
    P->graph_potential = potential;
  }
  GQ_HIP(hipGraphLaunch(P->graph_exec, s));
  P->graph_launches += 1;
  return GQ_OK;
}

gq_status gq_stats(gq_plan* P, gq_stats_t* out) {
  if (!P || !out) return fail(GQ_EINVAL, "NULL argument");
  if (P->ev_used > 0) {
    // sum the stage intervals of every density pass recorded since the last call
    const int slot[11] = {0, 10, 1, 2, 3, 4, 5, 6, 7, 8, 9};
    double ms[12] = {0};
    GQ_HIP(hipEventSynchronize(P->ev_sets[P->ev_used - 1][11]));
    for (size_t k = 0; k < P->ev_used; ++k) {
      auto& e = P->ev_sets[k];
      for (int i = 0; i < 11; ++i) {
        float t = 0.f;
        const hipEvent_t start = i == 7 ? e[12] : i == 8 ? e[13] : e[i];
        GQ_HIP(hipEventElapsedTime(&t, start, e[i + 1]));
        ms[slot[i]] += t;
      }
      float tot = 0.f;
      GQ_HIP(hipEventElapsedTime(&tot, e[0], e[11]));
      ms[11] += tot;
    }
    for (int i = 0; i < 12; ++i) P->stats.stage_ms[i] = ms[i];
    P->stats.timed_applies = P->timed_applies;
    P->ev_used = 0;
    P->timed_applies = 0;
  }
  P->stats.n_point_targets = P->n_pt;
  P->stats.device_bytes = P->dev_bytes;
  P->stats.nmax = P->prm.nmax;
  P->stats.wfar_direct_max = P->prm.wfar_direct_max;
  {
    // Table 7: q^2 per (source, center) pair of Lists 1, 3-close, 4-close; p^3 per List 2
    // pair and per List 3-far (box, center) pair; p^2 per List 4-far (source, box) pair
    const double p = P->prm.p_fmm, q = P->prm.p_qbx;
    const double w[6] = {q * q, p * p * p, q * q, p * p * p, q * q, p * p};
    double tot = 0.0;
    for (int i = 0; i < 6; ++i) {
      P->stats.modeled_flops[i] = w[i] * (double)P->stats.pairs[i];
      tot += P->stats.modeled_flops[i];
    }
    P->stats.modeled_flops[6] = tot;
  }
  P->stats.m2l_tile_cols = P->m2l_cols;
  P->stats.m2l_xcd_order = P->m2l_xcd ? 1 : 0;
  *out = P->stats;
  return GQ_OK;
}

gq_status gq_set_overlap(gq_plan* P, int on) {
  g_err.clear();
  if (!P) return fail(GQ_EINVAL, "NULL plan");
  if (on != 0 && on != 1) return fail(GQ_EINVAL, "on must be 0 or 1");
  if (P->overlap == (on == 1)) return GQ_OK;
  if (P->graph_exec) {  // the captured passes follow the old setting
    if (P->last_stream) GQ_HIP(hipStreamSynchronize(P->last_stream));
    GQ_HIP(hipGraphExecDestroy(P->graph_exec));
    P->graph_exec = nullptr;
  }
  P->overlap = on == 1;
  return GQ_OK;
}

gq_status gq_set_target_normals(gq_plan* P, const double* tgt_normal) {
  g_err.clear();
  if (!P || !tgt_normal) return fail(GQ_EINVAL, "NULL argument");
  if (P->prm.flags & GQ_FLAG_HOST_ONLY) return fail(GQ_EINVAL, "plan was created host-only");
  if (P->is_batch) return fail(GQ_EINVAL, "a batch plan takes its members' target normals");
  if (!finite3(tgt_normal, P->n_tgt)) return fail(GQ_EINVAL, "non-finite normal");
  std::vector<double> a(P->n_qt), b(P->n_qt), c(P->n_qt);
  for (int64_t i = 0; i < P->n_qt; ++i) {
    const double* nn = tgt_normal + 3 * P->h_tgt_out[i];
    const double l = std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    if (std::fabs(l - 1.0) > 1e-6) return fail(GQ_EINVAL, "target normals must have unit length");
    a[i] = nn[0];
    b[i] = nn[1];
    c[i] = nn[2];
  }
  hipStream_t s = P->last_stream;
  double** dst[3] = {&P->tnx, &P->tny, &P->tnz};
  const std::vector<double>* src[3] = {&a, &b, &c};
  for (int k = 0; k < 3; ++k) {
    if (!*dst[k]) GQ_TRY(alloc(P, (size_t)P->n_qt, dst[k]));
    GQ_HIP(hipMemcpyAsync(*dst[k], src[k]->data(), (size_t)P->n_qt * sizeof(double),
                          hipMemcpyHostToDevice, s));
  }
  GQ_HIP(hipStreamSynchronize(s));
  return GQ_OK;
}

gq_status gq_points_near(int64_t n_q, const double* q_xyz, const double* radius, int strict,
                         int64_t n_p, const double* p_xyz, uint8_t* hit, void* hip_stream) {
  g_err.clear();
  gq::NearQuery Q;
  bool done = false;
  GQ_TRY(gq::near_prepare(n_q, q_xyz, radius, n_p, p_xyz, hit, (int64_t)1 << 24, Q, done));
  if (done) return GQ_OK;
  struct DevBufs {
    std::vector<void*> p;
    ~DevBufs() {
      for (void* q : p) (void)hipFree(q);
    }
  } bufs;
  hipStream_t s = (hipStream_t)hip_stream;
  auto up = [&](const void* h, size_t bytes, void** d) -> gq_status {
    GQ_HIP(hipMalloc(d, bytes));
    bufs.p.push_back(*d);
    if (h) GQ_HIP(hipMemcpyAsync(*d, h, bytes, hipMemcpyHostToDevice, s));
    return GQ_OK;
  };
  void *dst, *dpx, *dpy, *dpz, *dqx, *dqy, *dqz, *dqr, *dhit;
  GQ_TRY(up(Q.start.data(), Q.start.size() * sizeof(int64_t), &dst));
  GQ_TRY(up(Q.px.data(), n_p * sizeof(double), &dpx));
  GQ_TRY(up(Q.py.data(), n_p * sizeof(double), &dpy));
  GQ_TRY(up(Q.pz.data(), n_p * sizeof(double), &dpz));
  GQ_TRY(up(Q.qx.data(), n_q * sizeof(double), &dqx));
  GQ_TRY(up(Q.qy.data(), n_q * sizeof(double), &dqy));
  GQ_TRY(up(Q.qz.data(), n_q * sizeof(double), &dqz));
  GQ_TRY(up(radius, n_q * sizeof(double), &dqr));
  GQ_TRY(up(nullptr, n_q, &dhit));
  const gq::AssocCells pts{(const int64_t*)dst, (const double*)dpx, (const double*)dpy,
                           (const double*)dpz, nullptr, nullptr, nullptr};
  gq::launch_points_near(s, n_q, (const double*)dqx, (const double*)dqy, (const double*)dqz,
                         (const double*)dqr, strict, Q.g, pts, (uint8_t*)dhit);
  GQ_HIP(hipGetLastError());
  GQ_HIP(hipMemcpyAsync(hit, dhit, n_q, hipMemcpyDeviceToHost, s));
  GQ_HIP(hipStreamSynchronize(s));
  return GQ_OK;
}

gq_status gq_associate_targets(int64_t n_src, const double* src_xyz, const double* src_danger,
                               int64_t n_ctr, const double* ctr_xyz, const double* ctr_radius,
                               const int8_t* ctr_side, int64_t n_tgt, const double* tgt_xyz,
                               const int8_t* tgt_side, double tol, int64_t* tgt_center,
                               void* hip_stream) {
  g_err.clear();
  if (n_src < 0 || n_ctr < 0 || n_tgt < 0) return fail(GQ_EINVAL, "negative count");
  if ((n_src && (!src_xyz || !src_danger)) || (n_ctr && (!ctr_xyz || !ctr_radius)) ||
      (n_tgt && (!tgt_xyz || !tgt_center)))
    return fail(GQ_EINVAL, "NULL array with a nonzero count");
  if (tgt_side && !ctr_side) return fail(GQ_EINVAL, "target sides need center sides");
  if (!std::isfinite(tol) || tol < 0) return fail(GQ_EINVAL, "tolerance must be finite and >= 0");
  if (!finite3(src_xyz, n_src) || !finite3(ctr_xyz, n_ctr) || !finite3(tgt_xyz, n_tgt))
    return fail(GQ_EINVAL, "non-finite coordinate");
  for (int64_t i = 0; i < n_src; ++i)
    if (!std::isfinite(src_danger[i]) || src_danger[i] < 0)
      return fail(GQ_EINVAL, "danger radii must be finite and >= 0");
  for (int64_t i = 0; i < n_ctr; ++i)
    if (!std::isfinite(ctr_radius[i]) || ctr_radius[i] <= 0)
      return fail(GQ_EINVAL, "center radii must be finite and > 0");
  if (ctr_side)
    for (int64_t i = 0; i < n_ctr; ++i)
      if (ctr_side[i] != 1 && ctr_side[i] != -1) return fail(GQ_EINVAL, "center side must be +-1");
  if (tgt_side)
    for (int64_t i = 0; i < n_tgt; ++i)
      if (tgt_side[i] < -1 || tgt_side[i] > 1) return fail(GQ_EINVAL, "target side must be -1, 0 or 1");
  if (n_src + n_ctr + n_tgt >= ((int64_t)1 << 31))
    return fail(GQ_EUNSUPPORTED, "more than 2^31 points");
  if (n_tgt == 0) return GQ_OK;
  if (n_src == 0) {  // nothing endangers any target
    for (int64_t i = 0; i < n_tgt; ++i) tgt_center[i] = GQ_TARGET_FAR;
    return GQ_OK;
  }
  // grid: cells at least as wide as every query radius, so a 27-cell neighbourhood holds
  // every source or center a target can reach
  std::vector<double> cr(n_ctr);
  for (int64_t i = 0; i < n_ctr; ++i) cr[i] = ctr_radius[i] * (1.0 + tol);
  double lo[3], hi[3], rmax = 0.0;
  for (int a = 0; a < 3; ++a) {
    lo[a] = tgt_xyz[a];
    hi[a] = tgt_xyz[a];
  }
  auto grow = [&](const double* p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], p[3 * i + a]);
        hi[a] = std::max(hi[a], p[3 * i + a]);
      }
  };
  grow(src_xyz, n_src);
  grow(ctr_xyz, n_ctr);
  grow(tgt_xyz, n_tgt);
  for (int64_t i = 0; i < n_src; ++i) rmax = std::max(rmax, src_danger[i]);
  for (int64_t i = 0; i < n_ctr; ++i) rmax = std::max(rmax, cr[i]);
  const gq::AssocGrid g = make_grid(lo, hi, rmax);
  const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
  auto cell_of = [&](const double* p) { return grid_cell(g, p); };
  // counting sort of sources and centers by cell
  struct Sorted {
    std::vector<int64_t> start, id;
    std::vector<double> x, y, z, r;
    std::vector<int8_t> side;
  };
  auto sort_cells = [&](int64_t n, const double* p, const double* r, const int8_t* sd, Sorted& o) {
    std::vector<int64_t> cell(n);
    o.start.assign(ncell + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
      cell[i] = cell_of(p + 3 * i);
      o.start[cell[i] + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) o.start[c + 1] += o.start[c];
    std::vector<int64_t> fill(o.start.begin(), o.start.end() - 1);
    o.id.resize(n);
    o.x.resize(n);
    o.y.resize(n);
    o.z.resize(n);
    o.r.resize(n);
    if (sd) o.side.resize(n);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t k = fill[cell[i]]++;
      o.id[k] = i;
      o.x[k] = p[3 * i];
      o.y[k] = p[3 * i + 1];
      o.z[k] = p[3 * i + 2];
      o.r[k] = r[i];
      if (sd) o.side[k] = sd[i];
    }
  };
  Sorted S, Cs;
  sort_cells(n_src, src_xyz, src_danger, nullptr, S);
  sort_cells(n_ctr, ctr_xyz, cr.data(), ctr_side, Cs);
  std::vector<double> tx(n_tgt), ty(n_tgt), tz(n_tgt);
  for (int64_t i = 0; i < n_tgt; ++i) {
    tx[i] = tgt_xyz[3 * i];
    ty[i] = tgt_xyz[3 * i + 1];
    tz[i] = tgt_xyz[3 * i + 2];
  }
  // device copies, freed on every exit
  struct DevBufs {
    std::vector<void*> p;
    ~DevBufs() {
      for (void* q : p) (void)hipFree(q);
    }
  } bufs;
  hipStream_t s = (hipStream_t)hip_stream;
  auto up = [&](const void* h, size_t bytes, void** d) -> gq_status {
    *d = nullptr;
    if (bytes == 0) return GQ_OK;
    GQ_HIP(hipMalloc(d, bytes));
    bufs.p.push_back(*d);
    if (h) GQ_HIP(hipMemcpyAsync(*d, h, bytes, hipMemcpyHostToDevice, s));
    return GQ_OK;
  };
  void *dtx, *dty, *dtz, *dts, *dout;
  GQ_TRY(up(tx.data(), n_tgt * sizeof(double), &dtx));
  GQ_TRY(up(ty.data(), n_tgt * sizeof(double), &dty));
  GQ_TRY(up(tz.data(), n_tgt * sizeof(double), &dtz));
  GQ_TRY(up(tgt_side, tgt_side ? n_tgt : 0, &dts));
  GQ_TRY(up(nullptr, n_tgt * sizeof(int64_t), &dout));
  gq::AssocCells dc[2]{};
  Sorted* hs[2] = {&S, &Cs};
  for (int w = 0; w < 2; ++w) {
    Sorted& o = *hs[w];
    const size_t n = o.x.size();
    void *st, *x, *y, *z, *r, *sd = nullptr, *id = nullptr;
    GQ_TRY(up(o.start.data(), o.start.size() * sizeof(int64_t), &st));
    GQ_TRY(up(o.x.data(), n * sizeof(double), &x));
    GQ_TRY(up(o.y.data(), n * sizeof(double), &y));
    GQ_TRY(up(o.z.data(), n * sizeof(double), &z));
    GQ_TRY(up(o.r.data(), n * sizeof(double), &r));
    if (w == 1) {
      GQ_TRY(up(o.side.empty() ? nullptr : o.side.data(), o.side.size(), &sd));
      GQ_TRY(up(o.id.data(), n * sizeof(int64_t), &id));
    }
    dc[w] = gq::AssocCells{(const int64_t*)st, (const double*)x, (const double*)y,
                           (const double*)z, (const double*)r, (const int8_t*)sd,
                           (const int64_t*)id};
  }
  gq::launch_associate(s, n_tgt, (const double*)dtx, (const double*)dty, (const double*)dtz,
                       (const int8_t*)dts, g, dc[0], dc[1], (int64_t*)dout);
  GQ_HIP(hipGetLastError());
  GQ_HIP(hipMemcpyAsync(tgt_center, dout, n_tgt * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  GQ_HIP(hipStreamSynchronize(s));
  return GQ_OK;
}

gq_status gq_set_source_interp(gq_plan* P, int64_t n_elem, int n_node, int n_quad,
                               const double* interp) {
  g_err.clear();
  if (!P || !interp) return fail(GQ_EINVAL, "NULL argument");
  if (P->is_batch) return fail(GQ_EUNSUPPORTED, "a batch plan cannot take a source interpolation");
  if (n_node < 1 || n_node > 64 || n_quad < 1 || (int64_t)n_quad * n_node > (1 << 20))
    return fail(GQ_EINVAL, "interpolation size out of range (1 <= n_node <= 64, "
                           "n_quad * n_node <= 2^20)");
  if (n_elem < 1 || n_elem * n_quad != P->n_src)
    return fail(GQ_EINVAL, "n_elem * n_quad must equal the plan's source count");
  const int64_t nm = (int64_t)n_quad * n_node;
  for (int64_t i = 0; i < nm; ++i)
    if (!std::isfinite(interp[i])) return fail(GQ_EINVAL, "non-finite interpolation entry");
  if (P->prm.flags & GQ_FLAG_HOST_ONLY) return fail(GQ_EINVAL, "plan was created host-only");
  hipStream_t s = P->last_stream;
  if (P->graph_exec) {  // the captured apply reads the old layout: capture anew
    GQ_HIP(hipStreamSynchronize(s));
    GQ_HIP(hipGraphExecDestroy(P->graph_exec));
    P->graph_exec = nullptr;
  }
  if (P->interp && (int64_t)P->n_quad * P->n_node < nm) {
    GQ_HIP(hipStreamSynchronize(s));
    P->interp = nullptr;  // the old buffer stays in P->allocs until the plan is destroyed
  }
  if (!P->interp) GQ_TRY(alloc(P, (size_t)nm, &P->interp));
  GQ_HIP(hipMemcpyAsync(P->interp, interp, (size_t)nm * sizeof(double), hipMemcpyHostToDevice, s));
  GQ_HIP(hipStreamSynchronize(s));
  P->n_elem = n_elem;
  P->n_node = n_node;
  P->n_quad = n_quad;
  return GQ_OK;
}

gq_status gq_batch_create(int n_plans, gq_plan* const* plans, unsigned flags, void* hip_stream,
                          gq_plan** out) {
  g_err.clear();
  auto t0 = std::chrono::steady_clock::now();
  if (!plans || !out || n_plans < 1) return fail(GQ_EINVAL, "need at least one plan");
  const unsigned allowed = GQ_FLAG_TIMING | GQ_FLAG_GRAPH | GQ_FLAG_AUTOTUNE;
  if (flags & ~allowed) return fail(GQ_EINVAL, "unsupported batch flag");
  if ((flags & GQ_FLAG_TIMING) && (flags & GQ_FLAG_GRAPH))
    return fail(GQ_EINVAL, "GQ_FLAG_TIMING and GQ_FLAG_GRAPH are exclusive");
  const gq_plan* P0 = plans[0];
  for (int k = 0; k < n_plans; ++k) {
    const gq_plan* P = plans[k];
    if (!P) return fail(GQ_EINVAL, "NULL plan in batch");
    if (P->prm.flags & GQ_FLAG_HOST_ONLY) return fail(GQ_EINVAL, "host-only plan in batch");
    if (P->prm.p_qbx != P0->prm.p_qbx || P->prm.p_fmm != P0->prm.p_fmm ||
        P->prm.kernel != P0->prm.kernel || P->prm.precision != P0->prm.precision ||
        P->prm.m2l_rotation != P0->prm.m2l_rotation ||
        P->prm.n_densities != P0->prm.n_densities ||
        (P->prm.flags & GQ_FLAG_DETERMINISTIC) != (P0->prm.flags & GQ_FLAG_DETERMINISTIC))
      return fail(GQ_EINVAL, "batch members must share p_qbx, p_fmm, kernel, precision, "
                             "n_densities and GQ_FLAG_DETERMINISTIC");
    for (int j = 0; j < k; ++j)
      if (plans[j] == P) return fail(GQ_EINVAL, "plan listed twice in batch");
  }
  for (int k = 0; k < n_plans; ++k)
    if (plans[k]->interp)
      return fail(GQ_EUNSUPPORTED, "batch members with an oversampled source quadrature");
  gq_plan* B = new (std::nothrow) gq_plan();
  if (!B) return fail(GQ_ENOMEM, "host allocation failed");
  B->is_batch = true;
  B->prm = P0->prm;
  B->prm.flags = (P0->prm.flags & ~(GQ_FLAG_TIMING | GQ_FLAG_GRAPH | GQ_FLAG_AUTOTUNE)) | flags;
  B->np = P0->np;
  B->nq = P0->nq;
  for (int k = 0; k < n_plans; ++k) {
    B->n_src += plans[k]->n_src;
    B->n_ctr += plans[k]->n_ctr;
    B->n_tgt += plans[k]->n_tgt;
    B->n_qt += plans[k]->n_qt;
  }
  B->last_stream = (hipStream_t)hip_stream;
  gq_status st = merge_plans(B, plans, n_plans);
  if (st == GQ_OK) st = merge_geometry(B, plans, n_plans, B->last_stream);
  if (st == GQ_OK) st = upload_work(B);
  if (st == GQ_OK && (flags & GQ_FLAG_AUTOTUNE)) st = autotune_m2l(B, B->last_stream);
  if (st == GQ_OK) st = upload_slot_sums(B);
  if (st != GQ_OK) {
    delete B;
    return st;
  }
  B->stats.plan_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = B;
  return GQ_OK;
}

void gq_plan_destroy(gq_plan* P) {
  if (!P) return;
  if (!(P->prm.flags & GQ_FLAG_HOST_ONLY)) (void)hipDeviceSynchronize();
  delete P;
}

gq_status gq_tree_export(const gq_plan* P, double* box_center, double* box_h, int32_t* level,
                         int32_t* parent, int64_t* ctr_owner) {
  if (!P) return fail(GQ_EINVAL, "NULL plan");
  const gq::Tree& T = P->tree;
  for (int b = 0; b < T.nboxes; ++b) {
    if (box_center)
      for (int a = 0; a < 3; ++a) box_center[3 * b + a] = T.center[3 * b + a];
    if (box_h) box_h[b] = T.h[b];
    if (level) level[b] = T.level[b];
    if (parent) parent[b] = T.parent[b];
  }
  if (ctr_owner)
    for (int64_t i = 0; i < P->n_ctr; ++i) ctr_owner[T.ctr_order[i]] = T.ctr_box[i];
  return GQ_OK;
}

gq_status gq_list_export(const gq_plan* P, int list, int64_t* ptr, int32_t* items,
                         int64_t* n_items) {
  if (!P) return fail(GQ_EINVAL, "NULL plan");
  if (list < 0 || list >= gq::L_NLISTS) return fail(GQ_EINVAL, "list index out of range");
  const gq::BoxList& L = P->lists.lst[list];
  if (n_items) *n_items = L.total();
  if (ptr)
    for (size_t i = 0; i < L.ptr.size(); ++i) ptr[i] = L.ptr[i];
  if (items)
    for (size_t i = 0; i < L.items.size(); ++i) items[i] = L.items[i];
  return GQ_OK;
}

gq_status gq_qbx_locals(gq_plan* P, double* host_out) {
  if (!P || !host_out) return fail(GQ_EINVAL, "NULL argument");
  if (P->prm.flags & GQ_FLAG_HOST_ONLY) return fail(GQ_EINVAL, "plan was created host-only");
  std::vector<double> buf((size_t)P->n_ctr * P->nq);
  GQ_HIP(hipStreamSynchronize(P->last_stream));
  const int last = (P->prm.n_densities - 1) % P->nbuf;  // buffer of the last density
  GQ_HIP(hipMemcpy(buf.data(), P->Lq + (int64_t)last * P->n_ctr * P->nq,
                   buf.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < P->n_ctr; ++i) {
    int64_t j = P->tree.ctr_order[i];
    for (int k = 0; k < P->nq; ++k) host_out[j * P->nq + k] = buf[(size_t)k * P->n_ctr + i];
  }
  return GQ_OK;
}

gq_status gq_translation_matrix(int kind, int p, int a, int b, int c, double* out) {
  if (!out || p < 0 || p > gq::kPmax) return fail(GQ_EINVAL, "bad argument");
  if (kind == 0 || kind == 1) {
    if (a < 0 || a > 7) return fail(GQ_EINVAL, "octant out of range");
    (kind == 0 ? gq::m2m_matrix : gq::l2l_matrix)(p, a, out);
    return GQ_OK;
  }
  if (kind >= 2 && kind <= 5) {
    if (std::max(std::abs(a), std::max(std::abs(b), std::abs(c))) < 1)
      return fail(GQ_EINVAL, "offset must be nonzero");
    if (kind == 2) {
      gq::m2l_matrix(p, a, b, c, out);
    } else {
      const size_t np = (size_t)gq::ncoef(p);
      std::vector<double> f(3 * np * np);
      gq::m2l_rotation_factors(p, a, b, c, f.data(), f.data() + np * np, f.data() + 2 * np * np);
      std::copy(f.begin() + (kind - 3) * np * np, f.begin() + (kind - 2) * np * np, out);
    }
    return GQ_OK;
  }
  return fail(GQ_EINVAL, "unknown kind");
}

}  // extern "C"
