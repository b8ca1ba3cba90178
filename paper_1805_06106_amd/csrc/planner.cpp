// Octree and interaction lists for the GIGAQBX FMM (Algorithm 5 Stage 1; Section 5.2).
//
// Readings of the paper used here (all predicates are evaluated in FP64 on exactly
// representable box centers and radii, compiled without floating-point contraction):
//  * root: smallest cube holding all sources, centers, targets and expansion balls, with
//    half-width rounded up to a power of two and center on a multiple of it;
//  * particles move to the upper child along an axis when coordinate >= box center;
//  * sources, centers and targets count toward nmax; a box splits while it owns more than
//    nmax particles and at least one would move;
//  * a center moves to its child iff |c - x_child|_2 + r_c <= sqrt(3)|child|(1 + t_f);
//  * a < TCR(b): |x_a - x_b|_2 - sqrt(3)|b|(1+t_f) >= 3|a|;
//    TCR(a) < b: |x_a - x_b|_inf - |b| >= 3|a|(1+t_f);
//  * k-colleagues exclude the box itself; List 3's descendants are strict;
//  * adjacent: closed cubes touch and neither box contains the other;
//  * list entries are restricted to boxes whose subtree holds a source.
//  * level restriction (optional): afterwards, a leaf touching a leaf two or more levels
//    finer is split by the same rule, until no such pair is left (or nothing can move);
//  * box-shaped TCR variant (tcr_linf): TCR(b) is the closed box of half-width |b|(1+t_f);
//    a center descends iff |c - x_child|_inf + r_c <= |child|(1 + t_f), and
//    a < TCR(b) iff |x_a - x_b|_inf - |b|(1+t_f) >= 3|a|.
#include "planner.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <unordered_map>

namespace gq {

namespace {

struct CellKey {
  int level;
  int64_t x, y, z;
  bool operator==(const CellKey& o) const {
    return level == o.level && x == o.x && y == o.y && z == o.z;
  }
};
struct CellHash {
  size_t operator()(const CellKey& k) const {
    uint64_t h = (uint64_t)k.level * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)k.x * 0xC2B2AE3D27D4EB4Full + (h << 6) + (h >> 2);
    h ^= (uint64_t)k.y * 0x165667B19E3779F9ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)k.z * 0x27D4EB2F165667C5ull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

const double kSqrt3 = std::sqrt(3.0);

}  // namespace

std::string build_tree(const TreeParams& prm, int64_t n_src, const double* src,
                       int64_t n_ctr, const double* ctr, const double* crad, int64_t n_tgt,
                       const double* tgt, Tree& T) {
  // ---- root cube -------------------------------------------------------------------
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = INFINITY;
    hi[a] = -INFINITY;
  }
  for (int64_t i = 0; i < n_src; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], src[3 * i + a]);
      hi[a] = std::max(hi[a], src[3 * i + a]);
    }
  for (int64_t i = 0; i < n_tgt; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], tgt[3 * i + a]);
      hi[a] = std::max(hi[a], tgt[3 * i + a]);
    }
  for (int64_t i = 0; i < n_ctr; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], ctr[3 * i + a] - crad[i]);
      hi[a] = std::max(hi[a], ctr[3 * i + a] + crad[i]);
    }
  double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
  int k = (int)std::ceil(std::log2(std::max(ext, 1e-300) / 2.0)) - 2;
  double x0[3], h0;
  for (;; ++k) {
    h0 = std::ldexp(1.0, k);
    bool ok = true;
    for (int a = 0; a < 3 && ok; ++a) {
      double j = std::floor(lo[a] / h0) + 1.0;
      if (!(hi[a] <= (j + 1.0) * h0)) ok = false;
      x0[a] = j * h0;
    }
    if (ok) break;
    if (k > 1100) return "cannot fit a root box around the input";
  }
  T = Tree();
  for (int a = 0; a < 3; ++a) T.root_center[a] = x0[a];
  T.root_h = h0;

  // ---- level-by-level subdivision (breadth-first numbering) ---------------------------
  std::vector<std::vector<int64_t>> own_s(1), own_c(1), own_t(1);
  own_s[0].resize(n_src);
  own_c[0].resize(n_ctr);
  own_t[0].resize(n_tgt);
  for (int64_t i = 0; i < n_src; ++i) own_s[0][i] = i;
  for (int64_t i = 0; i < n_ctr; ++i) own_c[0][i] = i;
  for (int64_t i = 0; i < n_tgt; ++i) own_t[0][i] = i;
  T.center = {x0[0], x0[1], x0[2]};
  T.h = {h0};
  T.level = {0};
  T.parent = {-1};
  std::array<int, 8> none;
  none.fill(-1);
  T.child = {none};
  T.nchild = {0};

  auto octant = [](const double* p, const double* xb) {
    return (p[0] >= xb[0] ? 1 : 0) | (p[1] >= xb[1] ? 2 : 0) | (p[2] >= xb[2] ? 4 : 0);
  };

  // Split box b: its sources and targets go to the octants that hold them, and each center
  // descends to its octant's child iff its ball fits that child's confinement region (else
  // it stays, suspended).  Only non-empty children are created.  False if nothing would
  // move (the box stays a leaf).
  auto split = [&](int b, std::vector<int>* created) -> bool {
    const double xb[3] = {T.center[3 * b], T.center[3 * b + 1], T.center[3 * b + 2]};
    const double hc = T.h[b] * 0.5;
    double cc[8][3];
    for (int o = 0; o < 8; ++o) {
      cc[o][0] = xb[0] + ((o & 1) ? hc : -hc);
      cc[o][1] = xb[1] + ((o & 2) ? hc : -hc);
      cc[o][2] = xb[2] + ((o & 4) ? hc : -hc);
    }
    const double conf = prm.tcr_linf ? hc * (1.0 + prm.tcf) : (kSqrt3 * hc) * (1.0 + prm.tcf);
    std::vector<int64_t> cs[8], ct[8], cc_[8], stay;
    for (int64_t i : own_s[b]) cs[octant(src + 3 * i, xb)].push_back(i);
    for (int64_t i : own_t[b]) ct[octant(tgt + 3 * i, xb)].push_back(i);
    int64_t moved_c = 0;
    for (int64_t i : own_c[b]) {
      const double* p = ctr + 3 * i;
      int o = octant(p, xb);
      double dx = p[0] - cc[o][0], dy = p[1] - cc[o][1], dz = p[2] - cc[o][2];
      double dist = prm.tcr_linf
                        ? std::max(std::fabs(dx), std::max(std::fabs(dy), std::fabs(dz)))
                        : std::sqrt((dx * dx + dy * dy) + dz * dz);
      if (dist + crad[i] <= conf) {
        cc_[o].push_back(i);
        ++moved_c;
      } else {
        stay.push_back(i);
      }
    }
    if ((int64_t)own_s[b].size() + (int64_t)own_t[b].size() + moved_c == 0) return false;
    for (int o = 0; o < 8; ++o) {
      if (cs[o].empty() && ct[o].empty() && cc_[o].empty()) continue;
      int id = (int)T.h.size();
      T.center.insert(T.center.end(), {cc[o][0], cc[o][1], cc[o][2]});
      T.h.push_back(hc);
      T.level.push_back(T.level[b] + 1);
      T.parent.push_back(b);
      T.child.push_back(none);
      T.nchild.push_back(0);
      T.child[b][o] = id;
      T.nchild[b] += 1;
      own_s.push_back(std::move(cs[o]));
      own_t.push_back(std::move(ct[o]));
      own_c.push_back(std::move(cc_[o]));
      if (created) created->push_back(id);
    }
    own_s[b].clear();
    own_t[b].clear();
    own_c[b] = std::move(stay);
    return true;
  };

  std::vector<int> frontier = {0};
  while (!frontier.empty()) {
    std::vector<int> next;
    for (int b : frontier) {
      int64_t n_own = (int64_t)own_s[b].size() + own_c[b].size() + own_t[b].size();
      if (n_own <= prm.nmax || T.level[b] >= prm.max_level) continue;
      split(b, &next);
    }
    frontier = std::move(next);
  }

  if (prm.level_restrict) {
    // Level restriction (the remark on List 3 complexity): while a leaf touches a leaf two
    // or more levels finer, split the coarser one.  Splitting only refines, so the result
    // does not depend on the order; leaves that cannot split (nothing would move) or sit
    // at the level cap are left as they are.
    for (;;) {
      const int nb0 = (int)T.h.size();
      auto icoord = [&](int b, int a) {
        return (int64_t)std::floor((T.center[3 * b + a] - (x0[a] - h0)) / (2.0 * T.h[b]));
      };
      std::unordered_map<CellKey, int, CellHash> cells;
      cells.reserve(2 * nb0);
      for (int b = 0; b < nb0; ++b) cells[{T.level[b], icoord(b, 0), icoord(b, 1), icoord(b, 2)}] = b;
      auto touches = [&](int x, int y) {
        for (int a = 0; a < 3; ++a)
          if (std::fabs(T.center[3 * x + a] - T.center[3 * y + a]) > T.h[x] + T.h[y]) return false;
        return true;
      };
      // does the subtree of x hold a leaf of level >= lmin touching box a?
      std::function<bool(int, int, int)> finer = [&](int x, int a, int lmin) -> bool {
        if (!touches(x, a)) return false;
        if (T.nchild[x] == 0) return T.level[x] >= lmin;
        for (int o = 0; o < 8; ++o)
          if (T.child[x][o] >= 0 && finer(T.child[x][o], a, lmin)) return true;
        return false;
      };
      std::vector<int> todo;
      for (int a = 0; a < nb0; ++a) {
        if (T.nchild[a] != 0 || T.level[a] >= prm.max_level) continue;
        const int64_t ix = icoord(a, 0), iy = icoord(a, 1), iz = icoord(a, 2);
        bool bad = false;
        for (int dz = -1; dz <= 1 && !bad; ++dz)
          for (int dy = -1; dy <= 1 && !bad; ++dy)
            for (int dx = -1; dx <= 1 && !bad; ++dx) {
              if (!dx && !dy && !dz) continue;
              auto it = cells.find({T.level[a], ix + dx, iy + dy, iz + dz});
              if (it != cells.end() && finer(it->second, a, T.level[a] + 2)) bad = true;
            }
        if (bad) todo.push_back(a);
      }
      bool any = false;
      for (int a : todo) any = split(a, nullptr) || any;
      if (!any) break;
    }
    // canonical breadth-first numbering (children in octant order), as the plain build has
    const int nbt = (int)T.h.size();
    std::vector<int> order = {0}, newid(nbt, -1);
    newid[0] = 0;
    for (size_t i = 0; i < order.size(); ++i)
      for (int o = 0; o < 8; ++o) {
        const int c = T.child[order[i]][o];
        if (c >= 0) {
          newid[c] = (int)order.size();
          order.push_back(c);
        }
      }
    Tree R = T;
    std::vector<std::vector<int64_t>> os(nbt), oc(nbt), ot(nbt);
    for (int i = 0; i < nbt; ++i) {
      const int b = order[i];
      for (int a = 0; a < 3; ++a) R.center[3 * i + a] = T.center[3 * b + a];
      R.h[i] = T.h[b];
      R.level[i] = T.level[b];
      R.parent[i] = T.parent[b] < 0 ? -1 : newid[T.parent[b]];
      R.nchild[i] = T.nchild[b];
      for (int o = 0; o < 8; ++o) R.child[i][o] = T.child[b][o] < 0 ? -1 : newid[T.child[b][o]];
      os[i] = std::move(own_s[b]);
      oc[i] = std::move(own_c[b]);
      ot[i] = std::move(own_t[b]);
    }
    T = std::move(R);
    own_s = std::move(os);
    own_c = std::move(oc);
    own_t = std::move(ot);
  }
  const int nb = (int)T.h.size();
  T.nboxes = nb;
  T.nlevels = 1 + *std::max_element(T.level.begin(), T.level.end());

  // integer cell coordinates
  T.ix.resize(nb);
  T.iy.resize(nb);
  T.iz.resize(nb);
  for (int b = 0; b < nb; ++b) {
    double w = 2.0 * T.h[b];
    T.ix[b] = (int64_t)((T.center[3 * b] - (x0[0] - h0)) / w - 0.5);
    T.iy[b] = (int64_t)((T.center[3 * b + 1] - (x0[1] - h0)) / w - 0.5);
    T.iz[b] = (int64_t)((T.center[3 * b + 2] - (x0[2] - h0)) / w - 0.5);
  }

  // preorder and particle renumbering
  T.preorder.clear();
  T.pre_index.assign(nb, 0);
  std::vector<int> stack = {0};
  while (!stack.empty()) {
    int b = stack.back();
    stack.pop_back();
    T.pre_index[b] = (int)T.preorder.size();
    T.preorder.push_back(b);
    for (int o = 7; o >= 0; --o)
      if (T.child[b][o] >= 0) stack.push_back(T.child[b][o]);
  }
  T.src_start.assign(nb, 0);
  T.src_count.assign(nb, 0);
  T.ctr_start.assign(nb, 0);
  T.ctr_count.assign(nb, 0);
  T.src_order.clear();
  T.ctr_order.clear();
  T.ctr_box.clear();
  T.tgt_start.assign(nb, 0);
  T.tgt_count.assign(nb, 0);
  T.tgt_order.clear();
  for (int b : T.preorder) {
    T.tgt_start[b] = (int64_t)T.tgt_order.size();
    T.tgt_count[b] = (int64_t)own_t[b].size();
    T.tgt_order.insert(T.tgt_order.end(), own_t[b].begin(), own_t[b].end());
    T.src_start[b] = (int64_t)T.src_order.size();
    T.src_count[b] = (int64_t)own_s[b].size();
    T.src_order.insert(T.src_order.end(), own_s[b].begin(), own_s[b].end());
    T.ctr_start[b] = (int64_t)T.ctr_order.size();
    T.ctr_count[b] = (int64_t)own_c[b].size();
    T.ctr_order.insert(T.ctr_order.end(), own_c[b].begin(), own_c[b].end());
    T.ctr_box.insert(T.ctr_box.end(), own_c[b].size(), b);
  }
  T.sub_src.assign(nb, 0);
  for (int i = nb - 1; i >= 0; --i) {
    int b = T.preorder[i];
    T.sub_src[b] += T.src_count[b];
    if (T.parent[b] >= 0) T.sub_src[T.parent[b]] += T.sub_src[b];
  }
  return "";
}

namespace {

struct ListBuilder {
  const Tree& T;
  double tcf;
  bool linf;
  std::unordered_map<CellKey, int, CellHash> cell;

  ListBuilder(const Tree& t, double tf, bool tcr_linf) : T(t), tcf(tf), linf(tcr_linf) {
    cell.reserve(2 * T.nboxes);
    for (int b = 0; b < T.nboxes; ++b) cell[{T.level[b], T.ix[b], T.iy[b], T.iz[b]}] = b;
  }

  int find(int level, int64_t x, int64_t y, int64_t z) const {
    if (x < 0 || y < 0 || z < 0) return -1;
    auto it = cell.find({level, x, y, z});
    return it == cell.end() ? -1 : it->second;
  }

  // boxes of b's level with cell offset in [-k, k]^3, excluding b
  template <class F>
  void for_colleagues(int b, int k, F&& f) const {
    for (int dz = -k; dz <= k; ++dz)
      for (int dy = -k; dy <= k; ++dy)
        for (int dx = -k; dx <= k; ++dx) {
          if (!dx && !dy && !dz) continue;
          int a = find(T.level[b], T.ix[b] + dx, T.iy[b] + dy, T.iz[b] + dz);
          if (a >= 0) f(a);
        }
  }

  bool contains(int a, int b) const {  // a == b or a is an ancestor of b
    int la = T.level[a], lb = T.level[b];
    if (la > lb) return false;
    int s = lb - la;
    return (T.ix[b] >> s) == T.ix[a] && (T.iy[b] >> s) == T.iy[a] && (T.iz[b] >> s) == T.iz[a];
  }

  double dinf(int a, int b) const {
    return std::max(std::fabs(T.center[3 * a] - T.center[3 * b]),
                    std::max(std::fabs(T.center[3 * a + 1] - T.center[3 * b + 1]),
                             std::fabs(T.center[3 * a + 2] - T.center[3 * b + 2])));
  }

  bool adjacent(int a, int b) const {
    if (contains(a, b) || contains(b, a)) return false;
    return dinf(a, b) <= T.h[a] + T.h[b];
  }

  bool prec_tcr(int a, int b) const {  // a < TCR(b)
    if (linf) return dinf(a, b) - T.h[b] * (1.0 + tcf) >= 3.0 * T.h[a];
    double dx = T.center[3 * a] - T.center[3 * b];
    double dy = T.center[3 * a + 1] - T.center[3 * b + 1];
    double dz = T.center[3 * a + 2] - T.center[3 * b + 2];
    double dist = std::sqrt((dx * dx + dy * dy) + dz * dz);
    return dist - (kSqrt3 * T.h[b]) * (1.0 + tcf) >= 3.0 * T.h[a];
  }

  bool tcr_prec(int a, int d) const {  // TCR(a) < d
    return dinf(a, d) - T.h[d] >= (3.0 * T.h[a]) * (1.0 + tcf);
  }

  bool src_leaf(int d) const { return T.is_leaf(d) && T.src_count[d] > 0; }

  void leaves_below(int b, std::vector<int>& out) const {
    if (T.sub_src[b] == 0) return;
    if (T.is_leaf(b)) {
      out.push_back(b);
      return;
    }
    for (int c : T.child[b])
      if (c >= 0) leaves_below(c, out);
  }

  void adjacent_leaves_below(int a, int b, std::vector<int>& out) const {
    if (T.sub_src[a] == 0 || !adjacent(a, b)) return;
    if (T.is_leaf(a)) {
      out.push_back(a);
      return;
    }
    for (int c : T.child[a])
      if (c >= 0) adjacent_leaves_below(c, b, out);
  }

  std::vector<int> list_U(int b) const {
    std::vector<int> out;
    leaves_below(b, out);
    for_colleagues(b, 1, [&](int a) { adjacent_leaves_below(a, b, out); });
    for (int A = T.parent[b]; A >= 0; A = T.parent[A])
      for_colleagues(A, 1, [&](int a) {
        if (src_leaf(a) && adjacent(a, b)) out.push_back(a);
      });
    return out;
  }

  std::vector<int> list_V(int b) const {
    std::vector<int> out;
    int p = T.parent[b];
    if (p < 0) return out;
    for_colleagues(p, 2, [&](int P) {
      for (int d : T.child[P]) {
        if (d < 0 || T.sub_src[d] == 0) continue;
        if (std::llabs(T.ix[d] - T.ix[b]) <= 2 && std::llabs(T.iy[d] - T.iy[b]) <= 2 &&
            std::llabs(T.iz[d] - T.iz[b]) <= 2)
          continue;
        out.push_back(d);
      }
    });
    return out;
  }

  void w_descend(int c, int b, std::vector<int>& out) const {
    if (T.sub_src[c] == 0) return;
    if (adjacent(c, b)) {
      for (int g : T.child[c])
        if (g >= 0) w_descend(g, b, out);
    } else {
      out.push_back(c);
    }
  }

  std::vector<int> list_W(int b) const {
    std::vector<int> out;
    for_colleagues(b, 2, [&](int a) {
      if (T.sub_src[a] == 0) return;
      for (int c : T.child[a])
        if (c >= 0) w_descend(c, b, out);
    });
    return out;
  }

  std::vector<int> list_X(int b) const {
    std::vector<int> out;
    for_colleagues(b, 2, [&](int a) {
      if (src_leaf(a) && !adjacent(a, b)) out.push_back(a);
    });
    int pb = T.parent[b];
    if (pb >= 0)
      for (int A = pb; A >= 0; A = T.parent[A])
        for_colleagues(A, 2, [&](int d) {
          if (src_leaf(d) && adjacent(d, pb) && !adjacent(d, b)) out.push_back(d);
        });
    return out;
  }

  void wsplit(int d, int b, std::vector<int>& close, std::vector<int>& far) const {
    if (T.sub_src[d] == 0) return;
    if (prec_tcr(d, b)) {
      far.push_back(d);
    } else if (T.is_leaf(d)) {
      close.push_back(d);
    } else {
      for (int c : T.child[d])
        if (c >= 0) wsplit(c, b, close, far);
    }
  }
};

void to_csr(const std::vector<std::vector<int>>& per_box, BoxList& L) {
  L.ptr.assign(per_box.size() + 1, 0);
  for (size_t b = 0; b < per_box.size(); ++b) L.ptr[b + 1] = L.ptr[b] + (int64_t)per_box[b].size();
  L.items.resize(L.ptr.back());
  for (size_t b = 0; b < per_box.size(); ++b)
    std::copy(per_box[b].begin(), per_box[b].end(), L.items.begin() + L.ptr[b]);
}

void sort_unique(std::vector<int>& v) {
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
}

}  // namespace

void build_lists(const Tree& T, double tcf, int wfar_direct_max, Lists& out, bool tcr_linf,
                 const std::vector<int64_t>* point_targets) {
  const int nb = T.nboxes;
  ListBuilder B(T, tcf, tcr_linf);
  out.is_target.assign(nb, 0);
  out.is_owner.assign(nb, 0);
  for (int b = 0; b < nb; ++b)
    if (T.ctr_count[b] > 0 || (point_targets && (*point_targets)[b] > 0)) {
      out.is_target[b] = 1;
      for (int a = b; a >= 0 && !out.is_owner[a]; a = T.parent[a]) out.is_owner[a] = 1;
    }
  std::vector<std::vector<int>> per[L_NLISTS];
  for (auto& v : per) v.assign(nb, {});
  // breadth-first numbering puts parents before children (X close/far recursion)
  for (int b = 0; b < nb; ++b) {
    if (!out.is_owner[b]) continue;
    auto V = B.list_V(b);
    sort_unique(V);
    per[L_V][b] = std::move(V);
    auto X = B.list_X(b);
    std::vector<int> pool = X;
    if (T.parent[b] >= 0) {
      const auto& pc = per[L_XCLOSE][T.parent[b]];
      pool.insert(pool.end(), pc.begin(), pc.end());
    }
    sort_unique(pool);
    for (int d : pool) (B.tcr_prec(b, d) ? per[L_XFAR][b] : per[L_XCLOSE][b]).push_back(d);
    if (out.is_target[b]) {
      auto U = B.list_U(b);
      sort_unique(U);
      per[L_U][b] = std::move(U);
      auto W = B.list_W(b);
      std::vector<int> wc, wf0, wf;
      for (int d : W) B.wsplit(d, b, wc, wf0);
      for (int d : wf0) {
        if (wfar_direct_max > 0 && T.sub_src[d] <= wfar_direct_max)
          B.leaves_below(d, wc);  // Remark 4: evaluate this box's sources directly
        else
          wf.push_back(d);
      }
      sort_unique(wc);
      sort_unique(wf);
      per[L_WCLOSE][b] = std::move(wc);
      per[L_WFAR][b] = std::move(wf);
    }
  }
  // X-close of pure target-ancestors is only an intermediate; keep it for export but the
  // executor uses it for target boxes only.
  for (int l = 0; l < L_NLISTS; ++l) to_csr(per[l], out.lst[l]);
}

}  // namespace gq
