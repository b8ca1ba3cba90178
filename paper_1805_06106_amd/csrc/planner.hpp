// Host-side planner for the GIGAQBX FMM: octree with target-confinement-restricted QBX
// centers (Algorithm 5, Stage 1) and the interaction lists of Section 5.2 (Lists 1-4 and
// the close/far split of Lists 3 and 4).  Plain C++17; no device code.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace gq {

struct TreeParams {
  int nmax = 512;
  double tcf = 0.9;
  int max_level = 30;
  bool tcr_linf = false;  // box-shaped target confinement region (cost comparison only)
  bool level_restrict = false;  // adjacent leaves differ by at most one level
};

// Octree.  Boxes are numbered breadth-first, children in octant order (bit 0: x upper,
// bit 1: y upper, bit 2: z upper).  Particles are renumbered in depth-first (preorder)
// order of their owning box, so every box owns a contiguous range.
struct Tree {
  int nboxes = 0;
  int nlevels = 0;
  double root_center[3] = {0, 0, 0};
  double root_h = 0;
  std::vector<double> center;  // 3 * nboxes
  std::vector<double> h;       // half-width |b|
  std::vector<int> level, parent;
  std::vector<std::array<int, 8>> child;  // -1 where pruned
  std::vector<int> nchild;
  std::vector<int64_t> ix, iy, iz;        // integer cell coordinates at the box's level
  std::vector<int> preorder;              // boxes in depth-first order
  std::vector<int> pre_index;             // box -> position in preorder
  // ownership after renumbering
  std::vector<int64_t> src_start, src_count;  // owned sources (leaves only)
  std::vector<int64_t> ctr_start, ctr_count;  // owned centers
  std::vector<int64_t> tgt_start, tgt_count;  // owned targets (boxes they end up in)
  std::vector<int64_t> sub_src;               // sources in subtree
  std::vector<int64_t> src_order;  // tree position -> input source index
  std::vector<int64_t> ctr_order;  // tree position -> input center index
  std::vector<int64_t> ctr_box;    // tree position -> owning box
  std::vector<int64_t> tgt_order;  // tree position -> input target index
  bool is_leaf(int b) const { return nchild[b] == 0; }
};

// CSR list over boxes: entries of box b are items[ptr[b] .. ptr[b+1]).
struct BoxList {
  std::vector<int64_t> ptr;
  std::vector<int> items;
  int64_t size(int b) const { return ptr[b + 1] - ptr[b]; }
  int64_t total() const { return ptr.empty() ? 0 : ptr.back(); }
};

enum ListId { L_U = 0, L_V = 1, L_WCLOSE = 2, L_WFAR = 3, L_XCLOSE = 4, L_XFAR = 5, L_NLISTS = 6 };

struct Lists {
  std::vector<uint8_t> is_target;    // box owns >= 1 center
  std::vector<uint8_t> is_owner;     // target or target-ancestor box
  BoxList lst[L_NLISTS];
};

// Builds the tree.  Returns an empty string on success, else a message.
std::string build_tree(const TreeParams& prm, int64_t n_src, const double* src_xyz,
                       int64_t n_ctr, const double* ctr_xyz, const double* ctr_radius,
                       int64_t n_tgt, const double* tgt_xyz, Tree& tree);

// Builds all interaction lists for target and target-ancestor boxes.
// wfar_direct_max > 0: List 3 far boxes with at most that many sources are replaced by
// their source leaves in List 3 close (Remark 4).
// tcr_linf: box-shaped TCR of half-width |b|(1 + t_f) instead of the ball of radius
// sqrt(3)|b|(1 + t_f) (List 3 close/far split).  point_targets[b] (optional, per box): the
// number of conventional targets (no QBX center) box b owns; such boxes are target boxes
// too.
void build_lists(const Tree& tree, double tcf, int wfar_direct_max, Lists& lists,
                 bool tcr_linf = false, const std::vector<int64_t>* point_targets = nullptr);

// Dense real-packed translation matrices in scaled form (see translations.cpp).
int ncoef(int p);
void m2m_matrix(int p, int octant, double* T);                  // child multipole -> parent
void l2l_matrix(int p, int octant, double* T);                  // parent local -> child
void m2l_matrix(int p, int ox, int oy, int oz, double* T);      // same-level, offset 2*o
// N[(p+1)^2]: sqrt((n+m)! (n-m)!) per packed index (the balancing of the FP32 translations)
void expansion_norms(int p, double* N);
// The same M2L factored as T = B Z A: A rotates multipoles so that the offset points along
// +z, Z translates along z (it couples only equal orders), B rotates locals back.  A and B
// are block diagonal by degree; all three np x np, column-major.
void m2l_rotation_factors(int p, int ox, int oy, int oz, double* A, double* Z, double* B);

}  // namespace gq
