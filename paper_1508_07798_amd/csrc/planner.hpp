// Host planner: boxes, interior / boundary sets, orderings, height waves and
// HSS trees for one or more element-block operators.
//
// Section 3.0 defines the boundary dofs B of a box as those coupled to dofs
// outside it and the interior dofs I as the rest; for DG the coupling is the
// element-block sparsity, so both are unions of whole elements. Section 3.1
// defines, for a box with children mu and nu, I^ = (B^mu u B^nu) \ B and
// B^ = B (every dof of B is in B^mu u B^nu). The forest's two top boxes meet
// in the root block of equation (36).
//
// Orderings (not fixed by the paper):
//   B: elements counter-clockwise around the box's bounding rectangle,
//      rotated so that the elements that join the parent's I^ come first as
//      one run; I of a leaf: ascending element id; I^ of a merge node:
//      [B^mu part ; B^nu part] in the children's B order (the block order of
//      equation (32)); within an element, local dof order.
//   HSS tree over B: first split between that leading run and the rest,
//      then bisection by element count (first half floor(m/2)) down to
//      leaves of at most 4 elements.
//   Waves: boxes grouped by height (leaves 0); eliminating wave by wave
//      gives the same factors as the paper's level-by-level loop.
#pragma once

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hss.h"

namespace hss {

constexpr int kHssLeafElems = 4;  // default HSS leaf size over a box's boundary, in elements

struct HssNode {
  int lo, hi;        // dof range in the box's B order
  int left, right;   // indices into the box's HSS node list, -1 for leaves
  int height;        // 0 for leaves
};

struct PNode {
  int prob = 0, heap = 0, height = 0, depth = 0;
  int parent = -1;          // global index of the parent box, -1 below the virtual root
  int child[2] = {-1, -1};  // global indices of the children (merge boxes)
  bool leaf = false;
  std::vector<int> elems;       // ascending
  std::vector<int> bnd_elems;   // B order
  int n_top = 0;                // leading B elements that join the parent's I^
  std::vector<int64_t> idof;    // local dofs of I (leaf) / I^ (merge), factor order
  std::vector<int64_t> bdof;    // local dofs of B, B order
  std::vector<HssNode> hss;     // post-order, last entry is the HSS root
  // merge boxes: source of every I^ and B entry in the children's B order,
  // encoded as side * 2^30 + position
  std::vector<int32_t> isrc, bsrc;
  // tree-order positions (within the problem's segment)
  int64_t ipos = 0;             // I^ occupies [ipos, ipos + idof.size())
  std::vector<int64_t> bpos;    // tree position of every B dof
};

struct PRoot {
  int prob = 0;
  int g2 = -1, g3 = -1;         // global indices of boxes 2 and 3
  std::vector<int64_t> dofs;    // [B^2 ; B^3]
  int64_t ipos = 0;
};

struct PProblem {
  int n_el = 0, q = 0;
  int64_t ndof = 0, dof_off = 0;
  int64_t el_off = 0, blk_off = 0;
  std::vector<int32_t> row_ptr, col_idx;
  std::vector<int32_t> diag_blk;     // block index of (e, e) per element
  std::vector<int32_t> tblk;         // per block (e, f): index of the block (f, e)
  std::vector<int32_t> elem_leaf;    // heap id of the leaf holding each element
  std::vector<int64_t> perm;         // perm[tree position] = local dof
  int max_height = 0;
};

// Index arrays of a plan in the layout the device uses, built once with the plan
// (they depend on the structure only).
struct PlanFlat {
  // operator, all problems concatenated: element CSR with global element ids, first
  // dof of each element, problem segment offsets, element and problem of every dof,
  // and tree position -> global dof
  std::vector<int32_t> row_ptr, col_idx, dof_elem, dof_prob;
  std::vector<int64_t> elem_dof, seg, perm;
  std::vector<int32_t> tblk;  // per block (global index): the transposed block
  // per box: interior + boundary dofs (global), merge sources, parent positions,
  // each with its offset into the concatenation
  std::vector<int64_t> gidx, bpos;
  std::vector<int32_t> src;
  std::vector<size_t> goff, soff, boff;
  // factor storage per box: [A^_ii^-1 | X] at foff, A^_bi at aoff (64-element
  // aligned, total fsz), row permutation at poff (total psz)
  std::vector<size_t> foff, aoff, poff;
  size_t fsz = 0, psz = 0;
};

struct Plan {
  std::vector<PProblem> probs;
  std::vector<PNode> nodes;
  std::vector<std::vector<int>> waves;   // waves[h] = global box indices of height h
  std::vector<PRoot> roots;              // one per problem
  int64_t ndof_total = 0;
  int q_max = 0;
  PlanFlat flat;
  // Device copies of flat's index arrays, one set per device, made by the first
  // factorization on that device and shared by the later ones (the arrays depend
  // on the structure only). The set's owner frees it when the plan goes.
  struct DevSlot {
    int dev;
    std::shared_ptr<void> data;
  };
  struct DevCache {
    std::mutex mu;
    std::vector<DevSlot> slots;
  };
  std::shared_ptr<DevCache> dev_cache = std::make_shared<DevCache>();
  int find(int prob, int heap) const;
};

// Fills plan.flat from the rest of the plan.
void flatten(Plan& plan);

// Builds the plan; throws hss::Error(HSS_EINVAL / HSS_EUNSUPPORTED, msg) on bad input.
Plan make_plan(int nprob, const hss_block_op_t* A, const hss_tree_t* T, int hss_leaf_elems = kHssLeafElems);

}  // namespace hss
