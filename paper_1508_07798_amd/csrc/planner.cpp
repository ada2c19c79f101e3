// Host planner (see planner.hpp for the sets and orderings it computes).
#include "planner.hpp"

#include <algorithm>
#include <map>
#include <unordered_map>

#include "common.hpp"

namespace hss {

namespace {

int depth_of(int node) {
  int d = -1;
  while (node) {
    node >>= 1;
    ++d;
  }
  return d;
}

bool inside(int box, int leaf) {
  int db = depth_of(box), dl = depth_of(leaf);
  return dl >= db && (leaf >> (dl - db)) == box;
}

[[noreturn]] void bad(const std::string& m) { throw Error(HSS_EINVAL, m); }

// Counter-clockwise perimeter position of a ring element of [x0,x1]x[y0,y1].
int64_t perimeter_key(int ix, int iy, int x0, int x1, int y0, int y1) {
  int64_t W = x1 - x0 + 1, H = y1 - y0 + 1;
  if (iy == y0) return ix - x0;
  if (ix == x1) return (W - 1) + (iy - y0);
  if (iy == y1) return (W - 1) + (H - 1) + (x1 - ix);
  if (ix == x0) return 2 * (W - 1) + (H - 1) + (y1 - iy);
  bad("a boundary element of a box is not on the box perimeter");
}

int bisect(std::vector<HssNode>& out, int lo_e, int hi_e, int q, int leaf) {
  if (hi_e - lo_e <= leaf) {
    out.push_back({lo_e * q, hi_e * q, -1, -1, 0});
    return (int)out.size() - 1;
  }
  int mid = lo_e + (hi_e - lo_e) / 2;
  int l = bisect(out, lo_e, mid, q, leaf);
  int r = bisect(out, mid, hi_e, q, leaf);
  out.push_back({lo_e * q, hi_e * q, l, r, 1 + std::max(out[l].height, out[r].height)});
  return (int)out.size() - 1;
}

void build_hss(PNode& nd, int q, bool split_top, int leaf) {
  int m = (int)nd.bnd_elems.size();
  nd.hss.clear();
  if (m == 0) return;
  if (split_top && nd.n_top > 0 && nd.n_top < m) {
    int l = bisect(nd.hss, 0, nd.n_top, q, leaf);
    int r = bisect(nd.hss, nd.n_top, m, q, leaf);
    nd.hss.push_back({0, m * q, l, r, 1 + std::max(nd.hss[l].height, nd.hss[r].height)});
  } else {
    bisect(nd.hss, 0, m, q, leaf);
  }
}

void dofs_of(const std::vector<int>& el, int q, std::vector<int64_t>& out) {
  out.clear();
  out.reserve(el.size() * q);
  for (int e : el)
    for (int k = 0; k < q; ++k) out.push_back((int64_t)e * q + k);
}

}  // namespace

int Plan::find(int prob, int heap) const {
  for (size_t i = 0; i < nodes.size(); ++i)
    if (nodes[i].prob == prob && nodes[i].heap == heap) return (int)i;
  return -1;
}

Plan make_plan(int nprob, const hss_block_op_t* A, const hss_tree_t* T, int hss_leaf_elems) {
  if (hss_leaf_elems < 1) bad("HSS leaf size must be at least one element");
  if (nprob < 1 || !A || !T) bad("null operator / tree or nprob < 1");
  Plan P;
  P.probs.resize(nprob);
  int64_t dof_off = 0, el_off = 0, blk_off = 0;
  for (int p = 0; p < nprob; ++p) {
    const hss_block_op_t& a = A[p];
    const hss_tree_t& t = T[p];
    PProblem& pr = P.probs[p];
    if (a.n_el < 2 || a.q < 1 || !a.row_ptr || !a.col_idx || !a.vals)
      bad("operator " + std::to_string(p) + ": bad sizes or null arrays");
    if (a.dtype != HSS_R64 && a.dtype != HSS_C128) bad("unknown dtype");
    if (a.dtype != A[0].dtype) bad("all problems of a batch must share one dtype");
    if (!t.leaf_node || !t.leaf_ptr || !t.leaf_elems || !t.elem_xy || t.n_leaves < 2)
      bad("tree " + std::to_string(p) + ": null arrays or fewer than two leaves");
    pr.n_el = a.n_el;
    pr.q = a.q;
    pr.ndof = (int64_t)a.n_el * a.q;
    pr.dof_off = dof_off;
    pr.el_off = el_off;
    pr.blk_off = blk_off;
    pr.row_ptr.assign(a.row_ptr, a.row_ptr + a.n_el + 1);
    if (pr.row_ptr[0] != 0) bad("row_ptr[0] != 0");
    for (int e = 0; e < a.n_el; ++e)
      if (pr.row_ptr[e + 1] < pr.row_ptr[e]) bad("row_ptr not monotone");
    int nnzb = pr.row_ptr[a.n_el];
    pr.col_idx.assign(a.col_idx, a.col_idx + nnzb);
    pr.diag_blk.assign(a.n_el, -1);
    for (int e = 0; e < a.n_el; ++e)
      for (int b = pr.row_ptr[e]; b < pr.row_ptr[e + 1]; ++b) {
        int c = pr.col_idx[b];
        if (c < 0 || c >= a.n_el) bad("col_idx out of range");
        if (b > pr.row_ptr[e] && pr.col_idx[b - 1] >= c) bad("col_idx not ascending in a row");
        if (c == e) pr.diag_blk[e] = b;
      }
    // the sets need a structurally symmetric operator; the block (c, e) of every
    // block (e, c) is recorded for the value-symmetry check
    pr.tblk.assign(nnzb, -1);
    for (int e = 0; e < a.n_el; ++e)
      for (int b = pr.row_ptr[e]; b < pr.row_ptr[e + 1]; ++b) {
        int c = pr.col_idx[b];
        const int32_t* beg = pr.col_idx.data() + pr.row_ptr[c];
        const int32_t* end = pr.col_idx.data() + pr.row_ptr[c + 1];
        const int32_t* it = std::lower_bound(beg, end, e);
        if (it == end || *it != e) throw Error(HSS_EUNSUPPORTED, "structurally nonsymmetric operator");
        pr.tblk[b] = (int32_t)(it - pr.col_idx.data());
      }
    // leaves
    pr.elem_leaf.assign(a.n_el, -1);
    std::map<int, std::vector<int>> box_elems;
    for (int i = 0; i < t.n_leaves; ++i) {
      int ln = t.leaf_node[i];
      if (ln < 2) bad("leaf heap id < 2");
      if (t.leaf_ptr[i + 1] < t.leaf_ptr[i]) bad("leaf_ptr not monotone");
      for (int k = t.leaf_ptr[i]; k < t.leaf_ptr[i + 1]; ++k) {
        int e = t.leaf_elems[k];
        if (e < 0 || e >= a.n_el) bad("leaf element out of range");
        if (pr.elem_leaf[e] != -1) bad("element in two leaves");
        pr.elem_leaf[e] = ln;
        for (int s = ln; s >= 2; s >>= 1) box_elems[s].push_back(e);
      }
    }
    if (t.leaf_ptr[0] != 0 || t.leaf_ptr[t.n_leaves] != a.n_el) bad("leaf_ptr does not cover the elements");
    for (int e = 0; e < a.n_el; ++e)
      if (pr.elem_leaf[e] < 0) bad("element in no leaf");
    std::vector<int> leafset(t.leaf_node, t.leaf_node + t.n_leaves);
    std::sort(leafset.begin(), leafset.end());
    for (size_t i = 1; i < leafset.size(); ++i)
      if (leafset[i] == leafset[i - 1]) bad("duplicate leaf id");
    if (!box_elems.count(2) || !box_elems.count(3)) bad("boxes 2 and 3 must both exist");
    for (auto& kv : box_elems) {
      int s = kv.first;
      bool is_leaf = std::binary_search(leafset.begin(), leafset.end(), s);
      if (is_leaf) {
        if (box_elems.count(2 * s) || box_elems.count(2 * s + 1)) bad("a leaf has descendants");
      } else if (!box_elems.count(2 * s) || !box_elems.count(2 * s + 1)) {
        bad("box " + std::to_string(s) + " lacks a child");
      }
    }
    // boxes, children before parents (deepest first)
    std::vector<int> heaps;
    for (auto& kv : box_elems) heaps.push_back(kv.first);
    std::sort(heaps.begin(), heaps.end(), [](int x, int y) {
      int dx = depth_of(x), dy = depth_of(y);
      return dx != dy ? dx > dy : x < y;
    });
    std::unordered_map<int, int> gidx;
    std::unordered_map<int, std::vector<char>> is_b;  // per box: element -> in B (dense over box elems)
    const int32_t* xy = t.elem_xy;
    std::vector<int> first_g(heaps.size());
    // B sets
    std::map<int, std::vector<char>> bflag;  // heap -> flag per element id (sparse via map of vectors)
    std::vector<char> inb;
    for (int s : heaps) {
      PNode nd;
      nd.prob = p;
      nd.heap = s;
      nd.depth = depth_of(s);
      nd.leaf = std::binary_search(leafset.begin(), leafset.end(), s);
      nd.elems = box_elems[s];
      std::sort(nd.elems.begin(), nd.elems.end());
      int x0 = 1 << 30, x1 = -1, y0 = 1 << 30, y1 = -1;
      for (int e : nd.elems) {
        x0 = std::min(x0, xy[2 * e]);
        x1 = std::max(x1, xy[2 * e]);
        y0 = std::min(y0, xy[2 * e + 1]);
        y1 = std::max(y1, xy[2 * e + 1]);
      }
      std::vector<std::pair<int64_t, int>> ring;
      for (int e : nd.elems) {
        bool bnd = false;
        for (int b = pr.row_ptr[e]; b < pr.row_ptr[e + 1] && !bnd; ++b) {
          int f = pr.col_idx[b];
          if (f != e && !inside(s, pr.elem_leaf[f])) bnd = true;
        }
        if (bnd) ring.push_back({perimeter_key(xy[2 * e], xy[2 * e + 1], x0, x1, y0, y1), e});
      }
      std::sort(ring.begin(), ring.end());
      for (size_t i = 1; i < ring.size(); ++i)
        if (ring[i].first == ring[i - 1].first) bad("two boundary elements share a perimeter position");
      for (auto& r : ring) nd.bnd_elems.push_back(r.second);
      gidx[s] = (int)P.nodes.size();
      P.nodes.push_back(std::move(nd));
    }
    // rotation to the parent-interior run, HSS trees, interiors
    auto in_parent_b = [&](int s, int e) {
      // e in B^{parent(s)}: some neighbour outside the parent box
      int par = s >> 1;
      for (int b = pr.row_ptr[e]; b < pr.row_ptr[e + 1]; ++b) {
        int f = pr.col_idx[b];
        if (f != e && !inside(par, pr.elem_leaf[f])) return true;
      }
      return false;
    };
    for (int s : heaps) {
      PNode& nd = P.nodes[gidx[s]];
      int m = (int)nd.bnd_elems.size();
      bool top = (s >> 1) == 1;
      if (top) {
        nd.n_top = m;
      } else {
        std::vector<char> fl(m);
        int cnt = 0;
        for (int i = 0; i < m; ++i) cnt += (fl[i] = !in_parent_b(s, nd.bnd_elems[i]));
        nd.n_top = cnt;
        if (cnt > 0 && cnt < m) {
          int r = -1;
          for (int i = 0; i < m; ++i)
            if (fl[i] && !fl[(i + m - 1) % m]) {
              r = i;
              break;
            }
          std::rotate(nd.bnd_elems.begin(), nd.bnd_elems.begin() + r, nd.bnd_elems.end());
          std::rotate(fl.begin(), fl.begin() + r, fl.end());
          for (int i = 0; i < cnt; ++i)
            if (!fl[i]) bad("parent-interior run of a box is not contiguous");
        }
      }
      build_hss(nd, pr.q, !top, hss_leaf_elems);
      dofs_of(nd.bnd_elems, pr.q, nd.bdof);
      if (nd.leaf) {
        std::vector<char> isb(0);
        std::vector<int> ie;
        std::vector<int> sb = nd.bnd_elems;
        std::sort(sb.begin(), sb.end());
        for (int e : nd.elems)
          if (!std::binary_search(sb.begin(), sb.end(), e)) ie.push_back(e);
        dofs_of(ie, pr.q, nd.idof);
      }
    }
    // merge boxes: I^ and the gather sources
    std::vector<int32_t> where(pr.ndof, -1);
    for (int s : heaps) {
      PNode& nd = P.nodes[gidx[s]];
      if (nd.leaf) continue;
      int gm = gidx[2 * s], gn = gidx[2 * s + 1];
      nd.child[0] = gm;
      nd.child[1] = gn;
      P.nodes[gm].parent = gidx[s];
      P.nodes[gn].parent = gidx[s];
      const PNode& mu = P.nodes[gm];
      const PNode& nu = P.nodes[gn];
      std::vector<int> ie(mu.bnd_elems.begin(), mu.bnd_elems.begin() + mu.n_top);
      ie.insert(ie.end(), nu.bnd_elems.begin(), nu.bnd_elems.begin() + nu.n_top);
      dofs_of(ie, pr.q, nd.idof);
      for (size_t k = 0; k < mu.bdof.size(); ++k) where[mu.bdof[k]] = (int32_t)k;
      for (size_t k = 0; k < nu.bdof.size(); ++k) where[nu.bdof[k]] = (int32_t)((1 << 30) + k);
      nd.isrc.resize(nd.idof.size());
      nd.bsrc.resize(nd.bdof.size());
      for (size_t k = 0; k < nd.idof.size(); ++k) {
        if (where[nd.idof[k]] < 0) bad("internal: I^ dof not in the children's B");
        nd.isrc[k] = where[nd.idof[k]];
      }
      for (size_t k = 0; k < nd.bdof.size(); ++k) {
        if (where[nd.bdof[k]] < 0) bad("internal: B dof not in the children's B");
        nd.bsrc[k] = where[nd.bdof[k]];
      }
      for (int64_t d : mu.bdof) where[d] = -1;
      for (int64_t d : nu.bdof) where[d] = -1;
    }
    // heights
    for (int s : heaps) {
      PNode& nd = P.nodes[gidx[s]];
      nd.height = nd.leaf ? 0
                          : 1 + std::max(P.nodes[nd.child[0]].height, P.nodes[nd.child[1]].height);
      pr.max_height = std::max(pr.max_height, nd.height);
    }
    // root
    PRoot rt;
    rt.prob = p;
    rt.g2 = gidx[2];
    rt.g3 = gidx[3];
    rt.dofs = P.nodes[rt.g2].bdof;
    rt.dofs.insert(rt.dofs.end(), P.nodes[rt.g3].bdof.begin(), P.nodes[rt.g3].bdof.end());
    // tree order: boxes by (height, heap id), root last
    std::vector<int> order;
    for (int s : heaps) order.push_back(gidx[s]);
    std::sort(order.begin(), order.end(), [&](int x, int y) {
      const PNode &a1 = P.nodes[x], &b1 = P.nodes[y];
      return a1.height != b1.height ? a1.height < b1.height : a1.heap < b1.heap;
    });
    std::vector<int64_t> tpos(pr.ndof, -1);
    pr.perm.clear();
    pr.perm.reserve(pr.ndof);
    for (int g : order) {
      PNode& nd = P.nodes[g];
      nd.ipos = (int64_t)pr.perm.size();
      for (int64_t d : nd.idof) {
        tpos[d] = (int64_t)pr.perm.size();
        pr.perm.push_back(d);
      }
    }
    rt.ipos = (int64_t)pr.perm.size();
    for (int64_t d : rt.dofs) {
      tpos[d] = (int64_t)pr.perm.size();
      pr.perm.push_back(d);
    }
    if ((int64_t)pr.perm.size() != pr.ndof) bad("internal: dofs not eliminated exactly once");
    for (int64_t d = 0; d < pr.ndof; ++d)
      if (tpos[d] < 0) bad("internal: dof without a tree position");
    for (int g : order) {
      PNode& nd = P.nodes[g];
      nd.bpos.resize(nd.bdof.size());
      for (size_t k = 0; k < nd.bdof.size(); ++k) nd.bpos[k] = tpos[nd.bdof[k]];
    }
    P.roots.push_back(std::move(rt));
    P.q_max = std::max(P.q_max, pr.q);
    dof_off += pr.ndof;
    el_off += a.n_el;
    blk_off += (int64_t)nnzb;
  }
  P.ndof_total = dof_off;
  int hmax = 0;
  for (auto& nd : P.nodes) hmax = std::max(hmax, nd.height);
  P.waves.assign(hmax + 1, {});
  for (size_t g = 0; g < P.nodes.size(); ++g) P.waves[P.nodes[g].height].push_back((int)g);
  flatten(P);
  return P;
}

void flatten(Plan& P) {
  P.dev_cache = std::make_shared<Plan::DevCache>();  // copies of older index arrays do not apply
  PlanFlat& F = P.flat;
  F = PlanFlat{};
  const int nprob = (int)P.probs.size();
  F.row_ptr.push_back(0);
  F.seg.push_back(0);
  for (int p = 0; p < nprob; ++p) {
    const PProblem& pr = P.probs[p];
    for (int e = 0; e < pr.n_el; ++e) {
      for (int b = pr.row_ptr[e]; b < pr.row_ptr[e + 1]; ++b) {
        F.col_idx.push_back((int32_t)(pr.el_off + pr.col_idx[b]));
        F.tblk.push_back((int32_t)(pr.blk_off + pr.tblk[b]));
      }
      F.row_ptr.push_back((int32_t)F.col_idx.size());
      F.elem_dof.push_back(pr.dof_off + (int64_t)e * pr.q);
      for (int k = 0; k < pr.q; ++k) {
        F.dof_elem.push_back((int32_t)(pr.el_off + e));
        F.dof_prob.push_back(p);
      }
    }
    F.seg.push_back(pr.dof_off + pr.ndof);
  }
  F.perm.assign(P.ndof_total, 0);
  for (int p = 0; p < nprob; ++p) {
    const PProblem& pr = P.probs[p];
    for (int64_t t = 0; t < pr.ndof; ++t) F.perm[pr.dof_off + t] = pr.dof_off + pr.perm[t];
  }
  const int nn = (int)P.nodes.size();
  F.goff.resize(nn);
  F.soff.resize(nn);
  F.boff.resize(nn);
  F.foff.resize(nn);
  F.aoff.resize(nn);
  F.poff.resize(nn);
  for (int g = 0; g < nn; ++g) {
    const PNode& n = P.nodes[g];
    const PProblem& pr = P.probs[n.prob];
    F.goff[g] = F.gidx.size();
    for (auto d : n.idof) F.gidx.push_back(pr.dof_off + d);
    for (auto d : n.bdof) F.gidx.push_back(pr.dof_off + d);
    F.soff[g] = F.src.size();
    if (!n.leaf) {
      F.src.insert(F.src.end(), n.isrc.begin(), n.isrc.end());
      F.src.insert(F.src.end(), n.bsrc.begin(), n.bsrc.end());
    }
    F.boff[g] = F.bpos.size();
    for (auto b : n.bpos) F.bpos.push_back(pr.dof_off + b);
    const size_t ni = n.idof.size(), nbd = n.bdof.size();
    F.foff[g] = F.fsz;
    F.fsz += ((ni * (ni + nbd) + 63) / 64) * 64;
    F.aoff[g] = F.fsz;
    F.fsz += ((nbd * ni + 63) / 64) * 64;
    F.poff[g] = F.psz;
    F.psz += ((ni + 63) / 64) * 64;
  }
}

}  // namespace hss
