"""Interior / boundary sets of the box tree (oracle side).

Follows Section 3.0 (matrix reordering): for a box sigma, the boundary
dofs B^sigma are those coupled to a dof outside sigma and the interior dofs
I^sigma are the rest; for DG the coupling is read from the element-block
sparsity, so the sets are unions of whole elements. Section 3.1 then
defines, for a box sigma with children mu and nu, the remaining interior
I^ hat = (B^mu u B^nu) minus B^sigma and the remaining boundary
B^ hat = B^sigma (every dof of B^sigma lies in B^mu u B^nu). The top of the
tree is a forest of two boxes; the virtual root 1 eliminates B^2 u B^3
(equation (36)).

Orderings (the paper leaves them open; this project's reading):
  * B^sigma: elements walked counter-clockwise around the box's bounding
    rectangle (bottom edge left to right, right edge bottom to top, top edge
    right to left, left edge top to bottom), then rotated so the elements
    that become interior at the parent come first as one run.
  * I^sigma of a leaf: elements in ascending id.
  * I^ hat of a merge node: [B^mu part ; B^nu part], each in its child's
    B order (the block order of equation (32)).
  * dofs: element by element, local dofs in order.
HSS tree over B^sigma: split first between the parent-interior run and the
rest, then bisect by element count (first half = floor(m/2) elements) down
to leaves of at most 4 elements.

Test infrastructure: written independently of the library's planner.
"""
from __future__ import annotations

import dataclasses

import numpy as np

HSS_LEAF_ELEMS = 4


@dataclasses.dataclass
class HssNode:
    lo: int                 # dof range [lo, hi) within B^sigma order
    hi: int
    left: "HssNode | None" = None
    right: "HssNode | None" = None

    @property
    def is_leaf(self):
        return self.left is None


@dataclasses.dataclass
class NodeSets:
    node: int
    is_leaf: bool
    elems: list                 # elements of the box (ascending)
    bnd_elems: list             # B^sigma elements in the B order above
    n_parent_interior: int      # leading elements of bnd_elems that join I^ hat(parent)
    idof: np.ndarray            # I^sigma (leaf) / I^ hat (merge) as global dofs, in order
    bdof: np.ndarray            # B^sigma global dofs, in order
    hss: "HssNode | None" = None
    height: int = 0


def depth_of(node: int) -> int:
    return int(node).bit_length() - 1


def is_ancestor_or_self(anc: int, node: int) -> bool:
    da, dn = depth_of(anc), depth_of(node)
    return dn >= da and (node >> (dn - da)) == anc


def perimeter_key(ix, iy, x0, x1, y0, y1):
    """Counter-clockwise position of a ring element of the box [x0,x1]x[y0,y1]."""
    W = x1 - x0 + 1
    H = y1 - y0 + 1
    if iy == y0:
        return ix - x0
    if ix == x1:
        return (W - 1) + (iy - y0)
    if iy == y1:
        return (W - 1) + (H - 1) + (x1 - ix)
    if ix == x0:
        return 2 * (W - 1) + (H - 1) + (y1 - iy)
    raise ValueError("boundary element not on the box perimeter")


def _bisect(lo_e: int, hi_e: int, q: int, leaf: int = HSS_LEAF_ELEMS) -> HssNode:
    node = HssNode(lo_e * q, hi_e * q)
    if hi_e - lo_e > leaf:
        mid = lo_e + (hi_e - lo_e) // 2
        node.left = _bisect(lo_e, mid, q, leaf)
        node.right = _bisect(mid, hi_e, q, leaf)
    return node


def hss_tree(m_elems: int, m_top: int, q: int, leaf: int = HSS_LEAF_ELEMS) -> HssNode:
    """HSS tree over m_elems boundary elements whose first m_top form the run
    that joins the parent's interior (m_top in {0, m_elems} means no top split);
    leaves of at most ``leaf`` elements."""
    if 0 < m_top < m_elems:
        root = HssNode(0, m_elems * q)
        root.left = _bisect(0, m_top, q, leaf)
        root.right = _bisect(m_top, m_elems, q, leaf)
        return root
    return _bisect(0, m_elems, q, leaf)


def hss_postorder(t: HssNode) -> list:
    out = []

    def rec(n):
        if n.left is not None:
            rec(n.left)
            rec(n.right)
        out.append(n)
    rec(t)
    return out


class TreeSets:
    """All sets of the box tree for one operator (structure only)."""

    def __init__(self, row_ptr, col_idx, q, tree, hss_leaf_elems: int = HSS_LEAF_ELEMS):
        self.q = int(q)
        self.hss_leaf = int(hss_leaf_elems)
        n_el = len(row_ptr) - 1
        self.n_el = n_el
        self.nbrs = [[int(c) for c in col_idx[row_ptr[e]:row_ptr[e + 1]] if c != e]
                     for e in range(n_el)]
        self.xy = np.asarray(tree.elem_xy)
        self.elem_leaf = np.full(n_el, -1, dtype=np.int64)
        leaves = {}
        for i, ln in enumerate(tree.leaf_node):
            es = [int(e) for e in tree.leaf_elems[tree.leaf_ptr[i]:tree.leaf_ptr[i + 1]]]
            leaves[int(ln)] = sorted(es)
            for e in es:
                if self.elem_leaf[e] != -1:
                    raise ValueError("element in two leaves")
                self.elem_leaf[e] = int(ln)
        if np.any(self.elem_leaf < 0):
            raise ValueError("element in no leaf")
        elems: dict[int, list] = {}
        for ln, es in leaves.items():
            s = ln
            while s >= 2:
                elems.setdefault(s, []).extend(es)
                s //= 2
        for s in elems:
            elems[s].sort()
        self.nodes = sorted(elems)
        self.leaves = set(leaves)
        for s in self.nodes:
            if s not in self.leaves and (2 * s not in elems or 2 * s + 1 not in elems):
                raise ValueError(f"node {s} lacks a child")
        if 2 not in elems or 3 not in elems:
            raise ValueError("the forest must have the two top boxes 2 and 3")
        self.elems = elems
        # boundary elements
        self.bset = {}
        for s in self.nodes:
            bs = [e for e in elems[s]
                  if any(not is_ancestor_or_self(s, int(self.elem_leaf[f])) for f in self.nbrs[e])]
            self.bset[s] = set(bs)
        # heights
        self.height = {}
        for s in sorted(self.nodes, key=lambda v: -depth_of(v)):
            if s in self.leaves:
                self.height[s] = 0
            else:
                self.height[s] = 1 + max(self.height[2 * s], self.height[2 * s + 1])
        self.sets = {}
        for s in self.nodes:
            self.sets[s] = self._node_sets(s)
        for s in self.nodes:
            if s not in self.leaves:
                self._merge_interior(s)
        self.root_idof = np.concatenate([self.sets[2].bdof, self.sets[3].bdof])

    def _dofs(self, es):
        q = self.q
        if len(es) == 0:
            return np.zeros(0, dtype=np.int64)
        return (np.asarray(es, dtype=np.int64)[:, None] * q + np.arange(q)[None, :]).reshape(-1)

    def _node_sets(self, s):
        es = self.elems[s]
        xs = self.xy[es, 0]
        ys = self.xy[es, 1]
        x0, x1, y0, y1 = int(xs.min()), int(xs.max()), int(ys.min()), int(ys.max())
        b = sorted(self.bset[s], key=lambda e: perimeter_key(int(self.xy[e, 0]), int(self.xy[e, 1]),
                                                            x0, x1, y0, y1))
        parent = s // 2
        if parent == 1:
            flags = [True] * len(b)
        else:
            flags = [e not in self.bset[parent] for e in b]
        m_top = sum(flags)
        if 0 < m_top < len(b):
            r = next(i for i in range(len(b)) if flags[i] and not flags[i - 1])
            b = b[r:] + b[:r]
            flags = flags[r:] + flags[:r]
            if not all(flags[:m_top]):
                raise ValueError("parent-interior run is not contiguous")
        ns = NodeSets(node=s, is_leaf=s in self.leaves, elems=es, bnd_elems=b,
                      n_parent_interior=m_top if parent != 1 else len(b),
                      idof=np.zeros(0, dtype=np.int64), bdof=self._dofs(b),
                      height=self.height[s])
        ns.hss = hss_tree(len(b), m_top if parent != 1 else 0, self.q, self.hss_leaf)
        if ns.is_leaf:
            ns.idof = self._dofs([e for e in es if e not in self.bset[s]])
        return ns

    def _merge_interior(self, s):
        mu, nu = self.sets[2 * s], self.sets[2 * s + 1]
        ie = mu.bnd_elems[:mu.n_parent_interior] + nu.bnd_elems[:nu.n_parent_interior]
        self.sets[s].idof = self._dofs(ie)

    def elimination_order(self):
        """Nodes by height, then heap id: the height-wave order."""
        return sorted(self.nodes, key=lambda v: (self.height[v], v))
