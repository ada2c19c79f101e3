"""Binary box partition of an n x m element grid (the separator-tree input).

The paper partitions the dofs by a binary tree of geometric boxes and notes
that the top of the tree is a forest of two boxes (Section 3.0, the box
figure and its footnote on the missing root). The tree here is heap
numbered: node 1 is a virtual root that owns no box of its own, its
children 2 and 3 are the two top-level boxes, node s has children 2s and
2s+1, and leaves may sit at different depths.

Cut rule: the first cut splits y (as in the box-partition panel of the
partition-scheme figure of Section 4); afterwards the longer side is cut,
and a tie cuts the direction the parent did not. A side of length L is
split at floor(L/2). Cutting stops once a box holds <= ``leaf_elems``
elements. Other schemes (horizontal or vertical slabs) are selected with
``scheme``.

Only this file decides the partition; both the oracle and the library
take its output as input.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Box:
    node: int
    x0: int
    x1: int  # exclusive
    y0: int
    y1: int  # exclusive
    cut: str  # direction of the cut that created this box ("x" or "y")

    @property
    def w(self):
        return self.x1 - self.x0

    @property
    def h(self):
        return self.y1 - self.y0


@dataclasses.dataclass
class Tree:
    """Leaves of the box tree (the separator-tree input of the factorisation)."""

    leaf_node: np.ndarray   # int32 [n_leaves], heap ids
    leaf_ptr: np.ndarray    # int32 [n_leaves + 1]
    leaf_elems: np.ndarray  # int32 [n_el], elements of each leaf, ascending
    elem_xy: np.ndarray     # int32 [n_el, 2] integer element coordinates (ix, iy)
    boxes: dict             # node -> Box (all nodes except the virtual root)

    @property
    def n_leaves(self):
        return int(self.leaf_node.size)


def build_tree(nx: int, ny: int | None = None, leaf_elems: int = 16,
               scheme: str = "boxes") -> Tree:
    if ny is None:
        ny = nx
    if nx < 2 or ny < 2:
        raise ValueError("grid must be at least 2 x 2 elements")
    boxes: dict[int, Box] = {}
    leaves: list[Box] = []

    def split(b: Box, direction: str):
        if direction == "x":
            xm = b.x0 + b.w // 2
            return (Box(2 * b.node, b.x0, xm, b.y0, b.y1, "x"),
                    Box(2 * b.node + 1, xm, b.x1, b.y0, b.y1, "x"))
        ym = b.y0 + b.h // 2
        return (Box(2 * b.node, b.x0, b.x1, b.y0, ym, "y"),
                Box(2 * b.node + 1, b.x0, b.x1, ym, b.y1, "y"))

    def choose(b: Box) -> str | None:
        if b.w * b.h <= leaf_elems:
            return None
        if scheme == "hslabs":      # horizontal slabs: always cut y
            return "y" if b.h >= 2 else None
        if scheme == "vslabs":      # vertical slabs: always cut x
            return "x" if b.w >= 2 else None
        if b.w > b.h:
            return "x"
        if b.h > b.w:
            return "y"
        return "y" if b.cut == "x" else "x"

    root = Box(1, 0, nx, 0, ny, "x")
    first = "y" if scheme != "vslabs" else "x"
    stack = list(split(root, first))
    while stack:
        b = stack.pop()
        boxes[b.node] = b
        d = choose(b)
        if d is None:
            leaves.append(b)
        else:
            stack.extend(split(b, d))
    leaves.sort(key=lambda b: b.node)
    leaf_node = np.array([b.node for b in leaves], dtype=np.int32)
    ptr = [0]
    elems = []
    for b in leaves:
        es = [ix + nx * iy for iy in range(b.y0, b.y1) for ix in range(b.x0, b.x1)]
        es.sort()
        elems.extend(es)
        ptr.append(len(elems))
    xy = np.array([[e % nx, e // nx] for e in range(nx * ny)], dtype=np.int32)
    return Tree(leaf_node=leaf_node, leaf_ptr=np.asarray(ptr, dtype=np.int32),
                leaf_elems=np.asarray(elems, dtype=np.int32), elem_xy=xy, boxes=boxes)
