"""Hierarchical box decompositions (input generation only).

The paper organises the sub-domains into a binary tree: the root is the whole
domain, every internal node splits its box in two, the leaves are the "true"
sub-domains and every internal node also stands for the interface between its
children (Section 2, Fig. 1).  This module generalises that construction to
axis-aligned cut planes in 2-D and 3-D (a node may cut along several axes,
giving 2^k children; an octree cuts along all three) and emits the two arrays
the RSD library takes as its description of the hierarchy:

* ``parent``   int32[T]: parent[0] = -1 and parent[t] < t (breadth-first ids);
* ``dof_node`` int32[n]: for each dof, the leaf whose interior holds it, or the
  internal node whose interface (cut planes) holds it.

A free grid node lying on several cut planes belongs to the shallowest node
whose cut plane contains it; otherwise it belongs to the leaf whose open box
contains it.  All dofs of a grid node share its tree node.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class BoxTree:
    parent: np.ndarray          # int32[T]
    depth: np.ndarray           # int32[T]
    lo: np.ndarray              # int64[T, dim] lower bounding node plane
    hi: np.ndarray              # int64[T, dim] upper bounding node plane
    cut: np.ndarray             # int64[T, dim] cut plane per axis, -1 if none
    children: list = field(default_factory=list)

    @property
    def num_nodes(self) -> int:
        return len(self.parent)

    def is_leaf(self, t: int) -> bool:
        return len(self.children[t]) == 0


def build_box_tree(shape_nodes: tuple, height: int, axes_per_level=None, cut_fn=None) -> BoxTree:
    """Breadth-first cut-plane tree over the node box [0, n_d - 1] per axis.

    axes_per_level(depth) -> tuple of axes cut at that depth (default: all axes).
    cut_fn(t_depth, axis, lo, hi) -> plane index strictly inside (lo, hi)
    (default: (lo + hi) // 2).
    """
    dim = len(shape_nodes)
    if axes_per_level is None:
        axes_per_level = lambda d: tuple(range(dim))  # noqa: E731
    if cut_fn is None:
        cut_fn = lambda depth, axis, lo, hi: (lo + hi) // 2  # noqa: E731
    parent, depth, lo, hi, cut, children = [-1], [0], [[0] * dim], [[s - 1 for s in shape_nodes]], [], []
    t = 0
    while t < len(parent):
        d = depth[t]
        c = [-1] * dim
        kids = []
        if d < height:
            axes = axes_per_level(d)
            for a in axes:
                m = cut_fn(d, a, lo[t][a], hi[t][a])
                if not (lo[t][a] < m < hi[t][a]):
                    raise ValueError("cut plane outside the box")
                c[a] = m
            for code in range(2 ** len(axes)):
                clo, chi = list(lo[t]), list(hi[t])
                for bit, a in enumerate(axes):
                    if (code >> bit) & 1:
                        clo[a] = c[a]
                    else:
                        chi[a] = c[a]
                kids.append(len(parent))
                parent.append(t)
                depth.append(d + 1)
                lo.append(clo)
                hi.append(chi)
        cut.append(c)
        children.append(kids)
        t += 1
    return BoxTree(np.array(parent, dtype=np.int32), np.array(depth, dtype=np.int32),
                   np.array(lo, dtype=np.int64), np.array(hi, dtype=np.int64),
                   np.array(cut, dtype=np.int64), children)


def assign_nodes(tree: BoxTree, ijk: np.ndarray) -> np.ndarray:
    """Tree node of each grid node (rows of ijk), by the ownership rule above."""
    m = ijk.shape[0]
    first_child = np.array([ch[0] if ch else -1 for ch in tree.children], dtype=np.int64)
    owner = np.zeros(m, dtype=np.int64)
    active = np.ones(m, dtype=bool)
    while active.any():
        idx = np.nonzero(active)[0]
        t = owner[idx]
        c = tree.cut[t]                                     # (k, dim)
        has_cut = c >= 0
        on_plane = np.any(has_cut & (ijk[idx] == c), axis=1)
        leaf = ~has_cut.any(axis=1)
        stop = on_plane | leaf
        active[idx[stop]] = False
        go = idx[~stop]
        if go.size == 0:
            break
        tg = owner[go]
        cg = tree.cut[tg]
        code = np.zeros(go.size, dtype=np.int64)
        bit = np.zeros(go.size, dtype=np.int64)
        for a in range(ijk.shape[1]):
            use = cg[:, a] >= 0
            code += np.where(use, (ijk[go, a] > cg[:, a]).astype(np.int64) << bit, 0)
            bit += use
        owner[go] = first_child[tg] + code
    return owner


def dof_node_map(tree: BoxTree, free_ijk: np.ndarray, ndof: int) -> np.ndarray:
    """dof_node int32[n] for node-major dof numbering with ndof dofs per grid node."""
    owner = assign_nodes(tree, free_ijk)
    return np.repeat(owner, ndof).astype(np.int32)
