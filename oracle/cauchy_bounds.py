"""Certified row-norm upper bounds for Cauchy-like matrices and the
rejection-sampled row draw, FP64 / complex128.

TEST INFRASTRUCTURE: part of the CPU oracle. Only tests, the smoke check and
the bench's CPU-baseline leg may import it; the product path never does, and
it shares no code with the HIP path.

What it computes (App. C, row norm bounds; Alg. 3, Step 1):

* Two quadtrees, on the target points x (rows) and the source points y
  (columns), and for every target leaf l two interaction lists built by a
  dual-tree traversal (Alg. C.1): A_l holds (source node s, alpha =
  1 / d_min^2(s, l)) for source nodes far enough from l that
  d_max^2 <= nu d_min^2 held for the pair of nodes where the traversal met
  them; E_l holds the source leaves handled pair by pair.
* For generators G, B: the Gram matrices H_s = sum_{j in s} B_:,j B_:,j^* of
  every source node, bottom-up, and the bounds (Alg. C.2)
      u_i = sum_{(s, alpha) in A_l} alpha G_i,: H_s G_i,:^*
            + sum_{s in E_l} sum_{j in s} |G_i,: B_:,j|^2 / |x_i - y_j|^2,
  which satisfy ||S_i,:||^2 <= u_i <= nu ||S_i,:||^2 (App. C).

Readings where the paper is silent (each also listed in the design notes):

* A node's box is the tight axis-aligned bounding box of its points (real
  and imaginary parts as the two axes). A node with more than `leaf` points
  and a box of positive extent is split at the midpoint of its box into the
  four quadrants, a point going to the upper (right) side when its
  coordinate is >= the midpoint; empty quadrants are dropped; children in
  quadrant order (lower-left, lower-right, upper-left, upper-right); points
  keep their relative order.
* size(node) = the longer side of its box; d_min^2 and d_max^2 of two nodes
  are the smallest and largest squared distances between points of their
  two boxes.
* When the pair (s, t) is neither admissible nor a pair of leaves, the
  traversal splits t if t is not a leaf and (s is a leaf or size(t) >=
  size(s)), else s: the printed rule (split the larger) would drop the pair
  when the larger node is a leaf. The stack pops the last pushed pair;
  children are pushed in quadrant order.
* Rejection sampling (Alg. 3, Step 1): trial q of step t uses the Philox
  block of counter (t, stream, q, 0): its word w0 draws the row i from the
  bounds (inverse CDF, as in the exact form), its word w2 gives the
  acceptance uniform v, and the row is accepted when v u_i < rho_i =
  ||S_i,:||^2 (probability rho_i / u_i). The column draw uses w1 of the
  block of trial 0 (the words of one block are independent). At most
  MAX_TRIALS trials per step.
* With bounds, the stop test runs on the bound total U = sum_i u_i: the
  tolerance stop fires when U <= (tol^2 / nu) U_0. Since ||S||_F^2 <= U and
  U_0 <= nu ||A||_F^2, the stop certifies ||S||_F <= tol ||A||_F.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

MAX_TRIALS = 256


@dataclass
class Node:
    lo: Tuple[float, float]          # box corner (re, im)
    hi: Tuple[float, float]
    idx: np.ndarray                  # point indices, in tree order
    children: List[int] = field(default_factory=list)

    @property
    def leaf(self) -> bool:
        return not self.children


def _box(pts: np.ndarray):
    return ((float(pts.real.min()), float(pts.imag.min())),
            (float(pts.real.max()), float(pts.imag.max())))


def build_quadtree(points: np.ndarray, leaf: int) -> List[Node]:
    """Nodes in creation order (node 0 is the root); see the module notes."""
    points = np.asarray(points, dtype=np.complex128)
    nodes: List[Node] = []

    def make(idx: np.ndarray) -> int:
        lo, hi = _box(points[idx])
        me = len(nodes)
        nodes.append(Node(lo, hi, idx))
        if len(idx) > leaf and (hi[0] > lo[0] or hi[1] > lo[1]):
            cx = 0.5 * (lo[0] + hi[0])
            cy = 0.5 * (lo[1] + hi[1])
            p = points[idx]
            quad = (p.real >= cx).astype(int) + 2 * (p.imag >= cy).astype(int)
            kids = []
            for q in range(4):
                sub = idx[quad == q]
                if len(sub):
                    kids.append(make(sub))
            nodes[me].children = kids
        return me

    make(np.arange(points.shape[0]))
    return nodes


def size(nd: Node) -> float:
    return max(nd.hi[0] - nd.lo[0], nd.hi[1] - nd.lo[1])


def dmin2(a: Node, b: Node) -> float:
    dx = max(0.0, b.lo[0] - a.hi[0], a.lo[0] - b.hi[0])
    dy = max(0.0, b.lo[1] - a.hi[1], a.lo[1] - b.hi[1])
    return dx * dx + dy * dy


def dmax2(a: Node, b: Node) -> float:
    dx = max(a.hi[0] - b.lo[0], b.hi[0] - a.lo[0])
    dy = max(a.hi[1] - b.lo[1], b.hi[1] - a.lo[1])
    return dx * dx + dy * dy


def leaves_under(nodes: List[Node], t: int) -> List[int]:
    """Leaves of the subtree at t, depth first in child order."""
    if nodes[t].leaf:
        return [t]
    out = []
    for c in nodes[t].children:
        out += leaves_under(nodes, c)
    return out


@dataclass
class Plan:
    tgt: List[Node]
    src: List[Node]
    tgt_leaves: List[int]
    A: dict                          # target leaf -> [(source node, alpha)]
    E: dict                          # target leaf -> [source leaf]
    nu: float


def interaction_lists(x, y, nu: float, leaf: int) -> Plan:
    """Alg. C.1: quadtrees on x (targets) and y (sources) and the lists."""
    tgt = build_quadtree(x, leaf)
    src = build_quadtree(y, leaf)
    tl = leaves_under(tgt, 0)
    A = {l: [] for l in tl}
    E = {l: [] for l in tl}
    stack = [(0, 0)]
    while stack:
        s, t = stack.pop()
        S, T = src[s], tgt[t]
        if dmax2(S, T) <= nu * dmin2(S, T):
            for l in leaves_under(tgt, t):
                A[l].append((s, 1.0 / dmin2(S, tgt[l])))
            continue
        if S.leaf and T.leaf:
            E[t].append(s)
            continue
        if not T.leaf and (S.leaf or size(T) >= size(S)):
            for c in T.children:
                stack.append((s, c))
        else:
            for c in S.children:
                stack.append((c, t))
    return Plan(tgt, src, tl, A, E, nu)


def gram_matrices(src: List[Node], B: np.ndarray) -> List[np.ndarray]:
    """H_s = sum_{j in s} B_:,j B_:,j^* for every source node, bottom-up:
    a leaf sums its points, an inner node its children."""
    B = np.asarray(B, dtype=np.complex128)
    p = B.shape[0]
    H: List[np.ndarray] = [None] * len(src)

    def up(s: int):
        nd = src[s]
        if nd.leaf:
            acc = np.zeros((p, p), dtype=np.complex128)
            for j in nd.idx:
                b = B[:, j]
                acc += np.outer(b, np.conj(b))
            H[s] = acc
        else:
            acc = np.zeros((p, p), dtype=np.complex128)
            for c in nd.children:
                up(c)
                acc += H[c]
            H[s] = acc

    up(0)
    return H


def row_norm_bounds(plan: Plan, x, y, G, B) -> np.ndarray:
    """Alg. C.2: u with ||S_i,:||^2 <= u_i <= nu ||S_i,:||^2 for the
    Cauchy-like matrix with generators G, B on the nodes x, y."""
    x = np.asarray(x, dtype=np.complex128)
    y = np.asarray(y, dtype=np.complex128)
    G = np.asarray(G, dtype=np.complex128)
    B = np.asarray(B, dtype=np.complex128)
    H = gram_matrices(plan.src, B)
    u = np.zeros(x.shape[0])
    for l in plan.tgt_leaves:
        rows = plan.tgt[l].idx
        g = G[rows]                                   # |l| x p
        for s, alpha in plan.A[l]:
            q = np.real(np.einsum("ia,ab,ib->i", g, H[s], np.conj(g)))
            u[rows] += alpha * q
        for s in plan.E[l]:
            cols = plan.src[s].idx
            num = np.abs(g @ B[:, cols]) ** 2
            den = np.abs(x[rows, None] - y[None, cols]) ** 2
            u[rows] += np.sum(num / den, axis=1)
    return u
