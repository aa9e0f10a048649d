// Host side of the certified row-norm bounds for the Cauchy-like form
// (App. C): the quadtrees on the target points x and the source points y and
// the interaction lists of every target leaf (Alg. C.1), flattened into the
// arrays the bound kernels read (cauchy_bounds.hip).
//
// Tree: a node's box is the tight bounding box of its points (real and
// imaginary parts as the axes). A node with more than `leaf` points and a
// box of positive extent splits at its box midpoint into the four quadrants
// (a point goes to the upper / right side when its coordinate is >= the
// midpoint); empty quadrants are dropped, children are kept in quadrant
// order and every child keeps its points' relative order, so the points of
// every node are one contiguous range of the tree order.
//
// Traversal: a stack of (source node, target node) pairs from the two roots.
// A pair with d_max^2 <= nu d_min^2 (over the two boxes) is aggregated: every
// target leaf under the target node gets (s, 1 / d_min^2(s, leaf)). A pair of
// leaves that is not admissible is handled pair by pair (the source leaf
// joins the target leaf's exact list). Otherwise the target node is split
// when it is not a leaf and the source node is a leaf or no larger (longer
// box side), else the source node; children are pushed in quadrant order and
// the last pushed pair is taken next.
#include <algorithm>
#include <cmath>
#include <vector>

#include "bounds_plan.hpp"

namespace rplu {
namespace {

struct QTree {
    std::vector<QNode> nodes;
    std::vector<int32_t> perm;       // tree order -> point index
};

void box_of(const CPoint* pts, const int32_t* idx, int cnt, double lo[2], double hi[2]) {
    lo[0] = hi[0] = pts[idx[0]].re;
    lo[1] = hi[1] = pts[idx[0]].im;
    for (int q = 1; q < cnt; ++q) {
        const CPoint p = pts[idx[q]];
        lo[0] = std::min(lo[0], p.re);
        hi[0] = std::max(hi[0], p.re);
        lo[1] = std::min(lo[1], p.im);
        hi[1] = std::max(hi[1], p.im);
    }
}

// Builds the subtree of perm[beg, end) (iteratively: an explicit stack of
// nodes still to split, in the order a recursive build would create them).
void build(const CPoint* pts, int npts, int leaf, QTree* T) {
    T->perm.resize(npts);
    for (int q = 0; q < npts; ++q) T->perm[q] = q;
    T->nodes.clear();
    auto make = [&](int beg, int end, int depth) {
        QNode nd;
        nd.beg = beg;
        nd.end = end;
        nd.depth = depth;
        nd.nchild = 0;
        for (int c = 0; c < 4; ++c) nd.child[c] = -1;
        box_of(pts, T->perm.data() + beg, end - beg, nd.lo, nd.hi);
        T->nodes.push_back(nd);
        return (int)T->nodes.size() - 1;
    };
    // Preorder creation: a node's children are created (and their subtrees
    // completed, child 0 first) right after it, as a recursive build does.
    std::vector<int32_t> scratch(npts);
    struct Frame { int node; int next_child; int cb[5]; };
    std::vector<Frame> st;
    auto open = [&](int node) {
        QNode& nd = T->nodes[node];
        Frame f;
        f.node = node;
        f.next_child = 0;
        const int cnt = nd.end - nd.beg;
        if (cnt > leaf && (nd.hi[0] > nd.lo[0] || nd.hi[1] > nd.lo[1])) {
            const double cx = 0.5 * (nd.lo[0] + nd.hi[0]);
            const double cy = 0.5 * (nd.lo[1] + nd.hi[1]);
            int count[4] = {0, 0, 0, 0};
            auto quad = [&](int32_t id) {
                const CPoint p = pts[id];
                return (p.re >= cx ? 1 : 0) + (p.im >= cy ? 2 : 0);
            };
            for (int q = nd.beg; q < nd.end; ++q) ++count[quad(T->perm[q])];
            int off[4];
            off[0] = nd.beg;
            for (int c = 1; c < 4; ++c) off[c] = off[c - 1] + count[c - 1];
            for (int c = 0; c < 4; ++c) f.cb[c] = off[c];
            f.cb[4] = nd.end;
            int w[4] = {off[0], off[1], off[2], off[3]};
            for (int q = nd.beg; q < nd.end; ++q) {
                const int32_t id = T->perm[q];
                scratch[w[quad(id)]++] = id;                 // stable within each quadrant
            }
            for (int q = nd.beg; q < nd.end; ++q) T->perm[q] = scratch[q];
        } else {
            f.cb[0] = f.cb[1] = f.cb[2] = f.cb[3] = f.cb[4] = nd.end;
            f.next_child = 4;
        }
        st.push_back(f);
    };
    open(make(0, npts, 0));
    while (!st.empty()) {
        Frame& f = st.back();
        while (f.next_child < 4 && f.cb[f.next_child] == f.cb[f.next_child + 1]) ++f.next_child;
        if (f.next_child >= 4) {
            st.pop_back();
            continue;
        }
        const int c = f.next_child++;
        const int parent = f.node;
        const int child = make(f.cb[c], f.cb[c + 1], T->nodes[parent].depth + 1);
        QNode& pn = T->nodes[parent];
        pn.child[pn.nchild++] = child;
        open(child);                                          // may reallocate st
    }
}

double node_size(const QNode& a) { return std::max(a.hi[0] - a.lo[0], a.hi[1] - a.lo[1]); }

double dmin2(const QNode& a, const QNode& b) {
    const double dx = std::max(0.0, std::max(b.lo[0] - a.hi[0], a.lo[0] - b.hi[0]));
    const double dy = std::max(0.0, std::max(b.lo[1] - a.hi[1], a.lo[1] - b.hi[1]));
    return dx * dx + dy * dy;
}

double dmax2(const QNode& a, const QNode& b) {
    const double dx = std::max(a.hi[0] - b.lo[0], b.hi[0] - a.lo[0]);
    const double dy = std::max(a.hi[1] - b.lo[1], b.hi[1] - a.lo[1]);
    return dx * dx + dy * dy;
}

void leaves_under(const QTree& T, int t, std::vector<int>* out) {
    std::vector<int> st{t};
    while (!st.empty()) {                 // depth first, children in order
        const int v = st.back();
        st.pop_back();
        const QNode& nd = T.nodes[v];
        if (nd.nchild == 0) {
            out->push_back(v);
            continue;
        }
        for (int c = nd.nchild - 1; c >= 0; --c) st.push_back(nd.child[c]);
    }
}

}  // namespace

void build_bounds_plan(const CPoint* x, int64_t n, const CPoint* y, int64_t m, double nu, int leaf,
                       HostBoundsPlan* P) {
    QTree tt, ss;
    build(x, (int)n, leaf, &tt);
    build(y, (int)m, leaf, &ss);
    P->nu = nu;
    P->tgt_perm = tt.perm;
    P->src_perm = ss.perm;
    P->src = ss.nodes;

    std::vector<int> tleaves;
    leaves_under(tt, 0, &tleaves);
    std::vector<int> leaf_slot(tt.nodes.size(), -1);
    for (size_t q = 0; q < tleaves.size(); ++q) leaf_slot[tleaves[q]] = (int)q;
    std::vector<std::vector<std::pair<int, double>>> A(tleaves.size());
    std::vector<std::vector<int>> E(tleaves.size());

    std::vector<std::pair<int, int>> stack{{0, 0}};
    std::vector<int> under;
    while (!stack.empty()) {
        const auto [s, t] = stack.back();
        stack.pop_back();
        const QNode& S = ss.nodes[s];
        const QNode& T = tt.nodes[t];
        if (dmax2(S, T) <= nu * dmin2(S, T)) {
            under.clear();
            leaves_under(tt, t, &under);
            for (int l : under) A[leaf_slot[l]].push_back({s, 1.0 / dmin2(S, tt.nodes[l])});
            continue;
        }
        const bool sl = S.nchild == 0, tl = T.nchild == 0;
        if (sl && tl) {
            E[leaf_slot[t]].push_back(s);
            continue;
        }
        if (!tl && (sl || node_size(T) >= node_size(S))) {
            for (int c = 0; c < T.nchild; ++c) stack.push_back({s, T.child[c]});
        } else {
            for (int c = 0; c < S.nchild; ++c) stack.push_back({S.child[c], t});
        }
    }

    P->tl_beg.clear();
    P->tl_end.clear();
    P->A_off.assign(1, 0);
    P->E_off.assign(1, 0);
    P->A_node.clear();
    P->A_alpha.clear();
    P->E_node.clear();
    for (size_t q = 0; q < tleaves.size(); ++q) {
        P->tl_beg.push_back(tt.nodes[tleaves[q]].beg);
        P->tl_end.push_back(tt.nodes[tleaves[q]].end);
        for (const auto& e : A[q]) {
            P->A_node.push_back(e.first);
            P->A_alpha.push_back(e.second);
        }
        for (int s : E[q]) P->E_node.push_back(s);
        P->A_off.push_back((int32_t)P->A_node.size());
        P->E_off.push_back((int32_t)P->E_node.size());
    }
    // source leaves, and the inner source nodes grouped by depth (deepest
    // last) for the bottom-up Gram pass
    P->src_leaves.clear();
    int maxd = 0;
    for (const QNode& nd : ss.nodes) maxd = std::max(maxd, nd.depth);
    std::vector<std::vector<int32_t>> bylevel(maxd + 1);
    for (size_t v = 0; v < ss.nodes.size(); ++v) {
        if (ss.nodes[v].nchild == 0) P->src_leaves.push_back((int32_t)v);
        else bylevel[ss.nodes[v].depth].push_back((int32_t)v);
    }
    P->inner.clear();
    P->level_off.assign(1, 0);
    for (int d = 0; d <= maxd; ++d) {
        for (int32_t v : bylevel[d]) P->inner.push_back(v);
        P->level_off.push_back((int32_t)P->inner.size());
    }
    P->max_depth = maxd;
}

}  // namespace rplu
