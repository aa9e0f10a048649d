// Certified row-norm bounds for the Cauchy-like form (App. C): the host
// plan (quadtrees and interaction lists, Alg. C.1) and its device form.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace rplu {

// Complex points as interleaved (re, im) doubles.
struct CPoint {
    double re, im;
};

struct QNode {
    double lo[2], hi[2];   // tight box (re, im)
    int32_t beg, end;      // points [beg, end) of the tree order
    int32_t child[4];      // children in quadrant order (-1: none)
    int32_t nchild;
    int32_t depth;
};

struct HostBoundsPlan {
    double nu = 0.0;
    int max_depth = 0;
    std::vector<int32_t> tgt_perm, src_perm;   // tree order -> point index
    std::vector<QNode> src;                    // source nodes (node 0 = root)
    std::vector<int32_t> src_leaves;           // source leaf node ids
    std::vector<int32_t> inner;                // inner source nodes by depth
    std::vector<int32_t> level_off;            // inner[level_off[d] .. level_off[d+1])
    std::vector<int32_t> tl_beg, tl_end;       // target leaves: ranges of the tree order
    std::vector<int32_t> A_off, A_node;        // aggregated entries per target leaf
    std::vector<double> A_alpha;
    std::vector<int32_t> E_off, E_node;        // exact source leaves per target leaf
};

void build_bounds_plan(const CPoint* x, int64_t n, const CPoint* y, int64_t m, double nu,
                       int leaf, HostBoundsPlan* P);

// The plan in device memory (one allocation carved by the caller) plus the
// per-run buffers of the bound kernels.
struct BoundsPlan {
    int n_src_nodes, n_src_leaves, n_tgt_leaves, max_depth;
    int n_inner;                 // inner source nodes (the length of `inner`)
    int pad;
    double nu;
    const int32_t* src_perm;     // m
    const int32_t* tgt_perm;     // n
    const int32_t* node_beg;     // per source node
    const int32_t* node_end;
    const int32_t* node_child;   // 4 per source node
    const int32_t* src_leaves;
    const int32_t* inner;
    const int32_t* level_off;    // max_depth + 2 entries
    const int32_t* tl_beg;
    const int32_t* tl_end;
    const int32_t* A_off;
    const int32_t* A_node;
    const double* A_alpha;
    const int32_t* E_off;
    const int32_t* E_node;
    void* H;                     // n_src_nodes p x p complex FP64 Gram matrices
    double* u;                   // n: the bounds (the row masses of the draws)
    double* rej_part;            // BH_REJ_CAND x BH_REJ_MAX_SPLIT partial row masses
    double* rej_cand;            // BH_REJ_CAND x {i, target, lo, hi} of the trials
};

// The rejection draw evaluates the first BH_REJ_CAND trials at once, each
// row's mass split over up to BH_REJ_MAX_SPLIT workgroups.
constexpr int BH_REJ_CAND = 4;
constexpr int BH_REJ_MAX_SPLIT = 16;

// Bytes of the device plan (256-byte aligned pieces) for a host plan.
size_t bounds_plan_bytes(const HostBoundsPlan& P, int64_t n, int p);



}  // namespace rplu
