// h2s_device.hpp -- device-side view of an uploaded H2* / (H2+H)* matrix and
// the launchers of the MVP kernels (h2s_kernels.hip).
//
// Layout in HBM (tree order throughout; boxes numbered globally, level by
// level, Morton order inside a level):
//   points      SoA px, py, pz.  FP64: absolute coordinates.  FP32: offsets
//               from the centre of the point's leaf box (leaf_cx/cy/cz).
//   per family  coefficients v (multipoles) and u (locals), one contiguous
//               slot of rank entries per box at coef_off[box];
//               pivot coordinates t^{X,i} aligned with the coefficients
//               (FP32: offsets from the box centre);
//               leaf L2P/P2M bases U_X column-major n_X x r at uoff[leaf];
//               stacked L2L/M2M operators row-major (sum r_c) x r at troff[box];
//               interaction list CSR il_off / il_idx over global boxes.
//   (H2+H)*     per vertex-sharing pair column-major factors Ub (n_X x r) and
//               Vb (n_Y x r); per-pair products w = Vb^T q_Y, w' = Ub^T q_X.
#pragma once

#include <cstdint>

namespace h2s {

template <typename T> struct DevFamily {
    int lmin;
    const int32_t *coef_off;  // nbox + 1
    const T *pvx, *pvy, *pvz; // pivot coordinates per coefficient
    const T *U;               // leaf bases
    const int64_t *uoff;      // per leaf (local index)
    const T *Tr;              // stacked transfer operators
    const int64_t *troff;     // per global box
    const int32_t *il_off;    // nbox + 1
    const int32_t *il_idx;
    const int32_t *targets;   // boxes with rank > 0 at levels >= lmin (M2L work list)
    int32_t ntargets;
    T *v, *u;                 // multipole / local coefficients
};

// (H2+H)* vertex-sharing low-rank blocks.
template <typename T> struct DevPairs {
    int32_t npairs;
    const int32_t *px, *py, *prank; // per pair: boxes (global) and rank
    const int64_t *pu, *pv;         // offsets of Ub and Vb
    const int64_t *pw;              // offset of the pair's w (2 * rank entries: Vb^T q_Y then Ub^T q_X)
    const T *data;
    T *w;
    // row side: for every box, the (pair, side) entries it receives; side 0:
    // X receives Ub w, side 1: Y receives Vb w'
    const int32_t *recv_off; // nbox + 1
    const int32_t *recv;     // 2 * pair + side
    // partial products of the coarse (split) pairs
    int32_t nchunks;
    const int32_t *chunk_pair, *chunk_side, *chunk_begin, *chunk_len; // one entry per chunk
    const int64_t *chunk_poff;                                         // offset of the chunk's rank partial sums
    const int32_t *side_chunk_off;                                     // 2 * npairs + 1: chunks of (pair, side)
    T *partial;
};

template <typename T> struct DevTree {
    int32_t n, d, kappa, nleaf, leaf0, nbox, kind;
    double diag, shift, kparam;   // K(x,x); shift * I; kernel parameter (1 / h^2 for Gaussian)
    const int32_t *perm;          // tree position -> user index
    const T *px, *py, *pz;        // tree-order coordinates
    const int32_t *box_begin, *box_end, *box_cbeg, *box_cend;
    const double *box_ctr;        // 3 per box: centre (FP32 differences of centres)
    const int32_t *leaf_anc;      // (kappa + 1) per leaf: global id of its ancestor at each level
    const int32_t *near_off, *near_idx; // leaf-local CSR
    DevFamily<T> fam[2];
    DevPairs<T> pairs;
    int32_t variant;
    T *qt;                        // charges in tree order
    T *phi;                       // potential in tree order (vertex part of (H2+H)*)
};

// Optional timing hook: mark(ctx, kernel class, 0 = before / 1 = after).
struct ProfileHook {
    void *ctx;
    void (*mark)(void *ctx, int cls, int end);
};

// Launchers; each enqueues on `stream` and returns a hipError_t as int.
// One product y = K~ x for a single right-hand side.  lev_off: host copy of
// the global box range of every level (kappa + 2 entries).
template <typename T>
int launch_mvp(const DevTree<T> &t, const int32_t *lev_off, const double *x, double *y, uint32_t mask,
               void *stream, const ProfileHook *prof);

} // namespace h2s
