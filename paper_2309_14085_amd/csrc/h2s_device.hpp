// h2s_device.hpp -- device-side view of an uploaded H2* / (H2+H)* matrix and
// the launcher of the MVP kernels (h2s_kernels.hip).
//
// Layout in HBM (tree order throughout; boxes numbered globally, level by
// level, Morton order inside a level):
//   points      SoA px, py, pz.  FP64: absolute coordinates.  FP32: offsets
//               from the centre of the point's leaf (centres box_ctr, double).
//   charges     qt (double, tree order).
//   per family  multipoles v and locals u (double), one slot of rank entries
//               per box at coef_off[box];
//               pivot coordinates t^{X,i} aligned with the coefficients
//               (far family in FP32 mode: offsets from the box centre);
//               leaf bases U_X twice: row-major n_X x r (P2M, sums over rows)
//               and column-major (L2P, one point per thread), at uoff[leaf];
//               stacked transfers U~ (double) twice: row-major (sum r_c) x r
//               (M2M) and column-major (L2L), at troff[box];
//               interaction list CSR il_off / il_idx; M2L work list targets.
//   (H2+H)*     per vertex-sharing pair column-major factors Ub (n_X x r) and
//               Vb (n_Y x r); per-pair products w = Vb^T q_Y, w' = Ub^T q_X.
//
// Precision policies.  P64: everything in double, and the sums whose
// results the interpolative operators amplify are taken in index order with
// separately rounded products and sums.  P32: near field and leaf bases in
// float (box-centred coordinates), M2L, transfers, coefficients and all
// accumulations in double.  P32M: as P32 and the far-field M2L in float as
// well (for log r split into a per-pair constant in double and a float
// remainder).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace h2s {

struct P64 {
    using basis_t = double;
    using pt_t = double;
    using far_t = double;
    static constexpr bool local = false;
    static constexpr bool ordered = true;
};

struct P32 {
    using basis_t = float;
    using pt_t = float;
    using far_t = double;
    static constexpr bool local = true;
    static constexpr bool ordered = false;
};

struct P32M {
    using basis_t = float;
    using pt_t = float;
    using far_t = float;
    static constexpr bool local = true;
    static constexpr bool ordered = false;
};

template <typename CT, typename BT> struct DevFamily {
    int32_t lmin;
    const int32_t *coef_off;     // nbox + 1
    const CT *pvx, *pvy, *pvz;   // pivot coordinates per coefficient
    const CT *pvw;               // NTI multiquadric: c(x) of each pivot (absolute)
    const BT *U_rm, *U_cm;       // leaf bases: the rows that are not unit rows, in order
    const int64_t *uoff;         // per leaf (local index)
    const uint16_t *ukeep;       // per point slot b + j: local row of the leaf's kept row j
    const int16_t *urow;         // per point: kept index of its row, or ~a for the unit row e_a
    const int16_t *uprow;        // per coefficient: local row of its unit row, or -1
    const int16_t *upos;         // per coefficient with a unit row: kept rows before that row
    const int32_t *unk;          // per leaf: kept rows
    const double *Tr_rm, *Tr_cm; // stacked transfers: the rows that are not unit rows, in order
    const int64_t *troff;        // per global box
    const int32_t *tnk;          // per box: kept rows of its transfer
    const uint16_t *tkeep;       // per child coefficient slot bf + j: stacked row of kept row j
    const int16_t *trow;         // per child coefficient: kept index of its row, or ~a for e_a
    const int16_t *tprow;        // per coefficient: stacked row of its unit row, or -1
    const int16_t *tpos;         // per coefficient with a unit row: kept rows before that row
    const int32_t *il_off;       // nbox + 1
    const int32_t *il_idx;
    const int32_t *targets;      // boxes with rank > 0 at levels >= lmin, in box (so level) order
    int32_t ntargets;
    int32_t targets_leaf;        // index in targets of the first leaf-level box
    int32_t ncoef;               // coefficients of the family (all boxes)
    double *v, *u;
    double *vb, *ub;             // multi-RHS: kGroupBlocks blocks of ncoef x kBatch (allocated on first use)
};

// (H2+H)* vertex-sharing low-rank blocks.
template <typename BT> struct DevPairs {
    int32_t npairs;
    const int32_t *px, *py, *prank; // per pair: boxes (global) and rank
    const int64_t *pu, *pv;         // offsets of Ub and Vb
    const int64_t *pw;              // offset of the pair's w (2 rank entries: Vb^T q_Y, then Ub^T q_X)
    const BT *data;
    double *w;
    const int32_t *recv_off; // nbox + 1: (pair, side) entries each box receives
    const int32_t *recv;     // 2 * pair + side; side 0: X += Ub w, side 1: Y += Vb w'
    int32_t nchunks;
    const int32_t *chunk_pair, *chunk_side, *chunk_begin, *chunk_len;
    const int64_t *chunk_poff;     // offset of the chunk's partial sums
    const int32_t *side_chunk_off; // 2 * npairs + 1
    double *partial;
};

template <class P> struct DevTree {
    using pt_t = typename P::pt_t;
    using basis_t = typename P::basis_t;
    int32_t n, d, kappa, nleaf, leaf0, nbox, kind, variant;
    int32_t max_leaf, max_rows, max_rank; // LDS sizing: largest leaf, stacked transfer rows, rank
    double diag, shift, kparam; // K(x,x); shift * I; -1/h^2 for the Gaussian (exponent r^2 kparam)
    double kc[3];               // piecewise RBFs of radius a: a^2, then a, 1/a (a/r | r/a) or
                                // 1/log a, 1/(a log a - 1) (log r | r log r - 1)
    const int32_t *perm;        // tree position -> user index
    const pt_t *px, *py, *pz;
    const pt_t *pw;             // NTI multiquadric: c(x) = exp(-(x_1 + x_3)) per point (absolute)
    const int32_t *box_begin, *box_end, *box_cbeg, *box_cend;
    const double *box_ctr;      // 3 per box
    const int32_t *leaf_anc;    // (kappa + 1) per leaf: ancestor at each level
    const int32_t *near_off, *near_idx; // leaf-local CSR (sorted: leaves below, the leaf, leaves above)
    const int32_t *near_self;   // per leaf: its own entry in the near list
    const int64_t *near_w;      // per near entry: offset in near_wv of the pair's column sums (upper: written
                                // by this leaf's block; lower: read by this leaf's L2P)
    double *near_wv;            // column sums of the symmetric near field: n_X' entries per pair X < X'
    DevFamily<typename P::far_t, basis_t> far;
    DevFamily<double, basis_t> ver;
    DevPairs<basis_t> pairs;
    double *qt;           // charges in tree order
    double *yn;           // near-field potentials in tree order
    double *qb, *ynb;     // multi-RHS blocks of both: kBatch entries per point (allocated on first use)
    const double *ktab;   // kernel-function table: log r and RBF_LOG (c_i, -0.5 ln c_i) x 256;
                          // exponentials 2^(j/64) x 64
};

// Host-side launch shapes, fixed at upload.
constexpr int kMaxLevels = 32;
constexpr int kMaxList = 256; // boxes of an interaction list (6^d at most in a 2^d tree); checked at build
struct LaunchPlan {
    const int32_t *lev_off;              // global box range of every level (kappa + 2 entries)
    int32_t up_threads[kMaxLevels + 1];  // block size of P2M (level kappa) and M2M (levels < kappa)
    int32_t dn_threads[kMaxLevels + 1];  // block size of L2L per level
    double near_first;                   // share of the leaves whose near field runs beside P2M and M2M
    int32_t m2l_stream;                  // 1: leaf-level M2L on a third stream right after P2M; 2: also the
                                         // M2L of level kappa - 1 on a fourth stream right after its M2M
    const int32_t *tlev[2];              // per family: index in its targets of the first box of every
                                         // level (kappa + 2 entries)
};

constexpr double kNearFirstDefault = 0.8;

// Optional timing hook: mark(ctx, kernel class, 0 = before / 1 = after, stream).
struct ProfileHook {
    void *ctx;
    void (*mark)(void *ctx, int cls, int end, void *stream);
};

// The caller's stream, the handle's second stream (near field) and the
// events that fork the second stream from the first (twice per product) and
// join it back.
// The caller's stream, the near-field stream (forked at fork / fork2, joined
// at join) and the leaf-level M2L stream (forked at fork3, joined at join2).
struct Streams {
    void *main, *aux, *fork, *fork2, *join, *aux2, *fork3, *join2;
    void *aux3, *fork4, *join3; // fourth stream (M2L of the level above the leaves), fork / join events
};

// Many trees of one precision, kernel function and dimension (H2*) applied
// with one launch per step: every array lives in device memory and maps a
// block (after the XCD remap) to (tree, work item).  Steps: the charge
// permutation (items: 256-point chunks), the near field and L2P (items:
// leaves), P2M (leaves of trees with kappa >= 1), M2M step s (boxes of level
// kappa_i - 1 - s of tree i), M2L per family (target-list indices), L2L step s
// (boxes of level 1 + s).
template <class P> struct MultiPlan {
    const DevTree<P> *trees;
    const double *const *xs; // per tree
    double *const *ys;
    const int2 *perm_map, *leaf_map, *up_map, *far_map, *ver_map;
    int32_t n_perm, n_leaf, n_up, n_far, n_ver;
    int32_t steps;                                 // M2M and L2L steps (max kappa - 1)
    const int2 *m2m_map[kMaxLevels], *l2l_map[kMaxLevels];
    int32_t n_m2m[kMaxLevels], n_l2l[kMaxLevels];
    int32_t w_up, w_m2m[kMaxLevels], w_l2l[kMaxLevels]; // block widths (largest of the trees')
    size_t lds_leaf, lds_rows, lds_rank;           // dynamic LDS (largest of the trees')
};

template <class P> int launch_multi(int kind, int d, const MultiPlan<P> &mp, const Streams &s);

// Right-hand sides per block of the batched product, and blocks taken
// through one launch sequence (their M2L shares each kernel evaluation).
constexpr int kBatch = 8;
constexpr int kGroupBlocks = 4;
constexpr int kGroupCols = kBatch * kGroupBlocks;

// Enqueue the product for ncols <= kGroupCols right-hand sides at once (x, y
// column-major with leading dimensions ldx, ldy), ordered on st.main, as
// ceil(ncols / kBatch) blocks of kBatch columns.  H2* only; the block buffers
// must be allocated.  With a float far field (P32M) the far M2L runs on the
// matrix cores in float, or with bfloat16 inputs when bf16_m2l is set.
template <class P>
int launch_mvp_batch(const DevTree<P> &t, const LaunchPlan &plan, const double *x, int64_t ldx, double *y,
                     int64_t ldy, int ncols, uint32_t mask, const Streams &st, bool bf16_m2l = false);

// Device address of the file-scope batch scratch array on `device` (current), for
// h2s_apply_noalloc; H2S_NOALLOC_SCRATCH_BYTES long.
hipError_t noalloc_scratch(int device, double **ptr);

// Enqueue one product y = K~ x (single right-hand side), ordered on st.main.
// Returns a hipError_t as int.
template <class P>
int launch_mvp(const DevTree<P> &t, const LaunchPlan &plan, const double *x, double *y, uint32_t mask,
               const Streams &st, const ProfileHook *prof);

} // namespace h2s
