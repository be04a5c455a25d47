// h2s_host.hpp -- host-side representation of an H2* / (H2+H)* matrix.
//
// Built on the host by build_host() (h2s_host_build.cpp) and uploaded to the
// device by the C ABI (h2s_api.cpp).  Boxes use one global numbering: level
// by level from the root, Morton order inside a level, so the children of a
// box are a contiguous range of the next level and the leaves come last.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "h2s.h"

namespace h2s {

struct KernelSpec {
    int kind;
    double param, diag, shift;
};

// One basis family: far field (B2T NCA) or vertex sharing (T2B NCA).
struct Family {
    int lmin = 0;                  // coarsest level with a basis (2 far, 1 vertex)
    std::vector<int32_t> rank;     // per global box
    std::vector<int64_t> coef_off; // per global box + 1: prefix sum of ranks
    std::vector<int32_t> piv_row;  // t^{X,i}, tree positions, aligned with coef_off
    std::vector<int32_t> piv_col;  // s^{X,i}, tree positions, aligned with coef_off
    std::vector<int64_t> op_off;   // per global box + 1: offset into op
    std::vector<int32_t> op_rows;  // per global box: rows of its operator
    std::vector<double> op;        // leaf: U_X column-major n_X x r; non-leaf: stacked L2L, row-major (sum r_c) x r
};

// (H2+H)* vertex-sharing pair: K(t^X, t^Y) ~ Ub Vb^T, column-major factors.
struct LowRankPair {
    int32_t level, x, y, rank; // x < y, global box ids
    int64_t off_u, off_v;      // into LowRank data
};

struct HostRep {
    int d = 0, kappa = 0;
    int64_t n = 0;
    KernelSpec ker{};
    int variant = 0;
    double eps_far = 0, eps_ver = 0;
    double ctr[3] = {0, 0, 0}, half = 1, origin[3] = {0, 0, 0};

    std::vector<int32_t> perm; // tree position -> user index
    std::vector<double> pts;   // tree order, row-major n x d

    std::vector<int32_t> lev_off; // kappa + 2 entries: global id range of each level
    std::vector<int32_t> box_begin, box_end, box_parent, box_cbeg, box_cend;
    std::vector<int32_t> box_coord; // 3 per box
    std::vector<int64_t> box_morton;

    // CSR lists over global boxes; entries are global box ids in Morton order.
    // 0 = near field N* (leaf level only, includes the box), 1 = IL_far, 2 = IL_ver.
    std::vector<int64_t> list_off[3];
    std::vector<int32_t> list_idx[3];

    Family fam[2];
    std::vector<LowRankPair> pairs;
    std::vector<double> pair_data;

    double build_seconds = 0;

    int32_t nbox() const { return lev_off.empty() ? 0 : lev_off.back(); }
    int32_t leaf0() const { return lev_off[kappa]; }
    int32_t nleaf() const { return lev_off[kappa + 1] - lev_off[kappa]; }
    int level_of(int32_t g) const;
};

// Host kernel entry K(x, y) in double (same formulas as the device code).
double kernel_entry(const KernelSpec &k, int d, const double *x, const double *y);

// Steps of Sec. 3.1, 3.3, 5.1.1 / 5.2.1 and 3.4.3.  Returns H2S_OK or an error
// with a message.  `threads` <= 0 leaves the OpenMP default.
h2s_status build_host(const double *points, int64_t n, int d, const KernelSpec &k, int32_t leaf_size,
                      double eps_far, double eps_ver, int variant, int threads, HostRep &rep, std::string &err);

// Write the named-array container described in the design notes.
h2s_status export_host(const HostRep &rep, const char *path, std::string &err);

} // namespace h2s
