// h2s_host_build.cpp -- host construction of the H2* / (H2+H)* representation.
//
// Steps, in the paper's order (Khan & Ambikasaran, arXiv 2309.14085):
//   tree          uniform 2^d tree, kappa = ceil(log_{2^d}(N / n_max))     Sec. 3.1
//   lists         near field N*, IL_far, IL_ver of every box               Sec. 3.3, Table "HOD_notation", Sec. 5.1
//   far pivots    B2T NCA on IL_far, levels kappa .. 2                     Sec. 5.1.1 (1), Alg. "b2t"
//   vertex pivots T2B NCA on IL_ver, levels 1 .. kappa                     Sec. 5.1.1 (2), Alg. "t2b"
//                 or, for (H2+H)*, ACA of every vertex-sharing pair        Sec. 5.2.1, Alg. "pure_aca"
//   operators     L2P U_X, L2L U~_{X_c X} (P2M / M2M are transposes)       Sec. 3.4.3
//
// Where the paper leaves a point open (bounding cube, point order, ACA start
// row, tie-breaks, zero pivots, stopping test, outgoing pivots, duplicate
// columns, LU solves) the interpretation is stated where it is used.
// Integer decisions that floating point takes (leaf coordinates, ACA pivots)
// use a fixed operation order in double so that they are reproducible.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <omp.h>

#include "h2s_host.hpp"

namespace h2s {

double kernel_entry(const KernelSpec &k, int d, const double *x, const double *y)
{
    double r2 = 0.0;
    for (int c = 0; c < d; ++c) {
        const double t = x[c] - y[c];
        r2 += t * t;
    }
    if (r2 == 0.0) return k.diag;
    switch (k.kind) {
    case H2S_K_LOG_R: return 0.5 * std::log(r2); // log r, without rounding r itself
    case H2S_K_INV_R: return 1.0 / std::sqrt(r2);
    case H2S_K_GAUSSIAN: return std::exp(-r2 / (k.param * k.param));
    case H2S_K_RBF_AR: {
        const double r = std::sqrt(r2), a = k.param;
        return r >= a ? a / r : r / a;
    }
    case H2S_K_RBF_LOG: {
        const double r = std::sqrt(r2), a = k.param, lr = 0.5 * std::log(r2);
        return r >= a ? lr / std::log(a) : (r * lr - 1.0) / (a * std::log(a) - 1.0);
    }
    case H2S_K_NTI_MQ: { // d == 3 (checked at build)
        const double dc = std::exp(-(x[0] + x[2])) - std::exp(-(y[0] + y[2]));
        const double t = r2 + dc * dc + 1.0;
        return t * std::sqrt(t);
    }
    default: return std::exp(-std::sqrt(r2));
    }
}

int HostRep::level_of(int32_t g) const
{
    int l = 0;
    while (l + 1 < (int)lev_off.size() && lev_off[l + 1] <= g) ++l;
    return l;
}

namespace {

// ---------------------------------------------------------------------------
// Partially pivoted adaptive cross approximation (Sec. 3.4).
// ---------------------------------------------------------------------------
struct Cross {
    int64_t nI = 0, nJ = 0;
    int rank = 0;
    std::vector<double> U, V;        // k-major: U[k*nI + i], V[k*nJ + j]
    std::vector<int32_t> prow, pcol; // positions in I and J
};

// The iteration ends when ||u_p|| ||v_p|| <= eps ||S||_F (the condition of
// Sec. 3.4) has held for kAcaRun successive terms, all of them kept.  Partial
// pivoting sees only the rows and columns it visits, so a single small term
// can end it while the residual elsewhere is still large (vertex-sharing
// blocks keep theirs on the close pairs near the shared corner); six
// successive terms give the relative errors of the paper's 2D and 3D MVP
// tables (smvp2d_lap_*, smvp3d_lap_*).  With drop_confirm the five terms after
// the first of the run only confirm the stop and are dropped (the T2B vertex
// bases: kept, they are the smallest pivots of near-singular pivot blocks).
constexpr int kAcaRun = 6;

// `entry(a, b)` is K(I[a], J[b]).  `par` lets the elementwise loops use the
// OpenMP team (used when few large approximations run one after another);
// every reduction stays sequential so the result does not depend on it.
template <class Entry>
void cross_approx(const Entry &entry, int64_t nI, int64_t nJ, double eps, bool par, bool drop_confirm, Cross &c)
{
    c.nI = nI;
    c.nJ = nJ;
    c.rank = 0;
    c.U.clear(); c.V.clear(); c.prow.clear(); c.pcol.clear();
    if (nI <= 0 || nJ <= 0) return;
    const int64_t maxr = std::min(nI, nJ);
    std::vector<char> rowused(nI, 0), colused(nJ, 0);
    std::vector<double> R(nJ);
    double s2 = 0.0;
    int64_t istar = 0;
    int run = 0;  // successive terms whose norm met the tolerance
    const bool parJ = par && nJ >= 16384, parI = par && nI >= 16384;
    // Residual entries are taken in chunks of kChunk: the chunk stays in cache while the earlier
    // terms' rows stream through it in order k = 0, 1, ..., so every entry sees the same
    // operations in the same order as an entry-by-entry loop.
    constexpr int64_t kChunk = 512;
    for (;;) {
        rowused[istar] = 1;
        const int p = c.rank;
#pragma omp parallel for if (parJ) schedule(static)
        for (int64_t j0 = 0; j0 < nJ; j0 += kChunk) {
            const int64_t j1 = std::min(j0 + kChunk, nJ);
            for (int64_t j = j0; j < j1; ++j) R[j] = entry(istar, j);
            for (int k = 0; k < p; ++k) {
                const double u = c.U[(size_t)k * nI + istar];
                const double *vk = c.V.data() + (size_t)k * nJ;
                for (int64_t j = j0; j < j1; ++j) R[j] -= u * vk[j];
            }
        }
        int64_t jstar = -1;
        double best = -1.0;
        for (int64_t j = 0; j < nJ; ++j)
            if (!colused[j] && std::fabs(R[j]) > best) {
                best = std::fabs(R[j]);
                jstar = j;
            }
        if (jstar < 0) break;
        if (R[jstar] == 0.0) {
            int64_t next = -1;
            for (int64_t i = 0; i < nI; ++i)
                if (!rowused[i]) { next = i; break; }
            if (next < 0) break;
            istar = next;
            continue;
        }
        c.U.resize((size_t)(p + 1) * nI);
        c.V.resize((size_t)(p + 1) * nJ);
        double *up = c.U.data() + (size_t)p * nI;
        double *vp = c.V.data() + (size_t)p * nJ;
        const double piv = R[jstar];
#pragma omp parallel for if (parJ) schedule(static)
        for (int64_t j = 0; j < nJ; ++j) vp[j] = R[j] / piv;
#pragma omp parallel for if (parI) schedule(static)
        for (int64_t i0 = 0; i0 < nI; i0 += kChunk) {
            const int64_t i1 = std::min(i0 + kChunk, nI);
            for (int64_t i = i0; i < i1; ++i) up[i] = entry(i, jstar);
            for (int k = 0; k < p; ++k) {
                const double v = c.V[(size_t)k * nJ + jstar];
                const double *uk = c.U.data() + (size_t)k * nI;
                for (int64_t i = i0; i < i1; ++i) up[i] -= uk[i] * v;
            }
        }
        colused[jstar] = 1;
        double nu2 = 0.0, nv2 = 0.0;
        for (int64_t i = 0; i < nI; ++i) nu2 += up[i] * up[i];
        for (int64_t j = 0; j < nJ; ++j) nv2 += vp[j] * vp[j];
        // (u_k . u_p)(v_k . v_p) for every earlier term; the dot products are
        // independent, so they may run in parallel, and are summed in order.
        std::vector<double> dots((size_t)p);
#pragma omp parallel for if (par && p > 1 && (nI + nJ) >= 16384) schedule(dynamic, 1)
        for (int k = 0; k < p; ++k) {
            const double *uk = c.U.data() + (size_t)k * nI, *vk = c.V.data() + (size_t)k * nJ;
            double a = 0.0, b = 0.0;
            for (int64_t i = 0; i < nI; ++i) a += uk[i] * up[i];
            for (int64_t j = 0; j < nJ; ++j) b += vk[j] * vp[j];
            dots[k] = a * b;
        }
        double cross = 0.0;
        for (int k = 0; k < p; ++k) cross += dots[k];
        s2 = s2 + (nu2 * nv2 + 2.0 * cross);
        c.prow.push_back((int32_t)istar);
        c.pcol.push_back((int32_t)jstar);
        c.rank = p + 1;
        run = std::sqrt(nu2 * nv2) <= eps * std::sqrt(s2) ? run + 1 : 0;
        if (run == kAcaRun) {
            if (drop_confirm) {
                c.rank -= kAcaRun - 1;
                c.prow.resize(c.rank);
                c.pcol.resize(c.rank);
                c.U.resize((size_t)c.rank * nI);
                c.V.resize((size_t)c.rank * nJ);
            }
            break;
        }
        if (c.rank == maxr) break;
        int64_t inext = -1;
        best = -1.0;
        for (int64_t i = 0; i < nI; ++i)
            if (!rowused[i] && std::fabs(up[i]) > best) {
                best = std::fabs(up[i]);
                inext = i;
            }
        if (inext < 0) break;
        istar = inext;
    }
}

// ---------------------------------------------------------------------------
// LU with partial pivoting and the row solve x A = b (operators, Sec. 3.4.3).
// ---------------------------------------------------------------------------
void lu_inplace(std::vector<double> &A, int r, std::vector<int> &piv)
{
    piv.resize(r);
    for (int k = 0; k < r; ++k) {
        int p = k;
        double best = std::fabs(A[(size_t)k * r + k]);
        for (int i = k + 1; i < r; ++i) {
            const double a = std::fabs(A[(size_t)i * r + k]);
            if (a > best) { best = a; p = i; }
        }
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < r; ++j) std::swap(A[(size_t)k * r + j], A[(size_t)p * r + j]);
        const double akk = A[(size_t)k * r + k];
        if (akk == 0.0) continue;
        for (int i = k + 1; i < r; ++i) {
            double &lik = A[(size_t)i * r + k];
            lik /= akk;
            for (int j = k + 1; j < r; ++j) A[(size_t)i * r + j] -= lik * A[(size_t)k * r + j];
        }
    }
}

// With P A = L U: A^T = U^T L^T P; solve U^T y = b, L^T z = y, then undo P.
void solve_row(const std::vector<double> &LU, const std::vector<int> &piv, int r, double *b)
{
    for (int j = 0; j < r; ++j) {
        double s = b[j];
        for (int i = 0; i < j; ++i) s -= LU[(size_t)i * r + j] * b[i];
        b[j] = s / LU[(size_t)j * r + j];
    }
    for (int j = r - 1; j >= 0; --j) {
        double s = b[j];
        for (int i = j + 1; i < r; ++i) s -= LU[(size_t)i * r + j] * b[i];
        b[j] = s;
    }
    for (int k = r - 1; k >= 0; --k)
        if (piv[k] != k) std::swap(b[k], b[piv[k]]);
}

uint64_t morton_key(const int32_t *a, int d, int bits)
{
    uint64_t key = 0;
    for (int b = 0; b < bits; ++b)
        for (int c = 0; c < d; ++c) key |= (uint64_t)((a[c] >> b) & 1) << (d * b + c);
    return key;
}

// Global id of the box with Morton index m at level l, or -1.
int32_t find_box(const HostRep &rep, int l, int64_t m)
{
    const int64_t *b = rep.box_morton.data() + rep.lev_off[l];
    const int64_t *e = rep.box_morton.data() + rep.lev_off[l + 1];
    const int64_t *it = std::lower_bound(b, e, m);
    if (it == e || *it != m) return -1;
    return rep.lev_off[l] + (int32_t)(it - b);
}

// Sec. 3.1 with the reading: bounding cube (centre of the bounding box,
// half-width the largest half extent, 1 for coincident points); leaf
// coordinate floor((x - (c - h)) 2^kappa / 2h) clamped; order by (Morton key,
// user index).
void make_tree(HostRep &rep, const double *points, int64_t leaf_size)
{
    const int d = rep.d;
    const int64_t n = rep.n;
    double lo[3], hi[3];
    for (int c = 0; c < d; ++c) lo[c] = hi[c] = points[c];
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < d; ++c) {
            const double x = points[i * d + c];
            lo[c] = std::min(lo[c], x);
            hi[c] = std::max(hi[c], x);
        }
    rep.half = 0.0;
    for (int c = 0; c < d; ++c) {
        rep.ctr[c] = (lo[c] + hi[c]) * 0.5;
        rep.half = std::max(rep.half, (hi[c] - lo[c]) * 0.5);
    }
    if (rep.half == 0.0) rep.half = 1.0;
    for (int c = 0; c < d; ++c) rep.origin[c] = rep.ctr[c] - rep.half;

    int kappa = 0;
    while (leaf_size * ((int64_t)1 << (d * kappa)) < n) ++kappa;
    rep.kappa = kappa;
    const int64_t side = (int64_t)1 << kappa;

    std::vector<uint64_t> key(n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int32_t a[3] = {0, 0, 0};
        for (int c = 0; c < d; ++c) {
            const double s = (points[i * d + c] - rep.origin[c]) * (double)side / (2.0 * rep.half);
            const double f = std::floor(s);
            int64_t v = f < 0.0 ? 0 : (int64_t)f;
            if (v > side - 1) v = side - 1;
            a[c] = (int32_t)v;
        }
        key[i] = morton_key(a, d, kappa);
    }
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return key[a] != key[b] ? key[a] < key[b] : a < b;
    });
    rep.perm = order;
    rep.pts.resize((size_t)n * d);
    std::vector<uint64_t> skey(n);
    for (int64_t t = 0; t < n; ++t) {
        std::memcpy(&rep.pts[(size_t)t * d], points + (size_t)order[t] * d, sizeof(double) * d);
        skey[t] = key[order[t]];
    }

    rep.lev_off.assign(kappa + 2, 0);
    for (int l = 0; l <= kappa; ++l) {
        const int sh = d * (kappa - l);
        int32_t nb = 0;
        for (int64_t t = 0; t < n; ++t)
            if (t == 0 || (skey[t] >> sh) != (skey[t - 1] >> sh)) ++nb;
        rep.lev_off[l + 1] = rep.lev_off[l] + nb;
    }
    const int32_t total = rep.lev_off[kappa + 1];
    rep.box_begin.assign(total, 0);
    rep.box_end.assign(total, 0);
    rep.box_parent.assign(total, -1);
    rep.box_cbeg.assign(total, 0);
    rep.box_cend.assign(total, 0);
    rep.box_coord.assign((size_t)total * 3, 0);
    rep.box_morton.assign(total, 0);
    for (int l = 0; l <= kappa; ++l) {
        const int sh = d * (kappa - l);
        int32_t g = rep.lev_off[l] - 1;
        for (int64_t t = 0; t < n; ++t) {
            if (t == 0 || (skey[t] >> sh) != (skey[t - 1] >> sh)) {
                ++g;
                const uint64_t m = skey[t] >> sh;
                rep.box_morton[g] = (int64_t)m;
                rep.box_begin[g] = (int32_t)t;
                for (int c = 0; c < d; ++c) {
                    int32_t v = 0;
                    for (int b = 0; b < l; ++b) v |= (int32_t)((m >> (d * b + c)) & 1) << b;
                    rep.box_coord[(size_t)g * 3 + c] = v;
                }
            }
            rep.box_end[g] = (int32_t)(t + 1);
        }
    }
    for (int l = 1; l <= kappa; ++l)
        for (int32_t g = rep.lev_off[l]; g < rep.lev_off[l + 1]; ++g) {
            const int32_t p = find_box(rep, l - 1, rep.box_morton[g] >> d);
            rep.box_parent[g] = p;
            if (rep.box_cend[p] == 0) rep.box_cbeg[p] = g;
            rep.box_cend[p] = g + 1;
        }
}

// Sec. 3.3 / Table "HOD_notation" with the reading clan(X) = children of the
// parent and of the parent's edge/face neighbours.  Classification of a
// same-level candidate Y != X by the offsets delta = |a_X - a_Y|: far if
// max delta >= 2, vertex sharing if every delta is 1, near otherwise.
void make_lists(HostRep &rep)
{
    const int d = rep.d, kappa = rep.kappa;
    const int32_t total = rep.nbox();
    std::vector<std::vector<int32_t>> L[3];
    for (int w = 0; w < 3; ++w) L[w].assign(total, {});
    int nofs = 1;
    for (int c = 0; c < d; ++c) nofs *= 3;
    L[0][0].push_back(0);
    for (int l = 1; l <= kappa; ++l) {
#pragma omp parallel for schedule(static)
        for (int32_t x = rep.lev_off[l]; x < rep.lev_off[l + 1]; ++x) {
            const int32_t P = rep.box_parent[x];
            const int32_t *aP = &rep.box_coord[(size_t)P * 3];
            const int32_t *ax = &rep.box_coord[(size_t)x * 3];
            const int32_t pside = 1 << (l - 1);
            for (int o = 0; o < nofs; ++o) {
                int32_t aq[3] = {0, 0, 0};
                int rem = o, nz = 0;
                bool inside = true;
                for (int c = 0; c < d; ++c) {
                    const int off = rem % 3 - 1;
                    rem /= 3;
                    nz += off != 0;
                    aq[c] = aP[c] + off;
                    inside = inside && aq[c] >= 0 && aq[c] < pside;
                }
                if (nz == d || !inside) continue;
                const int32_t Q = find_box(rep, l - 1, (int64_t)morton_key(aq, d, l - 1));
                if (Q < 0) continue;
                for (int32_t y = rep.box_cbeg[Q]; y < rep.box_cend[Q]; ++y) {
                    const int32_t *ay = &rep.box_coord[(size_t)y * 3];
                    int mx = 0, ones = 0;
                    for (int c = 0; c < d; ++c) {
                        const int dl = std::abs(ax[c] - ay[c]);
                        mx = std::max(mx, dl);
                        ones += dl == 1;
                    }
                    int w;
                    if (y == x) w = 0;
                    else if (mx >= 2) w = 1;
                    else if (ones == d) w = 2;
                    else w = 0;
                    if (w == 0 && l != kappa) continue;
                    L[w][x].push_back(y);
                }
            }
            for (int w = 0; w < 3; ++w) std::sort(L[w][x].begin(), L[w][x].end());
        }
    }
    for (int w = 0; w < 3; ++w) {
        rep.list_off[w].assign(total + 1, 0);
        for (int32_t x = 0; x < total; ++x) rep.list_off[w][x + 1] = rep.list_off[w][x] + (int64_t)L[w][x].size();
        rep.list_idx[w].resize(rep.list_off[w][total]);
        for (int32_t x = 0; x < total; ++x)
            std::copy(L[w][x].begin(), L[w][x].end(), rep.list_idx[w].begin() + rep.list_off[w][x]);
    }
    if (kappa > 0) { rep.list_off[0].assign(total + 1, 0); }
    if (kappa > 0) {
        // the near list lives at the leaf level only
        for (int32_t x = 0; x < total; ++x)
            rep.list_off[0][x + 1] = rep.list_off[0][x] + (int64_t)(x >= rep.leaf0() ? L[0][x].size() : 0);
        rep.list_idx[0].resize(rep.list_off[0][total]);
        for (int32_t x = rep.leaf0(); x < total; ++x)
            std::copy(L[0][x].begin(), L[0][x].end(), rep.list_idx[0].begin() + rep.list_off[0][x]);
    }
}

struct PivotSets {
    std::vector<std::vector<int32_t>> row, col; // per global box
};

// Run the cross approximation of K(I, J) for every box of one level.
template <class MakeSets>
void level_pivots(const HostRep &rep, int l, double eps, bool drop_confirm, PivotSets &ps, const MakeSets &make_sets)
{
    const int32_t b0 = rep.lev_off[l], b1 = rep.lev_off[l + 1];
    const int nth = omp_get_max_threads();
    const bool by_box = (b1 - b0) >= 2 * nth;
    auto one = [&](int32_t x, bool inner_par) {
        std::vector<int32_t> I, J;
        make_sets(x, I, J);
        Cross c;
        const double *pts = rep.pts.data();
        const int d = rep.d;
        auto entry = [&](int64_t a, int64_t b) {
            return kernel_entry(rep.ker, d, pts + (size_t)I[a] * d, pts + (size_t)J[b] * d);
        };
        cross_approx(entry, (int64_t)I.size(), (int64_t)J.size(), eps, inner_par, drop_confirm, c);
        ps.row[x].resize(c.rank);
        ps.col[x].resize(c.rank);
        for (int p = 0; p < c.rank; ++p) {
            ps.row[x][p] = I[c.prow[p]];
            ps.col[x][p] = J[c.pcol[p]];
        }
    };
    if (by_box) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int32_t x = b0; x < b1; ++x) one(x, false);
    } else {
        for (int32_t x = b0; x < b1; ++x) one(x, true);
    }
}

// B2T NCA on IL_far (Sec. 5.1.1 (1), Alg. "b2t"); reading: outgoing pivots are
// the incoming ones transposed (symmetric kernels, Sec. 3.4.3 remark).
// Coincident points: dup[t] is 1 when an earlier point of t's leaf has the
// same coordinates.  Their rows and columns of K are identical, so the cross
// approximations of both families take one point of each coincident set;
// otherwise a second copy can become a pivot on a rounding-level residual and
// make the pivot block singular.
std::vector<char> coincident(const HostRep &rep)
{
    const int d = rep.d;
    std::vector<char> dup(rep.n, 0);
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t g = rep.leaf0(); g < rep.nbox(); ++g)
        for (int32_t i = rep.box_begin[g]; i < rep.box_end[g]; ++i)
            for (int32_t j = rep.box_begin[g]; j < i && !dup[i]; ++j)
                if (!dup[j] && std::memcmp(&rep.pts[(size_t)i * d], &rep.pts[(size_t)j * d], sizeof(double) * d) == 0)
                    dup[i] = 1;
    return dup;
}

void far_pivots(const HostRep &rep, const std::vector<char> &dup, PivotSets &ps)
{
    const int kappa = rep.kappa;
    for (int l = kappa; l >= 2; --l) {
        level_pivots(rep, l, rep.eps_far, false, ps, [&](int32_t x, std::vector<int32_t> &I, std::vector<int32_t> &J) {
            const int64_t e0 = rep.list_off[1][x], e1 = rep.list_off[1][x + 1];
            if (e0 == e1) return;
            if (l == kappa) {
                for (int32_t t = rep.box_begin[x]; t < rep.box_end[x]; ++t)
                    if (!dup[t]) I.push_back(t);
                for (int64_t e = e0; e < e1; ++e) {
                    const int32_t y = rep.list_idx[1][e];
                    for (int32_t t = rep.box_begin[y]; t < rep.box_end[y]; ++t)
                        if (!dup[t]) J.push_back(t);
                }
            } else {
                for (int32_t c = rep.box_cbeg[x]; c < rep.box_cend[x]; ++c)
                    I.insert(I.end(), ps.row[c].begin(), ps.row[c].end());
                for (int64_t e = e0; e < e1; ++e) {
                    const int32_t y = rep.list_idx[1][e];
                    for (int32_t c = rep.box_cbeg[y]; c < rep.box_cend[y]; ++c)
                        J.insert(J.end(), ps.row[c].begin(), ps.row[c].end());
                }
            }
        });
    }
}

// T2B NCA on IL_ver (Sec. 5.1.1 (2)); reading: J is the union over every
// Y in IL_ver(X) (the printed loop keeps only the last Y) followed by the
// parent's incoming column pivots not already in J.
void vertex_pivots(const HostRep &rep, const std::vector<char> &dup, PivotSets &ps)
{
    for (int l = 1; l <= rep.kappa; ++l) {
        level_pivots(rep, l, rep.eps_ver, true, ps, [&](int32_t x, std::vector<int32_t> &I, std::vector<int32_t> &J) {
            for (int32_t t = rep.box_begin[x]; t < rep.box_end[x]; ++t)
                if (!dup[t]) I.push_back(t);
            for (int64_t e = rep.list_off[2][x]; e < rep.list_off[2][x + 1]; ++e) {
                const int32_t y = rep.list_idx[2][e];
                for (int32_t t = rep.box_begin[y]; t < rep.box_end[y]; ++t)
                    if (!dup[t]) J.push_back(t);
            }
            if (l > 1) {
                const size_t base = J.size();
                for (int32_t s : ps.col[rep.box_parent[x]])
                    if (std::find(J.begin(), J.begin() + base, s) == J.begin() + base) J.push_back(s);
            }
        });
    }
}

// Operators of Sec. 3.4.3 for one family from its pivots.
void make_operators(HostRep &rep, int f, const PivotSets &ps)
{
    Family &F = rep.fam[f];
    const int32_t total = rep.nbox();
    const int kappa = rep.kappa, d = rep.d;
    F.rank.assign(total, 0);
    F.coef_off.assign(total + 1, 0);
    F.op_rows.assign(total, 0);
    F.op_off.assign(total + 1, 0);
    for (int32_t x = 0; x < total; ++x) {
        const int l = rep.level_of(x);
        F.rank[x] = l >= F.lmin ? (int32_t)ps.row[x].size() : 0;
        F.coef_off[x + 1] = F.coef_off[x] + F.rank[x];
    }
    F.piv_row.resize(F.coef_off[total]);
    F.piv_col.resize(F.coef_off[total]);
    for (int32_t x = 0; x < total; ++x)
        for (int k = 0; k < F.rank[x]; ++k) {
            F.piv_row[F.coef_off[x] + k] = ps.row[x][k];
            F.piv_col[F.coef_off[x] + k] = ps.col[x][k];
        }
    for (int32_t x = 0; x < total; ++x) {
        if (F.rank[x] == 0) continue;
        const int l = rep.level_of(x);
        int32_t rows = 0;
        if (l == kappa) rows = rep.box_end[x] - rep.box_begin[x];
        else
            for (int32_t c = rep.box_cbeg[x]; c < rep.box_cend[x]; ++c) rows += F.rank[c];
        F.op_rows[x] = rows;
    }
    for (int32_t x = 0; x < total; ++x) F.op_off[x + 1] = F.op_off[x] + (int64_t)F.op_rows[x] * F.rank[x];
    F.op.assign(F.op_off[total], 0.0);
    const double *pts = rep.pts.data();
    auto K = [&](int32_t i, int32_t j) { return kernel_entry(rep.ker, d, pts + (size_t)i * d, pts + (size_t)j * d); };
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t x = 0; x < total; ++x) {
        const int r = F.rank[x];
        if (r == 0) continue;
        const int32_t *row = &F.piv_row[F.coef_off[x]], *col = &F.piv_col[F.coef_off[x]];
        std::vector<double> A((size_t)r * r);
        for (int a = 0; a < r; ++a)
            for (int b = 0; b < r; ++b) A[(size_t)a * r + b] = K(row[a], col[b]);
        std::vector<int> piv;
        lu_inplace(A, r, piv);
        std::vector<double> b(r);
        double *op = F.op.data() + F.op_off[x];
        const int32_t nrows = F.op_rows[x];
        if (rep.level_of(x) == kappa) {
            for (int32_t i = 0; i < nrows; ++i) {
                for (int c = 0; c < r; ++c) b[c] = K(rep.box_begin[x] + i, col[c]);
                solve_row(A, piv, r, b.data());
                for (int c = 0; c < r; ++c) op[(size_t)c * nrows + i] = b[c]; // column-major
            }
        } else {
            int32_t ir = 0;
            for (int32_t ch = rep.box_cbeg[x]; ch < rep.box_cend[x]; ++ch)
                for (int k = 0; k < F.rank[ch]; ++k, ++ir) {
                    for (int c = 0; c < r; ++c) b[c] = K(F.piv_row[F.coef_off[ch] + k], col[c]);
                    solve_row(A, piv, r, b.data());
                    for (int c = 0; c < r; ++c) op[(size_t)ir * r + c] = b[c]; // row-major
                }
        }
    }
}

// (H2+H)*: one ACA per unordered vertex-sharing pair at every level
// (Sec. 5.2.1, Alg. "pure_aca"); K(t^Y, t^X) uses the transposed factors.
void make_pairs(HostRep &rep)
{
    std::vector<LowRankPair> pairs;
    for (int l = 1; l <= rep.kappa; ++l)
        for (int32_t x = rep.lev_off[l]; x < rep.lev_off[l + 1]; ++x)
            for (int64_t e = rep.list_off[2][x]; e < rep.list_off[2][x + 1]; ++e) {
                const int32_t y = rep.list_idx[2][e];
                if (y > x) pairs.push_back({l, x, y, 0, 0, 0});
            }
    std::vector<Cross> cr(pairs.size());
    const int d = rep.d;
    const double *pts = rep.pts.data();
    const int nth = omp_get_max_threads();
    auto one = [&](size_t p, bool par) {
        const LowRankPair &P = pairs[p];
        const int32_t bx = rep.box_begin[P.x], by = rep.box_begin[P.y];
        auto entry = [&](int64_t a, int64_t b) {
            return kernel_entry(rep.ker, d, pts + (size_t)(bx + a) * d, pts + (size_t)(by + b) * d);
        };
        cross_approx(entry, rep.box_end[P.x] - bx, rep.box_end[P.y] - by, rep.eps_ver, par, false, cr[p]);
    };
    // coarse levels hold few, large pairs: approximate them one at a time with
    // the team on the elementwise loops; the many small ones run concurrently
    std::vector<size_t> big, small;
    for (size_t p = 0; p < pairs.size(); ++p) {
        const int64_t sz = rep.box_end[pairs[p].x] - rep.box_begin[pairs[p].x];
        (sz >= 16384 ? big : small).push_back(p);
    }
    for (size_t p : big) one(p, nth > 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (size_t i = 0; i < small.size(); ++i) one(small[i], false);
    int64_t off = 0;
    for (size_t p = 0; p < pairs.size(); ++p) {
        pairs[p].rank = cr[p].rank;
        pairs[p].off_u = off;
        off += (int64_t)cr[p].rank * cr[p].nI;
        pairs[p].off_v = off;
        off += (int64_t)cr[p].rank * cr[p].nJ;
    }
    rep.pair_data.assign(off, 0.0);
    for (size_t p = 0; p < pairs.size(); ++p) {
        std::copy(cr[p].U.begin(), cr[p].U.end(), rep.pair_data.begin() + pairs[p].off_u);
        std::copy(cr[p].V.begin(), cr[p].V.end(), rep.pair_data.begin() + pairs[p].off_v);
    }
    rep.pairs = std::move(pairs);
}

} // namespace

h2s_status build_host(const double *points, int64_t n, int d, const KernelSpec &k, int32_t leaf_size,
                      double eps_far, double eps_ver, int variant, int threads, HostRep &rep, std::string &err)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int saved = omp_get_max_threads();
    if (threads > 0) omp_set_num_threads(threads);
    try {
        rep = HostRep();
        rep.d = d;
        rep.n = n;
        rep.ker = k;
        rep.variant = variant;
        rep.eps_far = eps_far;
        rep.eps_ver = eps_ver;
        make_tree(rep, points, leaf_size);
        make_lists(rep);
        const int32_t total = rep.nbox();
        const std::vector<char> dup = coincident(rep);
        PivotSets far;
        far.row.assign(total, {});
        far.col.assign(total, {});
        far_pivots(rep, dup, far);
        rep.fam[0].lmin = 2;
        make_operators(rep, 0, far);
        rep.fam[1].lmin = 1;
        if (variant == H2S_H2STAR) {
            PivotSets ver;
            ver.row.assign(total, {});
            ver.col.assign(total, {});
            vertex_pivots(rep, dup, ver);
            make_operators(rep, 1, ver);
        } else {
            PivotSets none;
            none.row.assign(total, {});
            none.col.assign(total, {});
            make_operators(rep, 1, none);
            make_pairs(rep);
        }
    } catch (const std::bad_alloc &) {
        if (threads > 0) omp_set_num_threads(saved);
        err = "host out of memory during build";
        return H2S_ERR_OUT_OF_MEMORY;
    } catch (const std::exception &e) {
        if (threads > 0) omp_set_num_threads(saved);
        err = std::string("host build failed: ") + e.what();
        return H2S_ERR_INTERNAL;
    }
    if (threads > 0) omp_set_num_threads(saved);
    rep.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return H2S_OK;
}

// ---------------------------------------------------------------------------
// Export: "H2SX" magic, uint32 version, uint32 array count, then per array:
// char name[32], uint32 dtype (1 int32, 2 int64, 3 float64), uint32 ndim,
// int64 dims[ndim], raw little-endian data.
// ---------------------------------------------------------------------------
namespace {
struct Writer {
    FILE *f;
    uint32_t count = 0;
    template <class T> void arr(const char *name, uint32_t dtype, const std::vector<T> &v)
    {
        char nm[32] = {0};
        std::snprintf(nm, sizeof(nm), "%s", name);
        const uint32_t ndim = 1;
        const int64_t dim = (int64_t)v.size();
        std::fwrite(nm, 1, 32, f);
        std::fwrite(&dtype, 4, 1, f);
        std::fwrite(&ndim, 4, 1, f);
        std::fwrite(&dim, 8, 1, f);
        if (!v.empty()) std::fwrite(v.data(), sizeof(T), v.size(), f);
        ++count;
    }
};
} // namespace

h2s_status export_host(const HostRep &rep, const char *path, std::string &err)
{
    FILE *f = std::fopen(path, "wb");
    if (!f) {
        err = std::string("cannot open ") + path;
        return H2S_ERR_INVALID_ARG;
    }
    std::fwrite("H2SX", 1, 4, f);
    const uint32_t version = 1;
    std::fwrite(&version, 4, 1, f);
    const long count_pos = std::ftell(f);
    uint32_t zero = 0;
    std::fwrite(&zero, 4, 1, f);
    Writer w{f};
    std::vector<int64_t> meta = {rep.d, rep.kappa, rep.n, rep.variant};
    w.arr("meta", 2, meta);
    std::vector<double> geo = {rep.ctr[0], rep.ctr[1], rep.ctr[2], rep.half};
    w.arr("cube", 3, geo);
    w.arr("perm", 1, rep.perm);
    w.arr("points", 3, rep.pts);
    w.arr("lev_off", 1, rep.lev_off);
    w.arr("box_begin", 1, rep.box_begin);
    w.arr("box_end", 1, rep.box_end);
    w.arr("box_parent", 1, rep.box_parent);
    w.arr("box_coord", 1, rep.box_coord);
    w.arr("box_morton", 2, rep.box_morton);
    const char *ln[3] = {"near", "far", "ver"};
    for (int i = 0; i < 3; ++i) {
        w.arr((std::string(ln[i]) + "_off").c_str(), 2, rep.list_off[i]);
        w.arr((std::string(ln[i]) + "_idx").c_str(), 1, rep.list_idx[i]);
    }
    const char *fn[2] = {"far", "ver"};
    for (int i = 0; i < 2; ++i) {
        const Family &F = rep.fam[i];
        const std::string p = std::string("fam_") + fn[i] + "_";
        w.arr((p + "rank").c_str(), 1, F.rank);
        w.arr((p + "coef_off").c_str(), 2, F.coef_off);
        w.arr((p + "piv_row").c_str(), 1, F.piv_row);
        w.arr((p + "piv_col").c_str(), 1, F.piv_col);
        w.arr((p + "op_off").c_str(), 2, F.op_off);
        w.arr((p + "op_rows").c_str(), 1, F.op_rows);
        w.arr((p + "op").c_str(), 3, F.op);
    }
    std::vector<int64_t> pr;
    for (const LowRankPair &P : rep.pairs) {
        pr.push_back(P.level); pr.push_back(P.x); pr.push_back(P.y);
        pr.push_back(P.rank); pr.push_back(P.off_u); pr.push_back(P.off_v);
    }
    w.arr("pairs", 2, pr);
    w.arr("pair_data", 3, rep.pair_data);
    std::fseek(f, count_pos, SEEK_SET);
    std::fwrite(&w.count, 4, 1, f);
    const bool ok = std::ferror(f) == 0;
    std::fclose(f);
    if (!ok) {
        err = std::string("write failed: ") + path;
        return H2S_ERR_INTERNAL;
    }
    return H2S_OK;
}

} // namespace h2s
