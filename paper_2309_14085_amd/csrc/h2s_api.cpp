// h2s_api.cpp -- the C ABI declared in include/h2s.h.
//
// build: validate, construct the representation on the host
// (h2s_host_build.cpp), pack it into the device layout of h2s_device.hpp in
// the requested precision and copy it to HBM on the caller's stream.
// apply: validate, then enqueue the MVP kernels (h2s_kernels.hip) once per
// right-hand side.  solve: validate, make sure the FP64 and inner-precision
// representations are on the device, and run the GMRES driver
// (h2s_solve.cpp) with the products as callbacks.  Nothing here computes any
// part of the product or of the solve.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "h2s.h"
#include "h2s_blas.hpp"
#include "h2s_device.hpp"
#include "h2s_eval_rate.hpp"
#include "h2s_host.hpp"
#include "h2s_solve.hpp"

namespace {

thread_local std::string g_last_error;

h2s_alloc_fn g_alloc = nullptr;
h2s_free_fn g_free = nullptr;
void *g_alloc_ctx = nullptr;

h2s_status fail(h2s_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

int default_alloc(void *, size_t bytes, void **p) { return hipMalloc(p, bytes) == hipSuccess ? 0 : 1; }

// Lookup table of the device kernel function (extended precision, rounded once).
std::vector<double> kernel_table(int kind)
{
    std::vector<double> tab;
    if (kind == H2S_K_LOG_R || kind == H2S_K_RBF_LOG) {
        // 0.5 ln x by table reduction: subinterval i of m in [1/2, 1) has centre
        // z_i = 1/2 + (i + 1/2)/512; store c_i = 1/z_i and T_i = -0.5 ln c_i,
        // then T_i once more as a head Th_i on the grid 2^-43 and the rest Tl_i
        tab.resize(1024);
        for (int i = 0; i < 256; ++i) {
            const double c = 1.0 / (0.5 + (i + 0.5) / 512.0);
            const long double T = -0.5L * std::log((long double)c);
            const long double h = std::ldexp(std::nearbyint(std::ldexp(T, 43)), -43);
            tab[2 * i] = c;
            tab[2 * i + 1] = (double)T;
            tab[512 + 2 * i] = (double)h;
            tab[512 + 2 * i + 1] = (double)(T - h);
        }
    } else if (kind == H2S_K_GAUSSIAN || kind == H2S_K_EXP_R) {
        for (int j = 0; j < 64; ++j) tab.push_back((double)std::exp2((long double)j / 64.0L)); // 2^(j/64)
    } else {
        tab.assign(2, 0.0);
    }
    return tab;
}

// Scalar parameters of the device kernel function: kparam = -1/h^2 for the
// Gaussian; for the piecewise RBFs of radius a, kc = (a^2, and the two branch
// factors: a, 1/a for a/r | r/a; 1/log a, 1/(a log a - 1) for the log RBF).
void kernel_scalars(int kind, double a, double &kparam, double kc[3])
{
    kparam = kind == H2S_K_GAUSSIAN ? -1.0 / (a * a) : 0.0;
    kc[0] = kc[1] = kc[2] = 0.0;
    if (kind == H2S_K_RBF_AR) {
        kc[0] = a * a;
        kc[1] = a;
        kc[2] = 1.0 / a;
    } else if (kind == H2S_K_RBF_LOG) {
        const long double la = std::log((long double)a);
        kc[0] = a * a;
        kc[1] = (double)(1.0L / la);
        kc[2] = (double)(1.0L / ((long double)a * la - 1.0L));
    }
}
void default_free(void *, void *p) { (void)hipFree(p); }

} // namespace

struct h2s_tree_s {
    h2s::HostRep rep;
    h2s_build_opts opts{};
    h2s_kernel ker{};
    bool host_only = false;
    int device = 0;
    h2s_alloc_fn afn = default_alloc;
    h2s_free_fn ffn = default_free;
    void *actx = nullptr;
    std::vector<void *> allocs;
    size_t device_bytes = 0;
    int64_t operator_bytes = 0;
    int64_t leaf_kept[2] = {0, 0}, transfer_kept[2] = {0, 0}; // stored (non-unit) operator entries per family
    std::vector<int32_t> lev_off;
    h2s::LaunchPlan plan{};
    h2s::DevTree<h2s::P64> t64{};
    h2s::DevTree<h2s::P32> t32{};
    h2s::DevTree<h2s::P32M> t32m{};
    // profiling: (class, start, stop) events recorded by apply while enabled
    bool profiling = false;
    struct Mark {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    // second stream for the near field and the events that fork / join it
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_fork2 = nullptr, ev_join = nullptr;
    // third stream for the leaf-level M2L and its fork / join events
    hipStream_t aux2 = nullptr;
    hipEvent_t ev_fork3 = nullptr, ev_join2 = nullptr;
    // fourth stream for the M2L of the level above the leaves and its fork / join events
    hipStream_t aux3 = nullptr;
    hipEvent_t ev_fork4 = nullptr, ev_join3 = nullptr;
    // per family: index in its targets of the first box of every level
    std::vector<int32_t> tlev[2];
    // which precisions are on the device
    bool up[3] = {false, false, false};
    // multi-RHS block buffers allocated for these precisions
    bool batch[3] = {false, false, false};
    // solve workspace for restart length solve_m (device memory is in allocs)
    int solve_m = 0;
    h2s::SolveWork work{};
    // lockstep workspace of several right-hand sides: restart length many_m, many.cols columns
    int many_m = 0;
    h2s::SolveWorkMany many{};

    void clear_marks()
    {
        for (Mark &m : marks) {
            (void)hipEventDestroy(m.a);
            (void)hipEventDestroy(m.b);
        }
        marks.clear();
    }

    ~h2s_tree_s()
    {
        clear_marks();
        if (aux) {
            (void)hipStreamSynchronize(aux);
            (void)hipStreamDestroy(aux);
        }
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_fork2) (void)hipEventDestroy(ev_fork2);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (aux2) {
            (void)hipStreamSynchronize(aux2);
            (void)hipStreamDestroy(aux2);
        }
        if (ev_fork3) (void)hipEventDestroy(ev_fork3);
        if (ev_join2) (void)hipEventDestroy(ev_join2);
        if (aux3) {
            (void)hipStreamSynchronize(aux3);
            (void)hipStreamDestroy(aux3);
        }
        if (ev_fork4) (void)hipEventDestroy(ev_fork4);
        if (ev_join3) (void)hipEventDestroy(ev_join3);
        if (work.small_host) (void)hipHostFree(work.small_host);
        if (many.host) (void)hipHostFree(many.host);
        if (many.host_idx) (void)hipHostFree(many.host_idx);
        for (void *p : allocs) ffn(actx, p);
    }
};

// A group of trees applied together (see h2s_group_apply).  H2* trees of
// one precision (FP64 or FP32), kernel function and dimension that number
// two or more form a fused class: one launch per step for all of them
// (h2s::MultiPlan).  Every other tree's product is captured, alone, as a HIP
// graph on the group's capture stream (the tree's near-field and M2L streams
// joining it through their events, as in any single-product capture) and
// replayed on the tree's lane.
struct h2s_group_s {
    struct Fused {
        int prec = 0, kind = 0, d = 0;
        std::vector<int32_t> members;                 // indices into trees
        h2s::MultiPlan<h2s::P64> mp64{};
        h2s::MultiPlan<h2s::P32> mp32{};
        const double **xs_dev = nullptr;              // device arrays of the members' vectors
        double **ys_dev = nullptr;
        std::vector<const double *> xs;               // what they hold
        std::vector<double *> ys;
    };
    std::vector<h2s_tree> trees;
    std::vector<Fused> fused;
    std::vector<char> in_fused;         // per tree
    std::vector<void *> dev;            // device allocations of the fused classes
    hipStream_t faux = nullptr;         // near-field stream of the fused classes
    hipEvent_t ffork = nullptr, fjoin = nullptr;
    int device = 0;
    hipStream_t cap = nullptr;          // capture stream
    std::vector<hipStream_t> lanes;     // one per tree: the stream its graph is launched on
    std::vector<hipEvent_t> done;       // one per tree: joins its lane back into the caller's stream
    hipEvent_t start = nullptr;         // forks every lane from the caller's stream
    std::vector<hipGraph_t> graphs;     // one per tree
    std::vector<hipGraphExec_t> execs;
    std::vector<const double *> xs;     // the vectors each graph holds
    std::vector<double *> ys;

    void drop_graph(size_t i)
    {
        if (execs[i]) (void)hipGraphExecDestroy(execs[i]);
        if (graphs[i]) (void)hipGraphDestroy(graphs[i]);
        execs[i] = nullptr;
        graphs[i] = nullptr;
    }

    ~h2s_group_s()
    {
        for (hipStream_t s : lanes)
            if (s) (void)hipStreamSynchronize(s);
        for (size_t i = 0; i < graphs.size(); ++i) drop_graph(i);
        for (hipStream_t s : lanes)
            if (s) (void)hipStreamDestroy(s);
        for (hipEvent_t e : done)
            if (e) (void)hipEventDestroy(e);
        if (start) (void)hipEventDestroy(start);
        if (cap) (void)hipStreamDestroy(cap);
        if (faux) {
            (void)hipStreamSynchronize(faux);
            (void)hipStreamDestroy(faux);
        }
        if (ffork) (void)hipEventDestroy(ffork);
        if (fjoin) (void)hipEventDestroy(fjoin);
        for (void *p : dev) (void)hipFree(p);
    }
};

namespace {
void record_mark(void *ctx, int cls, int end, void *stream)
{
    h2s_tree t = (h2s_tree)ctx;
    if (!end) {
        h2s_tree_s::Mark m{cls, nullptr, nullptr};
        if (hipEventCreate(&m.a) != hipSuccess || hipEventCreate(&m.b) != hipSuccess) return;
        (void)hipEventRecord(m.a, (hipStream_t)stream);
        t->marks.push_back(m);
    } else {
        // the most recent open mark of this class (marks of the two streams interleave)
        for (auto it = t->marks.rbegin(); it != t->marks.rend(); ++it)
            if (it->cls == cls) {
                (void)hipEventRecord(it->b, (hipStream_t)stream);
                break;
            }
    }
}
} // namespace

namespace {

struct Uploader {
    h2s_tree t;
    hipStream_t s;
    h2s_status st = H2S_OK;

    void *raw(size_t bytes)
    {
        if (st != H2S_OK) return nullptr;
        void *p = nullptr;
        if (bytes == 0) bytes = 256;
        const int64_t budget = t->opts.hbm_budget_bytes;
        if (budget > 0 && (int64_t)(t->device_bytes + bytes) > budget) {
            st = fail(H2S_ERR_OUT_OF_MEMORY, "device allocation of " + std::to_string(bytes) +
                                                 " bytes would exceed the handle's budget of " + std::to_string(budget) +
                                                 " bytes (" + std::to_string(t->device_bytes) + " held)");
            return nullptr;
        }
        if (t->afn(t->actx, bytes, &p) != 0 || !p) {
            st = fail(H2S_ERR_OUT_OF_MEMORY, "device allocation of " + std::to_string(bytes) + " bytes failed");
            return nullptr;
        }
        t->allocs.push_back(p);
        t->device_bytes += bytes;
        return p;
    }
    template <class T> T *copy(const std::vector<T> &v)
    {
        // the host vectors are temporaries: wait for each copy before they go away
        T *p = (T *)raw(sizeof(T) * v.size());
        if (p && !v.empty() &&
            (hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
             hipStreamSynchronize(s) != hipSuccess))
            st = fail(H2S_ERR_DEVICE, "host-to-device copy failed during upload");
        return p;
    }
    template <class T> T *zeros(size_t n)
    {
        T *p = (T *)raw(sizeof(T) * n);
        if (p && n && hipMemsetAsync(p, 0, sizeof(T) * n, s) != hipSuccess)
            st = fail(H2S_ERR_DEVICE, "hipMemsetAsync failed during upload");
        return p;
    }
};

// Centre of a global box from its integer coordinates.
void box_centre(const h2s::HostRep &r, int32_t g, double *c)
{
    const int l = r.level_of(g);
    const double w = 2.0 * r.half / (double)((int64_t)1 << l);
    for (int k = 0; k < 3; ++k) c[k] = k < r.d ? r.origin[k] + (r.box_coord[(size_t)g * 3 + k] + 0.5) * w : 0.0;
}

// Pack one family for the device: pivot coordinates (box-centred when
// `local`), both copies of the leaf bases and transfers, lists, work list.
template <typename CT, typename BT>
void upload_family(Uploader &up, const h2s::HostRep &r, int f, const std::vector<double> &ctr, bool local,
                   h2s::DevFamily<CT, BT> &G, int64_t &op_bytes, int64_t &leaf_kept, int64_t &transfer_kept)
{
    const h2s::Family &F = r.fam[f];
    const int d = r.d, kappa = r.kappa;
    const int32_t nbox = r.nbox(), leaf0 = r.leaf0();
    G.lmin = F.lmin;
    std::vector<int32_t> co(nbox + 1);
    for (int32_t g = 0; g <= nbox; ++g) co[g] = (int32_t)F.coef_off[g];
    G.coef_off = up.copy(co);
    const size_t nc = (size_t)F.coef_off[nbox];
    const bool xw = r.ker.kind == H2S_K_NTI_MQ; // pivots carry c(x) = exp(-(x_1 + x_3))
    std::vector<CT> pvx(nc ? nc : 1), pvy(nc ? nc : 1), pvz(nc ? nc : 1), pvw(xw && nc ? nc : 1);
    for (int32_t g = 0; g < nbox; ++g)
        for (int64_t c = F.coef_off[g]; c < F.coef_off[g + 1]; ++c) {
            const double *p = &r.pts[(size_t)F.piv_row[c] * d];
            const double *cc = &ctr[(size_t)g * 3];
            pvx[c] = (CT)(local ? p[0] - cc[0] : p[0]);
            pvy[c] = (CT)(local ? p[1] - cc[1] : p[1]);
            pvz[c] = d == 3 ? (CT)(local ? p[2] - cc[2] : p[2]) : CT(0);
            if (xw) pvw[c] = (CT)std::exp(-(p[0] + p[2]));
        }
    G.pvx = up.copy(pvx);
    G.pvy = up.copy(pvy);
    G.pvz = up.copy(pvz);
    G.pvw = up.copy(pvw);
    // leaf bases: the host keeps U_X column-major (n_X x r).  The row of U_X at the point of row
    // pivot a is e_a (K(t, s) K(t, s)^-1, Sec. 3.4.3); rows that are exactly e_a are not stored:
    // P2M adds the pivot's charge in the row's place and L2P copies the local.  The kept rows, in
    // order, are stored column-major and row-major; ukeep[b + j] = local row of kept row j,
    // urow[b + i] = kept index of local row i or ~a for the unit row of coefficient a, uprow[c] =
    // local row of coefficient c's unit row or -1, upos[c] = kept rows before that row.
    const int32_t nleaf = r.nleaf();
    const size_t npt = (size_t)r.n;
    std::vector<uint16_t> ukeep(npt ? npt : 1, 0);
    std::vector<int16_t> urow(npt ? npt : 1, 0), uprow(nc ? nc : 1, -1), upos(nc ? nc : 1, 0);
    std::vector<int32_t> unk(nleaf ? nleaf : 1, 0);
    std::vector<int64_t> uoff(nleaf + 1, 0);
    for (int32_t lf = 0; lf < nleaf; ++lf) {
        const int32_t g = leaf0 + lf, b = r.box_begin[g];
        const int64_t rk = F.rank[g], nx = F.op_rows[g];
        const double *src = F.op.data() + F.op_off[g];
        std::vector<int> unit(nx, -1);
        for (int64_t a = 0; a < rk; ++a) {
            const int64_t i = F.piv_row[F.coef_off[g] + a] - b;
            if (i < 0 || i >= nx || unit[i] >= 0) continue;
            bool e = true;
            for (int64_t k = 0; k < rk && e; ++k) e = src[k * nx + i] == (k == a ? 1.0 : 0.0);
            if (e) {
                unit[i] = (int)a;
                uprow[F.coef_off[g] + a] = (int16_t)i;
            }
        }
        int32_t j = 0;
        for (int64_t i = 0; i < nx; ++i) {
            if (unit[i] >= 0) {
                urow[b + i] = (int16_t)~unit[i];
                upos[F.coef_off[g] + unit[i]] = (int16_t)j;
            } else {
                urow[b + i] = (int16_t)j;
                ukeep[b + j] = (uint16_t)i;
                ++j;
            }
        }
        unk[lf] = j;
        uoff[lf + 1] = uoff[lf] + (int64_t)j * rk;
    }
    std::vector<BT> ucm(uoff.back() ? uoff.back() : 1), urm(uoff.back() ? uoff.back() : 1);
    for (int32_t lf = 0; lf < nleaf; ++lf) {
        const int32_t g = leaf0 + lf, b = r.box_begin[g];
        const int64_t rk = F.rank[g], nx = F.op_rows[g], nk = unk[lf];
        const double *src = F.op.data() + F.op_off[g];
        for (int64_t k = 0; k < rk; ++k)
            for (int64_t j = 0; j < nk; ++j) {
                const int64_t i = ukeep[b + j];
                ucm[uoff[lf] + k * nk + j] = (BT)src[k * nx + i];
                urm[uoff[lf] + j * rk + k] = (BT)src[k * nx + i];
            }
    }
    G.U_cm = up.copy(ucm);
    G.U_rm = up.copy(urm);
    G.uoff = up.copy(uoff);
    G.ukeep = up.copy(ukeep);
    G.urow = up.copy(urow);
    G.uprow = up.copy(uprow);
    G.upos = up.copy(upos);
    G.unk = up.copy(unk);
    op_bytes += (int64_t)(2 * sizeof(BT) * uoff.back());
    leaf_kept = uoff.back();
    // transfers: the host keeps them row-major ((sum r_c) x r).  Row k of box g's transfer
    // belongs to child coefficient bf + k (bf = the first child's first coefficient).  With
    // nested pivots, the row of a child pivot that is also the box's row pivot a is e_a; rows
    // that are exactly e_a are not stored, as for the leaf bases: M2M adds that child's
    // coefficient in the row's place, L2L copies the box's local.  tkeep[bf + j] = stacked row
    // of kept row j, trow[bf + k] = kept index of row k or ~a, tprow[c] = stacked row of
    // coefficient c's unit row or -1, tpos[c] = kept rows before it, tnk[g] = kept rows.
    std::vector<int32_t> tnk(nbox ? nbox : 1, 0);
    std::vector<uint16_t> tkeep(nc ? nc : 1, 0);
    std::vector<int16_t> trow(nc ? nc : 1, 0), tprow(nc ? nc : 1, -1), tpos(nc ? nc : 1, 0);
    std::vector<int64_t> toff(nbox + 1, 0);
    for (int32_t g = 0; g < nbox; ++g) {
        toff[g + 1] = toff[g];
        if (g >= leaf0 || F.rank[g] == 0) continue;
        const int64_t rk = F.rank[g], rows = F.op_rows[g];
        const int64_t c0 = F.coef_off[g], bf = F.coef_off[r.box_cbeg[g]];
        const double *src = F.op.data() + F.op_off[g];
        std::vector<std::pair<int32_t, int32_t>> pv; // (pivot point, a), sorted
        for (int64_t a = 0; a < rk; ++a) pv.push_back({F.piv_row[c0 + a], (int32_t)a});
        std::sort(pv.begin(), pv.end());
        std::vector<char> used(rk, 0);
        int32_t j = 0;
        for (int64_t k = 0; k < rows; ++k) {
            const int32_t pt = F.piv_row[bf + k];
            auto it = std::lower_bound(pv.begin(), pv.end(), std::make_pair(pt, (int32_t)-1));
            int a = -1;
            if (it != pv.end() && it->first == pt && !used[it->second]) {
                a = it->second;
                for (int64_t c = 0; c < rk && a >= 0; ++c)
                    if (src[k * rk + c] != (c == a ? 1.0 : 0.0)) a = -1;
            }
            if (a >= 0) {
                used[a] = 1;
                trow[bf + k] = (int16_t)~a;
                tprow[c0 + a] = (int16_t)k;
                tpos[c0 + a] = (int16_t)j;
            } else {
                trow[bf + k] = (int16_t)j;
                tkeep[bf + j] = (uint16_t)k;
                ++j;
            }
        }
        tnk[g] = j;
        toff[g + 1] = toff[g] + (int64_t)j * rk;
    }
    std::vector<double> trm(toff.back() ? toff.back() : 1), tcm(toff.back() ? toff.back() : 1);
    for (int32_t g = 0; g < leaf0; ++g) {
        const int64_t rk = F.rank[g], nk = tnk[g];
        if (rk == 0) continue;
        const int64_t bf = F.coef_off[r.box_cbeg[g]];
        const double *src = F.op.data() + F.op_off[g];
        for (int64_t j = 0; j < nk; ++j)
            for (int64_t k = 0; k < rk; ++k) {
                const double v = src[(int64_t)tkeep[bf + j] * rk + k];
                trm[toff[g] + j * rk + k] = v;
                tcm[toff[g] + k * nk + j] = v;
            }
    }
    G.Tr_rm = up.copy(trm);
    G.Tr_cm = up.copy(tcm);
    G.troff = up.copy(toff);
    G.tnk = up.copy(tnk);
    G.tkeep = up.copy(tkeep);
    G.trow = up.copy(trow);
    G.tprow = up.copy(tprow);
    G.tpos = up.copy(tpos);
    op_bytes += (int64_t)(2 * sizeof(double) * toff.back());
    transfer_kept = toff.back();
    const int w = f == 0 ? 1 : 2;
    std::vector<int32_t> ilo(nbox + 1);
    for (int32_t g = 0; g <= nbox; ++g) ilo[g] = (int32_t)r.list_off[w][g];
    G.il_off = up.copy(ilo);
    G.il_idx = up.copy(r.list_idx[w]);
    std::vector<int32_t> targets;
    for (int32_t g = 0; g < nbox; ++g)
        if (F.rank[g] > 0) targets.push_back(g);
    G.ntargets = (int32_t)targets.size();
    G.targets_leaf = (int32_t)(std::lower_bound(targets.begin(), targets.end(), leaf0) - targets.begin());
    G.targets = up.copy(targets);
    G.ncoef = (int32_t)nc;
    G.v = up.template zeros<double>(nc ? nc : 1);
    G.u = up.template zeros<double>(nc ? nc : 1);
    (void)kappa;
}

template <class P> h2s_status upload(h2s_tree t, hipStream_t s, h2s::DevTree<P> &D)
{
    using PT = typename P::pt_t;
    using BT = typename P::basis_t;
    const h2s::HostRep &r = t->rep;
    const int d = r.d, kappa = r.kappa;
    const int32_t nbox = r.nbox(), leaf0 = r.leaf0(), nleaf = r.nleaf();
    const int64_t n = r.n;
    Uploader up{t, s};

    D = h2s::DevTree<P>{};
    D.n = (int32_t)n;
    D.d = d;
    D.kappa = kappa;
    D.nleaf = nleaf;
    D.leaf0 = leaf0;
    D.nbox = nbox;
    D.kind = r.ker.kind;
    D.diag = r.ker.diag;
    D.shift = r.ker.shift;
    kernel_scalars(r.ker.kind, r.ker.param, D.kparam, D.kc);
    D.variant = r.variant;
    D.max_leaf = 1;
    for (int32_t g = leaf0; g < nbox; ++g) D.max_leaf = std::max(D.max_leaf, r.box_end[g] - r.box_begin[g]);
    D.max_rows = 1;
    D.max_rank = 1;
    for (int f = 0; f < 2; ++f)
        for (int32_t g = 0; g < nbox; ++g) {
            D.max_rank = std::max(D.max_rank, r.fam[f].rank[g]);
            if (g < leaf0) D.max_rows = std::max(D.max_rows, r.fam[f].op_rows[g]);
        }
    // Leaves (P2M: the kept rows' charges of both families), stacked transfer
    // rows (both families at once) and ranks are staged whole in LDS (64 KiB
    // per block); an M2L source box must fit the kernel's staging group, which
    // bounds the rank.
    const int32_t leaf_cap = 4096, lds_cap = 5120, rank_cap = 512;
    if (D.max_leaf > leaf_cap)
        return fail(H2S_ERR_UNSUPPORTED, "a leaf holds more than " + std::to_string(leaf_cap) +
                                             " points; use a smaller leaf_size");
    if (2 * D.max_rows > lds_cap)
        return fail(H2S_ERR_UNSUPPORTED, "a stacked transfer exceeds " + std::to_string(lds_cap / 2) +
                                             " rows; use a smaller leaf_size");
    for (int w = 0; w <= 2; ++w) // near, far and vertex lists
        for (int32_t g = 0; g + 1 < (int32_t)r.list_off[w].size(); ++g)
            if (r.list_off[w][g + 1] - r.list_off[w][g] > h2s::kMaxList)
                return fail(H2S_ERR_UNSUPPORTED, "an interaction list exceeds " + std::to_string(h2s::kMaxList) + " boxes");
    if (kappa > h2s::kMaxLevels)
        return fail(H2S_ERR_UNSUPPORTED, "tree depth exceeds " + std::to_string(h2s::kMaxLevels) + " levels");
    if (D.max_rank > rank_cap)
        return fail(H2S_ERR_UNSUPPORTED, "a basis rank exceeds " + std::to_string(rank_cap) +
                                             "; use a larger tolerance or a smaller leaf_size");

    std::vector<double> ctr((size_t)nbox * 3);
    for (int32_t g = 0; g < nbox; ++g) box_centre(r, g, &ctr[(size_t)g * 3]);

    D.perm = up.copy(r.perm);
    {
        const bool xw = r.ker.kind == H2S_K_NTI_MQ; // points carry c(x) = exp(-(x_1 + x_3)), not centred
        std::vector<PT> px(n), py(n), pz(d == 3 ? n : 1), pw(xw ? n : 1);
        for (int32_t g = leaf0; g < nbox; ++g)
            for (int32_t i = r.box_begin[g]; i < r.box_end[g]; ++i) {
                const double *p = &r.pts[(size_t)i * d];
                const double *c = &ctr[(size_t)g * 3];
                px[i] = (PT)(P::local ? p[0] - c[0] : p[0]);
                py[i] = (PT)(P::local ? p[1] - c[1] : p[1]);
                if (d == 3) pz[i] = (PT)(P::local ? p[2] - c[2] : p[2]);
                if (xw) pw[i] = (PT)std::exp(-(p[0] + p[2]));
            }
        D.px = up.copy(px);
        D.py = up.copy(py);
        D.pz = up.copy(pz);
        D.pw = up.copy(pw);
    }
    D.box_begin = up.copy(r.box_begin);
    D.box_end = up.copy(r.box_end);
    D.box_cbeg = up.copy(r.box_cbeg);
    D.box_cend = up.copy(r.box_cend);
    D.box_ctr = up.copy(ctr);
    {
        std::vector<int32_t> anc((size_t)nleaf * (kappa + 1));
        for (int32_t lf = 0; lf < nleaf; ++lf) {
            int32_t g = leaf0 + lf;
            for (int l = kappa; l >= 0; --l) {
                anc[(size_t)lf * (kappa + 1) + l] = g;
                g = l > 0 ? r.box_parent[g] : g;
            }
        }
        D.leaf_anc = up.copy(anc);
        std::vector<int32_t> noff(nleaf + 1, 0), nidx;
        for (int32_t lf = 0; lf < nleaf; ++lf) {
            const int32_t g = leaf0 + lf;
            for (int64_t e = r.list_off[0][g]; e < r.list_off[0][g + 1]; ++e) nidx.push_back(r.list_idx[0][e] - leaf0);
            noff[lf + 1] = (int32_t)nidx.size();
        }
        D.near_off = up.copy(noff);
        D.near_idx = up.copy(nidx);
        // symmetric near field: leaf X < X' evaluates the pair and writes n_X' column sums for X'
        std::vector<int32_t> nself(nleaf ? nleaf : 1, 0);
        std::vector<int64_t> nw(nidx.size() ? nidx.size() : 1, -1);
        int64_t nws = 0;
        for (int32_t lf = 0; lf < nleaf; ++lf) {
            int32_t e = noff[lf];
            while (e < noff[lf + 1] && nidx[e] < lf) ++e;
            nself[lf] = e; // nidx[e] == lf: every leaf is in its own near list
            for (int32_t u = e + 1; u < noff[lf + 1]; ++u) {
                nw[u] = nws;
                nws += r.box_end[leaf0 + nidx[u]] - r.box_begin[leaf0 + nidx[u]];
            }
        }
        for (int32_t lf = 0; lf < nleaf; ++lf)
            for (int32_t e = noff[lf]; e < nself[lf]; ++e) {
                const int32_t x = nidx[e]; // below lf: its entry for lf holds the offset
                const auto b0 = nidx.begin() + noff[x], b1 = nidx.begin() + noff[x + 1];
                nw[e] = nw[std::lower_bound(b0, b1, lf) - nidx.begin()];
            }
        if (nws > INT32_MAX) return fail(H2S_ERR_UNSUPPORTED, "near-field column sums exceed 2^31 entries");
        D.near_self = up.copy(nself);
        D.near_w = up.copy(nw);
        D.near_wv = up.template zeros<double>(nws ? nws : 1);
    }
    upload_family(up, r, 0, ctr, sizeof(typename P::far_t) == 4, D.far, t->operator_bytes, t->leaf_kept[0],
                  t->transfer_kept[0]);
    upload_family(up, r, 1, ctr, false, D.ver, t->operator_bytes, t->leaf_kept[1], t->transfer_kept[1]);
    if (r.variant == H2S_H2_PLUS_H) {
        auto &Pr = D.pairs;
        const size_t np = r.pairs.size();
        Pr.npairs = (int32_t)np;
        std::vector<int32_t> px(np), py(np), pr(np);
        std::vector<int64_t> pu(np), pv(np), pw(np);
        int64_t woff = 0;
        for (size_t p = 0; p < np; ++p) {
            px[p] = r.pairs[p].x;
            py[p] = r.pairs[p].y;
            pr[p] = r.pairs[p].rank;
            pu[p] = r.pairs[p].off_u;
            pv[p] = r.pairs[p].off_v;
            pw[p] = woff;
            woff += 2 * (int64_t)r.pairs[p].rank;
        }
        Pr.px = up.copy(px);
        Pr.py = up.copy(py);
        Pr.prank = up.copy(pr);
        Pr.pu = up.copy(pu);
        Pr.pv = up.copy(pv);
        Pr.pw = up.copy(pw);
        std::vector<BT> data(r.pair_data.size());
        for (size_t i = 0; i < data.size(); ++i) data[i] = (BT)r.pair_data[i];
        t->operator_bytes += (int64_t)(sizeof(BT) * data.size());
        Pr.data = up.copy(data);
        Pr.w = up.template zeros<double>(woff ? woff : 1);
        std::vector<std::vector<int32_t>> rec(nbox);
        for (size_t p = 0; p < np; ++p) {
            rec[px[p]].push_back((int32_t)(2 * p));
            rec[py[p]].push_back((int32_t)(2 * p + 1));
        }
        std::vector<int32_t> roff(nbox + 1, 0), ridx;
        for (int32_t g = 0; g < nbox; ++g) {
            ridx.insert(ridx.end(), rec[g].begin(), rec[g].end());
            roff[g + 1] = (int32_t)ridx.size();
        }
        Pr.recv_off = up.copy(roff);
        Pr.recv = up.copy(ridx);
        const int32_t CHR = 2048; // rows per chunk (the partial-product kernel stages them in LDS)
        std::vector<int32_t> cp, cs, cb, cl, sco(2 * np + 1, 0);
        std::vector<int64_t> cpo;
        int64_t poff = 0;
        for (size_t p = 0; p < np; ++p)
            for (int side = 0; side < 2; ++side) {
                const int32_t box = side == 0 ? py[p] : px[p];
                const int32_t rows = r.box_end[box] - r.box_begin[box];
                if (pr[p] > 0)
                    for (int32_t s0 = 0; s0 < rows; s0 += CHR) {
                        cp.push_back((int32_t)p);
                        cs.push_back(side);
                        cb.push_back(s0);
                        cl.push_back(std::min(CHR, rows - s0));
                        cpo.push_back(poff);
                        poff += pr[p];
                    }
                sco[2 * p + side + 1] = (int32_t)cp.size();
            }
        Pr.nchunks = (int32_t)cp.size();
        Pr.chunk_pair = up.copy(cp);
        Pr.chunk_side = up.copy(cs);
        Pr.chunk_begin = up.copy(cb);
        Pr.chunk_len = up.copy(cl);
        Pr.chunk_poff = up.copy(cpo);
        Pr.side_chunk_off = up.copy(sco);
        Pr.partial = up.template zeros<double>(poff ? poff : 1);
    }
    D.qt = up.template zeros<double>(n);
    D.yn = up.template zeros<double>(n);
    D.ktab = up.copy(kernel_table(r.ker.kind));
    if (up.st != H2S_OK) return up.st;
    if (hipStreamSynchronize(s) != hipSuccess) return fail(H2S_ERR_DEVICE, "stream synchronisation failed after upload");
    return H2S_OK;
}

bool is_finite(double v) { return std::isfinite(v); }

// The device copy a precision uses: FP32_M2L and FP32_BF16M2L share the float-far-field copy.
int rep_slot(int p) { return p == H2S_FP32_BF16M2L ? (int)H2S_FP32_M2L : p; }

bool low_m2l(int p) { return p == H2S_FP32_M2L || p == H2S_FP32_BF16M2L; }

// Upload the representation in precision p unless it is already on the device.
h2s_status ensure_uploaded(h2s_tree t, h2s_precision p, hipStream_t s)
{
    const int sl = rep_slot(p);
    if (t->up[sl]) return H2S_OK;
    h2s_status st;
    if (p == H2S_FP64) st = upload<h2s::P64>(t, s, t->t64);
    else if (p == H2S_FP32) st = upload<h2s::P32>(t, s, t->t32);
    else st = upload<h2s::P32M>(t, s, t->t32m);
    if (st == H2S_OK) t->up[sl] = true;
    return st;
}

// The near-field and leaf-level M2L streams and their fork / join events,
// created on first use on the handle's device at the default priority.
h2s_status ensure_streams(h2s_tree t)
{
    if (t->aux) return H2S_OK;
    constexpr int NE = 7;
    hipStream_t a = nullptr, a2 = nullptr, a3 = nullptr;
    hipEvent_t ev[NE] = {};
    bool ok = hipStreamCreateWithFlags(&a, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&a2, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&a3, hipStreamNonBlocking) == hipSuccess;
    for (int i = 0; ok && i < NE; ++i) ok = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        if (a) (void)hipStreamDestroy(a);
        if (a2) (void)hipStreamDestroy(a2);
        if (a3) (void)hipStreamDestroy(a3);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        return fail(H2S_ERR_DEVICE, "creating the near-field / M2L streams or their events failed");
    }
    t->aux = a;
    t->aux2 = a2;
    t->aux3 = a3;
    t->ev_fork = ev[0];
    t->ev_fork2 = ev[1];
    t->ev_join = ev[2];
    t->ev_fork3 = ev[3];
    t->ev_join2 = ev[4];
    t->ev_join3 = ev[5];
    t->ev_fork4 = ev[6];
    return H2S_OK;
}

h2s::Streams streams_of(h2s_tree t, void *stream)
{
    return h2s::Streams{stream,  t->aux,      t->ev_fork,  t->ev_fork2, t->ev_join,
                        t->aux2, t->ev_fork3, t->ev_join2, t->aux3,     t->ev_fork4, t->ev_join3};
}

// The default schedule: blocks as wide as the outputs of the widest box of
// a level (both families), in whole wavefronts, and the near field split
// kNearFirstDefault / rest around M2L.
void default_plan(h2s_tree t)
{
    const h2s::HostRep &r = t->rep;
    const int kappa = std::min(r.kappa, h2s::kMaxLevels);
    auto threads = [](int32_t outputs) { return std::min(512, std::max(64, (outputs + 63) / 64 * 64)); };
    t->plan = h2s::LaunchPlan{};
    t->plan.lev_off = t->lev_off.data();
    t->plan.near_first = h2s::kNearFirstDefault;
    t->plan.m2l_stream = 2;
    // targets of a family: its boxes of positive rank, in box order (as uploaded)
    for (int f = 0; f < 2; ++f) {
        std::vector<int32_t> &tl = t->tlev[f];
        tl.assign((size_t)r.kappa + 2, 0);
        int32_t k = 0;
        for (int l = 0; l <= r.kappa; ++l) {
            tl[l] = k;
            for (int32_t g = r.lev_off[l]; g < r.lev_off[l + 1]; ++g) k += r.fam[f].rank[g] > 0;
        }
        tl[(size_t)r.kappa + 1] = k;
        t->plan.tlev[f] = tl.data();
    }
    for (int l = 0; l <= h2s::kMaxLevels; ++l) t->plan.up_threads[l] = t->plan.dn_threads[l] = 64;
    for (int l = 0; l <= kappa; ++l) {
        int32_t cols = 0, rows = 0;
        for (int32_t g = r.lev_off[l]; g < r.lev_off[l + 1]; ++g) {
            cols = std::max(cols, r.fam[0].rank[g] + r.fam[1].rank[g]);
            if (l < kappa) rows = std::max(rows, r.fam[0].op_rows[g] + r.fam[1].op_rows[g]);
        }
        t->plan.up_threads[l] = threads(cols);
        t->plan.dn_threads[l] = threads(rows);
    }
}

// One product in precision p (uploaded, streams created) under plan; hipError_t as int.
int mvp_plan(h2s_tree t, const h2s::LaunchPlan &plan, h2s_precision p, uint32_t mask, const double *x, double *y,
             void *stream, const h2s::ProfileHook *prof)
{
    const h2s::Streams st = streams_of(t, stream);
    if (p == H2S_FP64) return h2s::launch_mvp<h2s::P64>(t->t64, plan, x, y, mask, st, prof);
    if (p == H2S_FP32) return h2s::launch_mvp<h2s::P32>(t->t32, plan, x, y, mask, st, prof);
    return h2s::launch_mvp<h2s::P32M>(t->t32m, plan, x, y, mask, st, prof);
}

int mvp(h2s_tree t, h2s_precision p, uint32_t mask, const double *x, double *y, void *stream,
        const h2s::ProfileHook *prof)
{
    return mvp_plan(t, t->plan, p, mask, x, y, stream, prof);
}

// Milliseconds per product under plan: the faster of two runs of reps products.
h2s_status time_plan(h2s_tree t, const h2s::LaunchPlan &plan, const double *x, double *y, int reps,
                     hipStream_t s, hipEvent_t e0, hipEvent_t e1, double &ms)
{
    ms = INFINITY;
    for (int trial = 0; trial < 2; ++trial) {
        if (hipEventRecord(e0, s) != hipSuccess) return fail(H2S_ERR_DEVICE, "hipEventRecord failed");
        for (int k = 0; k < reps; ++k) {
            const int rc = mvp_plan(t, plan, t->opts.prec, H2S_PHASE_ALL, x, y, s, nullptr);
            if (rc != 0)
                return fail(H2S_ERR_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString((hipError_t)rc));
        }
        float f = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&f, e0, e1) != hipSuccess)
            return fail(H2S_ERR_DEVICE, "timing the product failed");
        ms = std::min(ms, (double)f / reps);
    }
    return H2S_OK;
}

// Coordinate search over the schedule (see h2s_tune).
h2s_status tune_plan(h2s_tree t, const double *x, double *y, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                     h2s_tune_info &info)
{
    const int kappa = std::min(t->rep.kappa, h2s::kMaxLevels);
    h2s::LaunchPlan best = t->plan;
    double best_ms = 0.0, ms = 0.0;
    h2s_status st;
    // one untimed product, then the schedule at entry
    if (mvp_plan(t, best, t->opts.prec, H2S_PHASE_ALL, x, y, s, nullptr) != 0)
        return fail(H2S_ERR_DEVICE, "kernel launch failed");
    if ((st = time_plan(t, best, x, y, reps, s, e0, e1, best_ms)) != H2S_OK) return st;
    info.ms_entry = best_ms;
    info.candidates = 1;
    auto consider = [&](const h2s::LaunchPlan &cand) -> h2s_status {
        h2s_status r2 = time_plan(t, cand, x, y, reps, s, e0, e1, ms);
        if (r2 != H2S_OK) return r2;
        ++info.candidates;
        if (ms < best_ms * (1.0 - 0.005)) {
            best = cand;
            best_ms = ms;
        }
        return H2S_OK;
    };
    const double shares[] = {0.0, 0.2, 0.4, 0.5, 0.6, 0.7, 0.8, 1.0};
    auto tune_share = [&]() -> h2s_status {
        const double cur = best.near_first;
        for (double f : shares) {
            if (f == cur) continue;
            h2s::LaunchPlan c = best;
            c.near_first = f;
            h2s_status r2 = consider(c);
            if (r2 != H2S_OK) return r2;
        }
        return H2S_OK;
    };
    if (kappa >= 1) {
        {
            const int32_t cur = best.m2l_stream;
            for (int32_t m = 0; m <= 2; ++m) {
                if (m == cur) continue;
                h2s::LaunchPlan c = best;
                c.m2l_stream = m;
                if ((st = consider(c)) != H2S_OK) return st;
            }
        }
        if ((st = tune_share()) != H2S_OK) return st;
        // P2M (level kappa) and M2M (levels kappa-1 .. 1), then L2L (levels 1 .. kappa-1)
        for (int pass = 0; pass < 2; ++pass) {
            const int l0 = pass == 0 ? kappa : 1, l1 = pass == 0 ? 1 : kappa - 1, dl = pass == 0 ? -1 : 1;
            for (int l = l0; pass == 0 ? l >= l1 : l <= l1; l += dl) {
                const int cur = pass == 0 ? best.up_threads[l] : best.dn_threads[l];
                for (int w = 64; w <= 512; w += 64) {
                    if (w == cur) continue;
                    h2s::LaunchPlan c = best;
                    (pass == 0 ? c.up_threads[l] : c.dn_threads[l]) = w;
                    if ((st = consider(c)) != H2S_OK) return st;
                }
            }
        }
        if ((st = tune_share()) != H2S_OK) return st;
    }
    t->plan = best;
    info.ms_tuned = best_ms;
    // leave y = K~ x under the installed schedule
    if (mvp(t, t->opts.prec, H2S_PHASE_ALL, x, y, s, nullptr) != 0 || hipStreamSynchronize(s) != hipSuccess)
        return fail(H2S_ERR_DEVICE, "the final product failed");
    return H2S_OK;
}

// The batched product serves H2* with a double far field.
template <class P> bool batch_supported(h2s_tree t, const h2s::DevTree<P> &)
{
    return t->rep.variant == H2S_H2STAR;
}

// Allocate the multi-RHS block buffers of precision p on first use.
template <class P> h2s_status ensure_batch(h2s_tree t, h2s::DevTree<P> &D, int p, hipStream_t s)
{
    p = rep_slot(p);
    if (t->batch[p]) return H2S_OK;
    Uploader up{t, s};
    const size_t nb = (size_t)h2s::kBatch * h2s::kGroupBlocks; // kGroupBlocks blocks of kBatch columns
    D.qb = up.template zeros<double>((size_t)D.n * nb);
    D.ynb = up.template zeros<double>((size_t)D.n * nb);
    const size_t nf = (size_t)t->rep.fam[0].coef_off.back(), nv = (size_t)t->rep.fam[1].coef_off.back();
    D.far.vb = up.template zeros<double>((nf ? nf : 1) * nb);
    D.far.ub = up.template zeros<double>((nf ? nf : 1) * nb);
    D.ver.vb = up.template zeros<double>((nv ? nv : 1) * nb);
    D.ver.ub = up.template zeros<double>((nv ? nv : 1) * nb);
    if (up.st != H2S_OK) return up.st;
    t->batch[p] = true;
    return H2S_OK;
}

// y = K~ x for nrhs columns: blocks of kBatch through the batched product when
// it applies, otherwise one column at a time.
template <class P>
h2s_status apply_columns(h2s_tree t, h2s::DevTree<P> &D, int p, uint32_t mask, const double *x, double *y,
                         int32_t nrhs, int64_t ldx, int64_t ldy, void *stream, const h2s::ProfileHook *prof)
{
    const h2s::Streams st = streams_of(t, stream);
    int32_t c = 0;
    if (nrhs > 1 && !prof && batch_supported(t, D)) {
        const h2s_status bs = ensure_batch(t, D, p, (hipStream_t)stream);
        if (bs != H2S_OK) return bs;
        for (; c + 1 < nrhs; c += h2s::kGroupCols) {
            const int na = std::min<int32_t>(h2s::kGroupCols, nrhs - c);
            const int rc = h2s::launch_mvp_batch<P>(D, t->plan, x + c * ldx, ldx, y + c * ldy, ldy, na, mask, st,
                                                    p == H2S_FP32_BF16M2L);
            if (rc != 0)
                return fail(H2S_ERR_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString((hipError_t)rc));
        }
    }
    for (; c < nrhs; ++c) {
        const int rc = h2s::launch_mvp<P>(D, t->plan, x + c * ldx, y + c * ldy, mask, st, prof);
        if (rc != 0) return fail(H2S_ERR_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString((hipError_t)rc));
    }
    return H2S_OK;
}

struct SolveCtx {
    h2s_tree t;
    h2s_precision inner;
    void *stream;
};

int solve_apply_inner(void *c, const double *x, double *y)
{
    const SolveCtx *s = (const SolveCtx *)c;
    return mvp(s->t, s->inner, H2S_PHASE_ALL, x, y, s->stream, nullptr);
}

int solve_apply_outer(void *c, const double *x, double *y)
{
    const SolveCtx *s = (const SolveCtx *)c;
    return mvp(s->t, H2S_FP64, H2S_PHASE_ALL, x, y, s->stream, nullptr);
}

// Y = K~ X for ncols columns in precision p, through the batched product (h2s_apply's path).
int apply_many(h2s_tree t, h2s_precision p, const double *x, int64_t ldx, double *y, int64_t ldy, int ncols, void *stream)
{
    h2s_status st;
    if (p == H2S_FP64) st = apply_columns(t, t->t64, H2S_FP64, H2S_PHASE_ALL, x, y, ncols, ldx, ldy, stream, nullptr);
    else if (p == H2S_FP32) st = apply_columns(t, t->t32, H2S_FP32, H2S_PHASE_ALL, x, y, ncols, ldx, ldy, stream, nullptr);
    else st = apply_columns(t, t->t32m, p, H2S_PHASE_ALL, x, y, ncols, ldx, ldy, stream, nullptr);
    return st == H2S_OK ? 0 : (int)hipErrorUnknown;
}

int solve_apply_inner_many(void *c, const double *x, int64_t ldx, double *y, int64_t ldy, int ncols)
{
    const SolveCtx *s = (const SolveCtx *)c;
    return apply_many(s->t, s->inner, x, ldx, y, ldy, ncols, s->stream);
}

int solve_apply_outer_many(void *c, const double *x, int64_t ldx, double *y, int64_t ldy, int ncols)
{
    const SolveCtx *s = (const SolveCtx *)c;
    return apply_many(s->t, H2S_FP64, x, ldx, y, ldy, ncols, s->stream);
}

} // namespace

namespace {

// Device copy of a host vector, owned by the group.
template <typename T> T *group_copy(h2s_group g, const std::vector<T> &v, bool &ok)
{
    if (!ok || v.empty()) return nullptr;
    void *p = nullptr;
    if (hipMalloc(&p, v.size() * sizeof(T)) != hipSuccess) {
        ok = false;
        return nullptr;
    }
    g->dev.push_back(p);
    if (hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) ok = false;
    return (T *)p;
}

// The launch steps of a fused class (see h2s::MultiPlan).
template <class P>
bool build_multi(h2s_group g, h2s_group_s::Fused &f, h2s::MultiPlan<P> &mp, h2s::DevTree<P> h2s_tree_s::*member)
{
    bool ok = true;
    const int m = (int)f.members.size();
    std::vector<h2s::DevTree<P>> trees(m);
    std::vector<int2> perm, leaf, up, far, ver;
    std::vector<std::vector<int2>> m2m, l2l;
    std::vector<int32_t> w_m2m, w_l2l;
    int32_t w_up = 64, max_leaf = 1, max_rows = 1, max_rank = 1;
    for (int i = 0; i < m; ++i) {
        h2s_tree t = g->trees[f.members[i]];
        const h2s::DevTree<P> &D = t->*member;
        const h2s::HostRep &r = t->rep;
        trees[i] = D;
        const int kappa = std::min(r.kappa, h2s::kMaxLevels);
        for (int32_t c = 0; c < (D.n + 255) / 256; ++c) perm.push_back(make_int2(i, c));
        for (int32_t lf = 0; lf < D.nleaf; ++lf) leaf.push_back(make_int2(i, lf));
        max_leaf = std::max(max_leaf, D.max_leaf);
        max_rows = std::max(max_rows, D.max_rows);
        max_rank = std::max(max_rank, D.max_rank);
        if (kappa < 1) continue;
        for (int32_t lf = 0; lf < D.nleaf; ++lf) up.push_back(make_int2(i, lf));
        w_up = std::max(w_up, t->plan.up_threads[kappa]);
        for (int32_t k = 0; k < D.far.ntargets; ++k) far.push_back(make_int2(i, k));
        for (int32_t k = 0; k < D.ver.ntargets; ++k) ver.push_back(make_int2(i, k));
        for (int k = 0; k + 1 < kappa; ++k) {
            if ((int)m2m.size() <= k) {
                m2m.emplace_back();
                l2l.emplace_back();
                w_m2m.push_back(64);
                w_l2l.push_back(64);
            }
            const int lu = kappa - 1 - k, ld = 1 + k; // M2M into level lu, L2L from level ld
            for (int32_t b = r.lev_off[lu]; b < r.lev_off[lu + 1]; ++b) m2m[k].push_back(make_int2(i, b));
            for (int32_t b = r.lev_off[ld]; b < r.lev_off[ld + 1]; ++b) l2l[k].push_back(make_int2(i, b));
            w_m2m[k] = std::max(w_m2m[k], t->plan.up_threads[lu]);
            w_l2l[k] = std::max(w_l2l[k], t->plan.dn_threads[ld]);
        }
    }
    mp = h2s::MultiPlan<P>{};
    mp.trees = group_copy(g, trees, ok);
    mp.perm_map = group_copy(g, perm, ok);
    mp.leaf_map = group_copy(g, leaf, ok);
    mp.up_map = group_copy(g, up, ok);
    mp.far_map = group_copy(g, far, ok);
    mp.ver_map = group_copy(g, ver, ok);
    mp.n_perm = (int32_t)perm.size();
    mp.n_leaf = (int32_t)leaf.size();
    mp.n_up = (int32_t)up.size();
    mp.n_far = (int32_t)far.size();
    mp.n_ver = (int32_t)ver.size();
    mp.steps = (int32_t)m2m.size();
    for (int k = 0; k < mp.steps; ++k) {
        mp.m2m_map[k] = group_copy(g, m2m[k], ok);
        mp.l2l_map[k] = group_copy(g, l2l[k], ok);
        mp.n_m2m[k] = (int32_t)m2m[k].size();
        mp.n_l2l[k] = (int32_t)l2l[k].size();
        mp.w_m2m[k] = w_m2m[k];
        mp.w_l2l[k] = w_l2l[k];
    }
    mp.w_up = w_up;
    mp.lds_leaf = sizeof(double) * (size_t)(2 * max_leaf);
    mp.lds_rows = sizeof(double) * (size_t)(2 * max_rows);
    mp.lds_rank = sizeof(double) * (size_t)(2 * max_rank);
    f.xs_dev = group_copy(g, std::vector<const double *>(m, nullptr), ok);
    f.ys_dev = group_copy(g, std::vector<double *>(m, nullptr), ok);
    mp.xs = f.xs_dev;
    mp.ys = f.ys_dev;
    f.xs.assign(m, nullptr);
    f.ys.assign(m, nullptr);
    return ok;
}

} // namespace

extern "C" {

const char *h2s_status_string(h2s_status s)
{
    switch (s) {
    case H2S_OK: return "ok";
    case H2S_ERR_INVALID_ARG: return "invalid argument";
    case H2S_ERR_OUT_OF_MEMORY: return "out of memory";
    case H2S_ERR_DEVICE: return "device error";
    case H2S_ERR_NOT_CONVERGED: return "not converged";
    case H2S_ERR_UNSUPPORTED: return "unsupported";
    case H2S_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

h2s_status h2s_last_error(char *buf, size_t len)
{
    if (!buf || len == 0) return H2S_ERR_INVALID_ARG;
    std::strncpy(buf, g_last_error.c_str(), len - 1);
    buf[len - 1] = '\0';
    return H2S_OK;
}

h2s_status h2s_set_allocator(h2s_alloc_fn alloc_fn, h2s_free_fn free_fn, void *ctx)
{
    if ((alloc_fn == nullptr) != (free_fn == nullptr))
        return fail(H2S_ERR_INVALID_ARG, "allocator and free function must be given together");
    g_alloc = alloc_fn;
    g_free = free_fn;
    g_alloc_ctx = ctx;
    return H2S_OK;
}

h2s_status h2s_build(const double *points, int64_t n, int32_t d, const h2s_kernel *k, const h2s_build_opts *o,
                     void *stream, h2s_tree *out)
{
    if (!out) return fail(H2S_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!points) return fail(H2S_ERR_INVALID_ARG, "points is NULL");
    if (n < 1 || n > INT32_MAX) return fail(H2S_ERR_INVALID_ARG, "n must be in [1, 2^31 - 1]");
    if (d != 2 && d != 3) return fail(H2S_ERR_INVALID_ARG, "d must be 2 or 3");
    if (!k || !o) return fail(H2S_ERR_INVALID_ARG, "kernel or options is NULL");
    if (k->kind < H2S_K_LOG_R || k->kind > H2S_K_NTI_MQ) return fail(H2S_ERR_INVALID_ARG, "unknown kernel kind");
    if (k->kind == H2S_K_NTI_MQ && d != 3) return fail(H2S_ERR_INVALID_ARG, "the NTI multiquadric needs d = 3");
    if (k->kind == H2S_K_NTI_MQ && o && low_m2l(o->prec))
        return fail(H2S_ERR_UNSUPPORTED, "H2S_FP32_M2L and H2S_FP32_BF16M2L are not available for the NTI multiquadric");
    if ((k->kind == H2S_K_RBF_AR || k->kind == H2S_K_RBF_LOG) && !(is_finite(k->param) && k->param > 0))
        return fail(H2S_ERR_INVALID_ARG, "the RBF radius (param) must be finite and > 0");
    if (k->kind == H2S_K_RBF_LOG && k->param == 1.0) return fail(H2S_ERR_INVALID_ARG, "RBF_LOG needs param != 1");
    if (k->kind == H2S_K_GAUSSIAN && !(is_finite(k->param) && k->param > 0))
        return fail(H2S_ERR_INVALID_ARG, "Gaussian length scale must be finite and > 0");
    if (!is_finite(k->diag) || !is_finite(k->shift)) return fail(H2S_ERR_INVALID_ARG, "diag and shift must be finite");
    if (o->leaf_size < 1) return fail(H2S_ERR_INVALID_ARG, "leaf_size must be >= 1");
    if (!(is_finite(o->eps_far) && o->eps_far >= 0 && is_finite(o->eps_ver) && o->eps_ver >= 0))
        return fail(H2S_ERR_INVALID_ARG, "tolerances must be finite and >= 0");
    if (o->variant != H2S_H2STAR && o->variant != H2S_H2_PLUS_H) return fail(H2S_ERR_INVALID_ARG, "unknown variant");
    if (o->prec != H2S_FP64 && o->prec != H2S_FP32 && o->prec != H2S_FP32_M2L && o->prec != H2S_FP32_BF16M2L)
        return fail(H2S_ERR_INVALID_ARG, "unknown precision");
    for (int64_t i = 0; i < n * d; ++i)
        if (!is_finite(points[i])) return fail(H2S_ERR_INVALID_ARG, "points must be finite");

    int dev = 0;
    if (!o->host_only) {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
            return fail(H2S_ERR_DEVICE, "no HIP device available (use host_only for a host-side build)");
        if (hipGetDevice(&dev) != hipSuccess) return fail(H2S_ERR_DEVICE, "hipGetDevice failed");
    }

    h2s_tree t = new (std::nothrow) h2s_tree_s();
    if (!t) return fail(H2S_ERR_OUT_OF_MEMORY, "host allocation failed");
    t->opts = *o;
    t->ker = *k;
    t->host_only = o->host_only != 0;
    t->device = dev;
    if (g_alloc) {
        t->afn = g_alloc;
        t->ffn = g_free;
        t->actx = g_alloc_ctx;
    }
    std::string err;
    const h2s::KernelSpec ks{k->kind, k->param, k->diag, k->shift};
    h2s_status st = h2s::build_host(points, n, d, ks, o->leaf_size, o->eps_far, o->eps_ver, o->variant,
                                    o->host_threads, t->rep, err);
    if (st != H2S_OK) {
        delete t;
        return fail(st, err);
    }
    t->lev_off = t->rep.lev_off;
    default_plan(t);
    if (!t->host_only) {
        st = ensure_uploaded(t, o->prec, (hipStream_t)stream);
        if (st != H2S_OK) {
            const std::string keep = g_last_error;
            delete t;
            g_last_error = keep;
            return st;
        }
    }
    *out = t;
    return H2S_OK;
}

h2s_status h2s_apply_phases(h2s_tree t, uint32_t mask, const double *x, double *y, int32_t nrhs, int64_t ldx,
                            int64_t ldy, void *stream)
{
    if (!t) return fail(H2S_ERR_INVALID_ARG, "tree is NULL");
    if (t->host_only) return fail(H2S_ERR_UNSUPPORTED, "handle was built with host_only");
    if (mask == 0 || (mask & ~(uint32_t)H2S_PHASE_ALL)) return fail(H2S_ERR_INVALID_ARG, "bad phase mask");
    const int64_t n = t->rep.n;
    if (!x || !y) return fail(H2S_ERR_INVALID_ARG, "x or y is NULL");
    if (nrhs < 1) return fail(H2S_ERR_INVALID_ARG, "nrhs must be >= 1");
    if (ldx < n || ldy < n) return fail(H2S_ERR_INVALID_ARG, "leading dimensions must be >= n");
    const char *xb = (const char *)x, *xe = (const char *)(x + ldx * (nrhs - 1) + n);
    const char *yb = (const char *)y, *ye = (const char *)(y + ldy * (nrhs - 1) + n);
    if (xb < ye && yb < xe) return fail(H2S_ERR_INVALID_ARG, "x and y overlap");
    if (hipSetDevice(t->device) != hipSuccess) return fail(H2S_ERR_DEVICE, "hipSetDevice failed");
    if (ensure_streams(t) != H2S_OK) return H2S_ERR_DEVICE;
    h2s::ProfileHook hook{t, record_mark};
    const h2s::ProfileHook *prof = t->profiling ? &hook : nullptr;
    if (t->opts.prec == H2S_FP64) return apply_columns(t, t->t64, H2S_FP64, mask, x, y, nrhs, ldx, ldy, stream, prof);
    if (t->opts.prec == H2S_FP32) return apply_columns(t, t->t32, H2S_FP32, mask, x, y, nrhs, ldx, ldy, stream, prof);
    return apply_columns(t, t->t32m, t->opts.prec, mask, x, y, nrhs, ldx, ldy, stream, prof);
}

h2s_status h2s_apply(h2s_tree t, const double *x, double *y, int32_t nrhs, int64_t ldx, int64_t ldy, void *stream)
{
    return h2s_apply_phases(t, H2S_PHASE_ALL, x, y, nrhs, ldx, ldy, stream);
}

h2s_status h2s_apply_noalloc(h2s_tree t, const double *x, double *y, int32_t nrhs, int64_t ldx, int64_t ldy,
                             void *stream)
{
    if (!t) return fail(H2S_ERR_INVALID_ARG, "tree is NULL");
    if (t->host_only) return fail(H2S_ERR_UNSUPPORTED, "handle was built with host_only");
    const int64_t n = t->rep.n;
    if (!x || !y) return fail(H2S_ERR_INVALID_ARG, "x or y is NULL");
    if (nrhs < 1 || nrhs > h2s::kGroupCols) return fail(H2S_ERR_INVALID_ARG, "nrhs must be in 1..32");
    if (ldx < n || ldy < n) return fail(H2S_ERR_INVALID_ARG, "leading dimensions must be >= n");
    const char *xb = (const char *)x, *xe = (const char *)(x + ldx * (nrhs - 1) + n);
    const char *yb = (const char *)y, *ye = (const char *)(y + ldy * (nrhs - 1) + n);
    if (xb < ye && yb < xe) return fail(H2S_ERR_INVALID_ARG, "x and y overlap");
    if (t->rep.variant != H2S_H2STAR || (t->opts.prec != H2S_FP64 && t->opts.prec != H2S_FP32))
        return fail(H2S_ERR_UNSUPPORTED, "h2s_apply_noalloc takes H2* handles of precision FP64 or FP32");
    // the active blocks' buffers, each block's at a fixed stride as the batched kernels expect
    const size_t nblk = (size_t)(nrhs + h2s::kBatch - 1) / h2s::kBatch, NB = h2s::kBatch;
    const size_t nf = (size_t)t->rep.fam[0].coef_off.back(), nv = (size_t)t->rep.fam[1].coef_off.back();
    const size_t need = nblk * NB * (2 * (size_t)n + 2 * (nf ? nf : 1) + 2 * (nv ? nv : 1)) * sizeof(double);
    if (need > H2S_NOALLOC_SCRATCH_BYTES)
        return fail(H2S_ERR_UNSUPPORTED, "the batch buffers need " + std::to_string(need) + " bytes, above the " +
                                             std::to_string((size_t)H2S_NOALLOC_SCRATCH_BYTES) +
                                             "-byte scratch array: use fewer columns or h2s_apply");
    if (hipSetDevice(t->device) != hipSuccess) return fail(H2S_ERR_DEVICE, "hipSetDevice failed");
    double *scr = nullptr;
    const hipError_t se = h2s::noalloc_scratch(t->device, &scr);
    if (se != hipSuccess) return fail(H2S_ERR_DEVICE, std::string("hipGetSymbolAddress failed: ") + hipGetErrorString(se));
    if (ensure_streams(t) != H2S_OK) return H2S_ERR_DEVICE;
    const h2s::Streams st = streams_of(t, stream);
    auto run = [&](auto D) -> h2s_status { // D: a copy of the handle's tree, its batch buffers in the array
        double *p = scr;
        D.qb = p;
        p += nblk * NB * n;
        D.ynb = p;
        p += nblk * NB * n;
        D.far.vb = p;
        p += nblk * NB * (nf ? nf : 1);
        D.far.ub = p;
        p += nblk * NB * (nf ? nf : 1);
        D.ver.vb = p;
        p += nblk * NB * (nv ? nv : 1);
        D.ver.ub = p;
        const int rc = h2s::launch_mvp_batch(D, t->plan, x, ldx, y, ldy, nrhs, H2S_PHASE_ALL, st);
        if (rc != 0) return fail(H2S_ERR_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString((hipError_t)rc));
        return H2S_OK;
    };
    return t->opts.prec == H2S_FP64 ? run(t->t64) : run(t->t32);
}

h2s_status h2s_solve_opts_default(h2s_solve_opts *o)
{
    if (!o) return fail(H2S_ERR_INVALID_ARG, "opts is NULL");
    o->restart = 50;
    o->max_iter = 10000;
    o->max_refine = 1000;
    o->inner_prec = H2S_FP32;
    o->rtol = 1e-8;
    o->inner_rtol = 1e-6;
    o->use_x0 = 0;
    return H2S_OK;
}

h2s_status h2s_solve(h2s_tree t, const double *b, double *x, int32_t nrhs, int64_t ldb, int64_t ldx,
                     const h2s_solve_opts *opts, h2s_solve_info *info, void *stream)
{
    if (!t) return fail(H2S_ERR_INVALID_ARG, "tree is NULL");
    if (t->host_only) return fail(H2S_ERR_UNSUPPORTED, "handle was built with host_only");
    h2s_solve_opts o;
    h2s_solve_opts_default(&o);
    if (opts) o = *opts;
    const int64_t n = t->rep.n;
    if (!b || !x) return fail(H2S_ERR_INVALID_ARG, "b or x is NULL");
    if (nrhs < 1) return fail(H2S_ERR_INVALID_ARG, "nrhs must be >= 1");
    if (ldb < n || ldx < n) return fail(H2S_ERR_INVALID_ARG, "leading dimensions must be >= n");
    if (o.restart < 1 || o.restart > 1000) return fail(H2S_ERR_INVALID_ARG, "restart must be in 1..1000");
    if (o.max_iter < 0 || o.max_refine < 0) return fail(H2S_ERR_INVALID_ARG, "max_iter and max_refine must be >= 0");
    if (!(o.rtol >= 0.0) || !is_finite(o.rtol) || !(o.inner_rtol >= 0.0) || !is_finite(o.inner_rtol))
        return fail(H2S_ERR_INVALID_ARG, "rtol and inner_rtol must be finite and >= 0");
    if (low_m2l(o.inner_prec) && t->ker.kind == H2S_K_NTI_MQ)
        return fail(H2S_ERR_UNSUPPORTED, "H2S_FP32_M2L and H2S_FP32_BF16M2L are not available for the NTI multiquadric");
    if (o.inner_prec != H2S_FP64 && o.inner_prec != H2S_FP32 && o.inner_prec != H2S_FP32_M2L &&
        o.inner_prec != H2S_FP32_BF16M2L)
        return fail(H2S_ERR_INVALID_ARG, "bad inner precision");
    const char *bb = (const char *)b, *be = (const char *)(b + ldb * (nrhs - 1) + n);
    const char *xb = (const char *)x, *xe = (const char *)(x + ldx * (nrhs - 1) + n);
    if (bb < xe && xb < be) return fail(H2S_ERR_INVALID_ARG, "b and x overlap");
    if (hipSetDevice(t->device) != hipSuccess) return fail(H2S_ERR_DEVICE, "hipSetDevice failed");
    if (ensure_streams(t) != H2S_OK) return H2S_ERR_DEVICE;
    h2s_status st = ensure_uploaded(t, H2S_FP64, (hipStream_t)stream);
    if (st == H2S_OK) st = ensure_uploaded(t, o.inner_prec, (hipStream_t)stream);
    if (st != H2S_OK) return st;
    if (t->solve_m < o.restart) {
        // workspace for this restart length (a shorter restart reuses a larger one)
        Uploader up{t, (hipStream_t)stream};
        const int m = o.restart;
        h2s::SolveWork w{};
        w.V = (double *)up.raw(sizeof(double) * (size_t)n * (m + 1));
        w.w = (double *)up.raw(sizeof(double) * (size_t)n);
        w.r = (double *)up.raw(sizeof(double) * (size_t)n);
        w.y = (double *)up.raw(sizeof(double) * (size_t)n);
        w.part = (double *)up.raw(sizeof(double) * (size_t)h2s::blas_dots_blocks(n) * (m + 1));
        w.small = (double *)up.raw(sizeof(double) * (size_t)h2s::solve_small_doubles(m));
        if (up.st != H2S_OK) return up.st;
        if (hipHostMalloc((void **)&w.small_host, sizeof(double) * (size_t)h2s::solve_small_doubles(m),
                          hipHostMallocDefault) !=
            hipSuccess)
            return fail(H2S_ERR_OUT_OF_MEMORY, "pinned host allocation failed");
        if (t->work.small_host) (void)hipHostFree(t->work.small_host);
        t->work = w;
        t->solve_m = m;
    }
    // the kernels index V with ld = n; a larger workspace is used with the same n
    h2s::SolveWork w = t->work;
    const h2s::SolveParams prm{o.restart, o.max_iter, o.max_refine, o.rtol, o.inner_rtol, o.use_x0};
    SolveCtx ctx{t, o.inner_prec, stream};
    bool all = true;
    if (nrhs > 1 && t->rep.variant == H2S_H2STAR) {
        // several right-hand sides in lockstep, up to kGroupCols at a time, through the batched product
        const int cols = std::min<int32_t>(nrhs, h2s::kGroupCols), m = o.restart;
        if (t->many_m < m || t->many.cols < cols) {
            const int mm = std::max(m, t->many_m), cc = std::max(cols, t->many.cols);
            Uploader up{t, (hipStream_t)stream};
            h2s::SolveWorkMany wm{};
            wm.cols = cc;
            wm.V = up.template zeros<double>((size_t)cc * n * (mm + 1));
            wm.W = (double *)up.raw(sizeof(double) * (size_t)n * cc);
            wm.R = (double *)up.raw(sizeof(double) * (size_t)n * cc);
            wm.Y = (double *)up.raw(sizeof(double) * (size_t)n * cc);
            wm.part = (double *)up.raw(sizeof(double) * (size_t)cc * h2s::blas_dots_blocks(n) * (mm + 1));
            wm.small = (double *)up.raw(sizeof(double) * (size_t)cc * h2s::solve_small_doubles(mm));
            wm.vec = (double *)up.raw(sizeof(double) * (size_t)6 * cc);
            wm.idx = (int *)up.raw(sizeof(int) * (size_t)cc);
            if (up.st != H2S_OK) return up.st;
            if (hipHostMalloc((void **)&wm.host, sizeof(double) * (size_t)6 * cc, hipHostMallocDefault) != hipSuccess)
                return fail(H2S_ERR_OUT_OF_MEMORY, "pinned host allocation failed");
            if (hipHostMalloc((void **)&wm.host_idx, sizeof(int) * (size_t)cc, hipHostMallocDefault) != hipSuccess) {
                (void)hipHostFree(wm.host);
                return fail(H2S_ERR_OUT_OF_MEMORY, "pinned host allocation failed");
            }
            if (t->many.host) (void)hipHostFree(t->many.host);
            if (t->many.host_idx) (void)hipHostFree(t->many.host_idx);
            t->many = wm;
            t->many_m = mm;
        }
        // the kernels index V with the solve's own m: a workspace built for a larger m holds it
        const h2s::SolveOpsMany ops{&ctx, solve_apply_inner_many, solve_apply_outer_many};
        std::vector<h2s::SolveResult> rs(cols);
        for (int32_t c0 = 0; c0 < nrhs; c0 += cols) {
            const int nc = std::min<int32_t>(cols, nrhs - c0);
            const int rc = h2s::gmres_ir_many(ops, t->many, prm, n, nc, b + c0 * ldb, ldb, x + c0 * ldx, ldx, stream,
                                              rs.data());
            if (rc != 0) return fail(H2S_ERR_DEVICE, std::string("solve failed: ") + hipGetErrorString((hipError_t)rc));
            for (int c = 0; c < nc; ++c) {
                if (info) info[c0 + c] = h2s_solve_info{rs[c].iterations, rs[c].refinements, rs[c].converged, rs[c].residual};
                all = all && rs[c].converged;
            }
        }
    } else {
        const h2s::SolveOps ops{&ctx, solve_apply_inner, solve_apply_outer};
        for (int32_t c = 0; c < nrhs; ++c) {
            h2s::SolveResult r{};
            const int rc = h2s::gmres_ir(ops, w, prm, n, b + c * ldb, x + c * ldx, stream, &r);
            if (rc != 0) return fail(H2S_ERR_DEVICE, std::string("solve failed: ") + hipGetErrorString((hipError_t)rc));
            if (info) info[c] = h2s_solve_info{r.iterations, r.refinements, r.converged, r.residual};
            all = all && r.converged;
        }
    }
    if (!all) return fail(H2S_ERR_NOT_CONVERGED, "a right-hand side did not reach rtol");
    return H2S_OK;
}

h2s_status h2s_get_schedule(h2s_tree t, h2s_schedule *sc)
{
    if (!t || !sc) return fail(H2S_ERR_INVALID_ARG, "tree or schedule is NULL");
    *sc = h2s_schedule{};
    sc->near_first = t->plan.near_first;
    sc->m2l_stream = t->plan.m2l_stream;
    for (int l = 0; l <= h2s::kMaxLevels; ++l) {
        sc->up_threads[l] = t->plan.up_threads[l];
        sc->dn_threads[l] = t->plan.dn_threads[l];
    }
    return H2S_OK;
}

h2s_status h2s_set_schedule(h2s_tree t, const h2s_schedule *sc)
{
    if (!t || !sc) return fail(H2S_ERR_INVALID_ARG, "tree or schedule is NULL");
    if (!(sc->near_first >= 0.0 && sc->near_first <= 1.0))
        return fail(H2S_ERR_INVALID_ARG, "near_first must be in [0, 1]");
    if (sc->m2l_stream < 0 || sc->m2l_stream > 2) return fail(H2S_ERR_INVALID_ARG, "m2l_stream must be 0, 1 or 2");
    const int kappa = std::min(t->rep.kappa, h2s::kMaxLevels);
    auto ok = [](int32_t w) { return w >= 64 && w <= 512 && w % 64 == 0; };
    for (int l = 1; l <= kappa; ++l)
        if (!ok(sc->up_threads[l]) || (l < kappa && !ok(sc->dn_threads[l])))
            return fail(H2S_ERR_INVALID_ARG, "level " + std::to_string(l) +
                                                 ": block widths must be multiples of 64 in [64, 512]");
    t->plan.near_first = sc->near_first;
    t->plan.m2l_stream = sc->m2l_stream;
    for (int l = 1; l <= kappa; ++l) {
        t->plan.up_threads[l] = sc->up_threads[l];
        if (l < kappa) t->plan.dn_threads[l] = sc->dn_threads[l];
    }
    return H2S_OK;
}

h2s_status h2s_tune(h2s_tree t, const double *x, double *y, int32_t reps, h2s_tune_info *info, void *stream)
{
    if (!t) return fail(H2S_ERR_INVALID_ARG, "tree is NULL");
    if (t->host_only) return fail(H2S_ERR_UNSUPPORTED, "handle was built with host_only");
    if (!x || !y) return fail(H2S_ERR_INVALID_ARG, "x or y is NULL");
    const int64_t n = t->rep.n;
    if ((const char *)x < (const char *)(y + n) && (const char *)y < (const char *)(x + n))
        return fail(H2S_ERR_INVALID_ARG, "x and y overlap");
    if (reps < 1) reps = 5;
    if (hipSetDevice(t->device) != hipSuccess) return fail(H2S_ERR_DEVICE, "hipSetDevice failed");
    if (ensure_streams(t) != H2S_OK) return H2S_ERR_DEVICE;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(H2S_ERR_DEVICE, "creating the timing events failed");
    }
    h2s_tune_info res{};
    const h2s_status st = tune_plan(t, x, y, reps, (hipStream_t)stream, e0, e1, res);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == H2S_OK && info) *info = res;
    return st;
}

h2s_status h2s_group_create(const h2s_tree *trees, int32_t count, h2s_group *out)
{
    if (!out) return fail(H2S_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!trees || count < 1) return fail(H2S_ERR_INVALID_ARG, "a group needs count >= 1 trees");
    for (int32_t i = 0; i < count; ++i) {
        if (!trees[i]) return fail(H2S_ERR_INVALID_ARG, "tree " + std::to_string(i) + " is NULL");
        for (int32_t j = 0; j < i; ++j)
            if (trees[j] == trees[i]) return fail(H2S_ERR_INVALID_ARG, "a tree appears twice in the group");
    }
    for (int32_t i = 0; i < count; ++i) {
        if (trees[i]->host_only) return fail(H2S_ERR_UNSUPPORTED, "tree " + std::to_string(i) + " is host_only");
        if (trees[i]->device != trees[0]->device) return fail(H2S_ERR_INVALID_ARG, "the trees are on different devices");
    }
    if (hipSetDevice(trees[0]->device) != hipSuccess) return fail(H2S_ERR_DEVICE, "hipSetDevice failed");
    for (int32_t i = 0; i < count; ++i)
        if (ensure_streams(trees[i]) != H2S_OK) return H2S_ERR_DEVICE;
    h2s_group g = new (std::nothrow) h2s_group_s();
    if (!g) return fail(H2S_ERR_OUT_OF_MEMORY, "host allocation failed");
    g->trees.assign(trees, trees + count);
    g->device = trees[0]->device;
    g->lanes.assign(count, nullptr);
    g->done.assign(count, nullptr);
    g->graphs.assign(count, nullptr);
    g->execs.assign(count, nullptr);
    g->xs.assign(count, nullptr);
    g->ys.assign(count, nullptr);
    bool ok = hipEventCreateWithFlags(&g->start, hipEventDisableTiming) == hipSuccess &&
              hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&g->faux, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&g->ffork, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&g->fjoin, hipEventDisableTiming) == hipSuccess;
    for (int32_t i = 0; ok && i < count; ++i)
        ok = hipStreamCreateWithFlags(&g->lanes[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&g->done[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        delete g;
        return fail(H2S_ERR_DEVICE, "creating the group's streams or events failed");
    }
    // fused classes: H2* trees of one precision (FP64 / FP32), kernel function and dimension
    g->in_fused.assign(count, 0);
    for (int32_t i = 0; i < count; ++i) {
        h2s_tree t = trees[i];
        const int prec = t->opts.prec;
        if (g->in_fused[i] || t->rep.variant != H2S_H2STAR || (prec != H2S_FP64 && prec != H2S_FP32)) continue;
        h2s_group_s::Fused f;
        f.prec = prec;
        f.kind = t->ker.kind;
        f.d = t->rep.d;
        for (int32_t j = i; j < count; ++j) {
            h2s_tree u = trees[j];
            if (!g->in_fused[j] && u->rep.variant == H2S_H2STAR && (int)u->opts.prec == prec && u->ker.kind == f.kind &&
                u->rep.d == f.d)
                f.members.push_back(j);
        }
        if (f.members.size() < 2) continue;
        for (int32_t j : f.members) g->in_fused[j] = 1;
        g->fused.push_back(std::move(f));
    }
    for (h2s_group_s::Fused &f : g->fused) {
        const bool built = f.prec == H2S_FP64 ? build_multi(g, f, f.mp64, &h2s_tree_s::t64)
                                              : build_multi(g, f, f.mp32, &h2s_tree_s::t32);
        if (!built) {
            delete g;
            return fail(H2S_ERR_OUT_OF_MEMORY, "allocating the group's launch tables failed");
        }
    }
    *out = g;
    return H2S_OK;

}

h2s_status h2s_group_apply(h2s_group g, const double *const *x, double *const *y, void *stream)
{
    if (!g) return fail(H2S_ERR_INVALID_ARG, "group is NULL");
    if (!x || !y) return fail(H2S_ERR_INVALID_ARG, "x or y is NULL");
    const size_t count = g->trees.size();
    for (size_t i = 0; i < count; ++i) {
        const int64_t n = g->trees[i]->rep.n;
        if (!x[i] || !y[i]) return fail(H2S_ERR_INVALID_ARG, "x or y of tree " + std::to_string(i) + " is NULL");
        if ((const char *)x[i] < (const char *)(y[i] + n) && (const char *)y[i] < (const char *)(x[i] + n))
            return fail(H2S_ERR_INVALID_ARG, "x and y of tree " + std::to_string(i) + " overlap");
    }
    if (hipSetDevice(g->device) != hipSuccess) return fail(H2S_ERR_DEVICE, "hipSetDevice failed");
    // (re)capture the products whose vectors changed, one tree per capture
    for (size_t i = 0; i < count; ++i) {
        if (g->in_fused[i] || (g->execs[i] && g->xs[i] == x[i] && g->ys[i] == y[i])) continue;
        h2s_tree t = g->trees[i];
        g->drop_graph(i);
        if (hipStreamBeginCapture(g->cap, hipStreamCaptureModeGlobal) != hipSuccess)
            return fail(H2S_ERR_DEVICE, "hipStreamBeginCapture failed");
        const int rc = mvp(t, t->opts.prec, H2S_PHASE_ALL, x[i], y[i], g->cap, nullptr);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(g->cap, &graph);
        if (rc != 0 || ec != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(H2S_ERR_DEVICE, std::string("capturing the product of tree ") + std::to_string(i) + " failed: " +
                                            hipGetErrorString(rc != 0 ? (hipError_t)rc : ec));
        }
        g->graphs[i] = graph;
        if (hipGraphInstantiateWithFlags(&g->execs[i], graph, 0) != hipSuccess) {
            g->execs[i] = nullptr;
            g->drop_graph(i);
            return fail(H2S_ERR_DEVICE, "hipGraphInstantiateWithFlags failed");
        }
        g->xs[i] = x[i];
        g->ys[i] = y[i];
    }
    hipStream_t s = (hipStream_t)stream;
    // the fused classes' vector tables, refreshed (after the stream drains) when a pointer changed
    for (h2s_group_s::Fused &f : g->fused) {
        bool same = true;
        for (size_t k = 0; k < f.members.size(); ++k)
            same = same && f.xs[k] == x[f.members[k]] && f.ys[k] == y[f.members[k]];
        if (same) continue;
        for (size_t k = 0; k < f.members.size(); ++k) {
            f.xs[k] = x[f.members[k]];
            f.ys[k] = y[f.members[k]];
        }
        if (hipStreamSynchronize(s) != hipSuccess ||
            hipMemcpy(f.xs_dev, f.xs.data(), f.xs.size() * sizeof(void *), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(f.ys_dev, f.ys.data(), f.ys.size() * sizeof(void *), hipMemcpyHostToDevice) != hipSuccess)
            return fail(H2S_ERR_DEVICE, "updating the group's vector tables failed");
    }
    if (hipEventRecord(g->start, s) != hipSuccess) return fail(H2S_ERR_DEVICE, "hipEventRecord failed");
    for (h2s_group_s::Fused &f : g->fused) {
        const h2s::Streams st{stream, g->faux, g->ffork, nullptr, g->fjoin, nullptr, nullptr, nullptr};
        const int rc = f.prec == H2S_FP64 ? h2s::launch_multi<h2s::P64>(f.kind, f.d, f.mp64, st)
                                          : h2s::launch_multi<h2s::P32>(f.kind, f.d, f.mp32, st);
        if (rc != 0) return fail(H2S_ERR_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString((hipError_t)rc));
    }
    for (size_t i = 0; i < count; ++i) {
        if (g->in_fused[i]) continue;
        if (hipStreamWaitEvent(g->lanes[i], g->start, 0) != hipSuccess)

            return fail(H2S_ERR_DEVICE, "hipStreamWaitEvent failed");
        if (hipGraphLaunch(g->execs[i], g->lanes[i]) != hipSuccess) return fail(H2S_ERR_DEVICE, "hipGraphLaunch failed");
        if (hipEventRecord(g->done[i], g->lanes[i]) != hipSuccess || hipStreamWaitEvent(s, g->done[i], 0) != hipSuccess)
            return fail(H2S_ERR_DEVICE, "joining a tree's stream failed");
    }
    return H2S_OK;
}

h2s_status h2s_group_free(h2s_group g)
{
    if (!g) return H2S_OK;
    (void)hipSetDevice(g->device);
    delete g;
    return H2S_OK;
}

h2s_status h2s_free(h2s_tree t)
{
    if (!t) return H2S_OK;
    if (!t->host_only) (void)hipSetDevice(t->device);
    delete t;
    return H2S_OK;
}

h2s_status h2s_get_stats(h2s_tree t, h2s_stats *s)
{
    if (!t || !s) return fail(H2S_ERR_INVALID_ARG, "tree or stats is NULL");
    const h2s::HostRep &r = t->rep;
    std::memset(s, 0, sizeof(*s));
    s->d = r.d;
    s->kappa = r.kappa;
    s->variant = r.variant;
    s->prec = t->opts.prec;
    s->n = r.n;
    s->boxes = r.nbox();
    s->near_pairs = (int64_t)r.list_idx[0].size();
    s->far_pairs = (int64_t)r.list_idx[1].size();
    s->ver_pairs = (int64_t)r.list_idx[2].size();
    for (int32_t g = r.leaf0(); g < r.nbox(); ++g)
        for (int64_t e = r.list_off[0][g]; e < r.list_off[0][g + 1]; ++e) {
            const int32_t y = r.list_idx[0][e];
            s->p2p_evals += (int64_t)(r.box_end[g] - r.box_begin[g]) * (r.box_end[y] - r.box_begin[y]);
        }
    for (int f = 0; f < 2; ++f) {
        const h2s::Family &F = r.fam[f];
        std::vector<int64_t> cnt(32, 0), sum(32, 0);
        for (int32_t g = 0; g < r.nbox(); ++g) {
            const int32_t rk = F.rank[g];
            if (rk == 0) continue;
            const int l = r.level_of(g);
            s->rank_sum[f] += rk;
            if (rk > s->rank_max[f]) s->rank_max[f] = rk;
            if (l < 32) {
                if (rk > s->rank_max_level[f][l]) s->rank_max_level[f][l] = rk;
                cnt[l] += 1;
                sum[l] += rk;
            }
            const int w = f == 0 ? 1 : 2;
            for (int64_t e = r.list_off[w][g]; e < r.list_off[w][g + 1]; ++e) {
                s->m2l_evals += (int64_t)rk * F.rank[r.list_idx[w][e]];
                s->m2l_evals_family[f] += (int64_t)rk * F.rank[r.list_idx[w][e]];
            }
        }
        for (int l = 0; l < 32; ++l) s->rank_avg_level[f][l] = cnt[l] ? (double)sum[l] / cnt[l] : 0.0;
        for (int32_t g = 0; g < r.nbox(); ++g) {
            const int64_t e = (int64_t)F.op_rows[g] * F.rank[g];
            if (g >= r.leaf0()) s->leaf_basis_entries += e;
            else s->transfer_entries += e;
        }
    }
    for (const h2s::LowRankPair &P : r.pairs)
        s->pair_entries += (int64_t)P.rank *
                           ((r.box_end[P.x] - r.box_begin[P.x]) + (r.box_end[P.y] - r.box_begin[P.y]));
    s->operator_bytes = t->operator_bytes;
    s->leaf_basis_stored = t->leaf_kept[0] + t->leaf_kept[1];
    s->transfer_stored = t->transfer_kept[0] + t->transfer_kept[1];
    s->device_bytes = (int64_t)t->device_bytes;
    s->build_seconds = r.build_seconds;
    return H2S_OK;
}

h2s_status h2s_set_profiling(h2s_tree t, int32_t enable)
{
    if (!t) return fail(H2S_ERR_INVALID_ARG, "tree is NULL");
    if (t->host_only) return fail(H2S_ERR_UNSUPPORTED, "handle was built with host_only");
    t->profiling = enable != 0;
    return H2S_OK;
}

h2s_status h2s_get_profile(h2s_tree t, double *ms_total, int64_t *launches)
{
    if (!t) return fail(H2S_ERR_INVALID_ARG, "tree is NULL");
    double ms[H2S_NUM_PROF] = {0};
    int64_t cnt[H2S_NUM_PROF] = {0};
    for (auto &m : t->marks) {
        if (!m.b) continue;
        if (hipEventSynchronize(m.b) != hipSuccess) {
            t->clear_marks();
            return fail(H2S_ERR_DEVICE, "event synchronisation failed");
        }
        float e = 0.f;
        if (hipEventElapsedTime(&e, m.a, m.b) == hipSuccess) {
            ms[m.cls] += e;
            cnt[m.cls] += 1;
        }
    }
    t->clear_marks();
    for (int i = 0; i < H2S_NUM_PROF; ++i) {
        if (ms_total) ms_total[i] = ms[i];
        if (launches) launches[i] = cnt[i];
    }
    return H2S_OK;
}

h2s_status h2s_eval_rate(const h2s_kernel *k, int32_t d, int32_t prec, double *evals_per_s, void *stream)
{
    if (!k || !evals_per_s) return fail(H2S_ERR_INVALID_ARG, "kernel or output is NULL");
    if (d != 2 && d != 3) return fail(H2S_ERR_INVALID_ARG, "d must be 2 or 3");
    if (k->kind < H2S_K_LOG_R || k->kind > H2S_K_NTI_MQ) return fail(H2S_ERR_INVALID_ARG, "unknown kernel kind");
    if (k->kind == H2S_K_NTI_MQ && d != 3) return fail(H2S_ERR_INVALID_ARG, "the NTI multiquadric is 3D only");
    if (prec != H2S_FP64 && prec != H2S_FP32) return fail(H2S_ERR_INVALID_ARG, "prec must be FP64 or FP32");
    if ((k->kind == H2S_K_GAUSSIAN || k->kind == H2S_K_RBF_AR || k->kind == H2S_K_RBF_LOG) &&
        !(std::isfinite(k->param) && k->param > 0.0 && !(k->kind == H2S_K_RBF_LOG && k->param == 1.0)))
        return fail(H2S_ERR_INVALID_ARG, "kernel parameter out of range");
    hipStream_t s = (hipStream_t)stream;
    const int blocks = 8192, passes = 64;
    const std::vector<double> tab = kernel_table(k->kind);
    double kparam, kc[3];
    kernel_scalars(k->kind, k->param, kparam, kc);
    double *dtab = nullptr, *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    h2s_status st = H2S_OK;
    float best = 0.0f;
    if (hipMalloc(&dtab, tab.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&out, h2s::eval_rate_outputs(blocks) * sizeof(double)) != hipSuccess) {
        st = fail(H2S_ERR_OUT_OF_MEMORY, "device allocation failed");
    } else if (hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s) !=
                   hipSuccess ||
               hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        st = fail(H2S_ERR_DEVICE, "HIP error before the timed launches");
    } else {
        // one untimed launch, then the fastest of five
        for (int rep = 0; rep < 6 && st == H2S_OK; ++rep) {
            if (hipEventRecord(e0, s) != hipSuccess ||
                h2s::launch_eval_rate(k->kind, d, prec == H2S_FP32, blocks, dtab, kparam, kc, passes, out, s) !=
                    hipSuccess ||
                hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                st = fail(H2S_ERR_DEVICE, "evaluation-rate launch failed");
                break;
            }
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = fail(H2S_ERR_DEVICE, "event timing failed");
                break;
            }
            if (rep > 0 && (best == 0.0f || ms < best)) best = ms;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    if (dtab) (void)hipFree(dtab);
    if (st != H2S_OK) return st;
    *evals_per_s = (double)h2s::eval_rate_evals(blocks, passes) / (best * 1e-3);
    return H2S_OK;
}

h2s_status h2s_export(h2s_tree t, const char *path)
{
    if (!t || !path) return fail(H2S_ERR_INVALID_ARG, "tree or path is NULL");
    std::string err;
    const h2s_status st = h2s::export_host(t->rep, path, err);
    if (st != H2S_OK) return fail(st, err);
    return H2S_OK;
}

} // extern "C"
