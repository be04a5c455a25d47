// h2s_kernels.hip -- HIP kernels of the H2* / (H2+H)* matrix-vector product
// for CDNA4 (gfx950), Khan & Ambikasaran (arXiv 2309.14085), Sec. 5.1.2 and
// Sec. 5.2.2:
//
//   k_permute    charges to tree order         q = x[perm]
//   k_p2p        direct near field             yn_X = sum_{X' in N*(X)} K(X, X') q_X'
//   k_up_leaf    P2M                           v_X = U_X^T q_X            (both families)
//   k_m2m        one level of M2M              v_X = sum_c U~_{X_c X}^T v_{X_c}
//   k_m2l_slices all levels of one family      u_X = sum_{Y in IL(X)} K(t^{X,i}, t^{Y,i}) v_Y
//   k_m2l        the same with a float far field (FP32_M2L)
//   k_l2l        one level of L2L              u_{X_c} += U~_{X_c X} u_X
//   k_pair_part  (H2+H)*: partial products Vb^T q_Y, Ub^T q_X over row chunks
//   k_pair_sum   (H2+H)*: chunk sums in a fixed order
//   k_down_leaf  yn + shift q + L2P U_X u_X + (H2+H)* vertex blocks,
//                scattered back to user order
//
// k_p2p needs only the permuted charges, so it runs on a second stream while
// the main stream goes up and down the tree; k_down_leaf joins the two
// (under the profiling hook everything runs on the main stream, one class
// at a time).
//
// Accuracy of the sums.  The interpolative NCA operators have norms up to
// ~1e3 - 1e4 on coarse levels, so a rounding error in a multipole or local
// coefficient is amplified on its way to the potential.  In FP64 the sums of
// the transfers (P2M, M2M, L2L, L2P) are accurate dot products (Ogita, Rump
// and Oishi, "Accurate sum and dot product", 2005): the sum as if taken in
// twice the precision, rounded once, whatever the order of its terms.  So is
// the vertex-field M2L, whose T2B coefficients carry the largest
// amplification (with plain sums there, the product moved from the oracle's
// by up to 1e-12 at N = 2^17 in 2D), and its kernel values come from log r
// rounded about once.  The far-field M2L sums its terms with fused
// multiply-adds over slices of the list, of kernel values from the one-ulp
// log (it moves the product by about 1e-13 at N = 2^20 in 2D), which saves
// about 13 instructions and one table read per evaluation.  The direct near
// field is a plain sum of kernel values (nothing amplifies it).  No floating-point
// atomics are used; results are bitwise reproducible run to run.
//
// M2L and the near field evaluate the kernel on the fly from coordinates
// staged in LDS; the GEMV-shaped steps are HBM-bound and read each operator
// once, coalesced, from the copy laid out for them.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "h2s.h"
#include "h2s_device.hpp"
#include "h2s_kfun.hpp"

namespace h2s {

namespace {

// ---------------------------------------------------------------------------
// P2M, M2M, L2L: one output per thread, terms in index order.  Blocks are
// sized per level by the host to cover the outputs of a box (both families)
// in one pass.
// ---------------------------------------------------------------------------
constexpr int NT_GEMV_MAX = 512;
constexpr int GEMV_WAVES = 8; // waves per SIMD asked of the compiler (bytes in flight)
constexpr int LEAF_WAVES = 6; // the same for L2L's leaf-level partner, k_down_leaf (more live state)

// Charges to tree order: qt[i] = x[perm[i]], 256 per block.
template <class P> __device__ __forceinline__ void permute_body(const DevTree<P> &t, const double *__restrict__ x, int blk)
{
    const int i = blk * 256 + threadIdx.x;
    if (i < t.n) t.qt[i] = x[t.perm[i]];
}

template <class P> __global__ __launch_bounds__(256) void k_permute(DevTree<P> t, const double *__restrict__ x)
{
    permute_body(t, x, blockIdx.x);
}

template <class P> __device__ __forceinline__ void up_leaf_body(const DevTree<P> &t, int leaf, uint32_t mask)
{
    extern __shared__ double qs[]; // the kept rows' charges: far family, then vertex family
    const int g = t.leaf0 + leaf, tid = threadIdx.x, nt = blockDim.x;
    const int b = t.box_begin[g], n = t.box_end[g] - b;
    const int cf = t.far.coef_off[g], rf = (mask & kFar) && t.kappa >= t.far.lmin ? t.far.coef_off[g + 1] - cf : 0;
    const int cv = t.ver.coef_off[g], rv = (mask & kVer) && t.kappa >= t.ver.lmin ? t.ver.coef_off[g + 1] - cv : 0;
    const int nkf = rf ? t.far.unk[leaf] : 0, nkv = rv ? t.ver.unk[leaf] : 0;
    double *const qv = qs + nkf;
    for (int j = tid; j < nkf; j += nt) qs[j] = t.qt[b + t.far.ukeep[b + j]];
    for (int j = tid; j < nkv; j += nt) qv[j] = t.qt[b + t.ver.ukeep[b + j]];
    __syncthreads();
    // one column of the two families per thread (kept rows of U row-major: column k strided by r);
    // the column's unit row adds the pivot's charge where its row lies among the kept rows, so the
    // sum is the one over all rows in index order
    for (int k = tid; k < rf + rv; k += nt) {
        const bool f = k < rf;
        const int kk = f ? k : k - rf;
        const auto *A = f ? t.far.U_rm + t.far.uoff[leaf] + kk : t.ver.U_rm + t.ver.uoff[leaf] + kk;
        const int pr = f ? t.far.uprow[cf + kk] : t.ver.uprow[cv + kk];
        const int pos = pr < 0 ? -1 : f ? t.far.upos[cf + kk] : t.ver.upos[cv + kk];
        double *out = f ? t.far.v + cf + kk : t.ver.v + cv + kk;
        *out = ordered_dot<P::ordered>(A, (size_t)(f ? rf : rv), f ? nkf : nkv, f ? qs : qv, pos, pr < 0 ? 0.0 : t.qt[b + pr]);
    }
}

template <class P> __global__ __launch_bounds__(NT_GEMV_MAX, GEMV_WAVES) void k_up_leaf(DevTree<P> t, uint32_t mask)
{
    up_leaf_body(t, xcd_remap(blockIdx.x, gridDim.x), mask);
}

template <class P> __device__ __forceinline__ void m2m_body(const DevTree<P> &t, int g, uint32_t mask)
{
    extern __shared__ double xs[]; // both families' child coefficients of the kept transfer rows
    const int tid = threadIdx.x, nt = blockDim.x;
    const auto &Fa = t.far;
    const auto &Ve = t.ver;
    const int cf = Fa.coef_off[g], rf = (mask & kFar) ? Fa.coef_off[g + 1] - cf : 0;
    const int cv = Ve.coef_off[g], rv = (mask & kVer) ? Ve.coef_off[g + 1] - cv : 0;
    const int bf = Fa.coef_off[t.box_cbeg[g]], nkf = rf ? Fa.tnk[g] : 0;
    const int bv = Ve.coef_off[t.box_cbeg[g]], nkv = rv ? Ve.tnk[g] : 0;
    for (int j = tid; j < nkf; j += nt) xs[j] = Fa.v[bf + Fa.tkeep[bf + j]];
    for (int j = tid; j < nkv; j += nt) xs[nkf + j] = Ve.v[bv + Ve.tkeep[bv + j]];
    __syncthreads();
    // kept rows of the stacked transfer row-major: column k strided by r; the column's unit row
    // adds its child coefficient where the row lies among the kept rows (the full row order)
    for (int k = tid; k < rf + rv; k += nt) {
        const bool f = k < rf;
        const int kk = f ? k : k - rf;
        const double *A = f ? Fa.Tr_rm + Fa.troff[g] + kk : Ve.Tr_rm + Ve.troff[g] + kk;
        const int pr = f ? Fa.tprow[cf + kk] : Ve.tprow[cv + kk];
        const int pos = pr < 0 ? -1 : f ? Fa.tpos[cf + kk] : Ve.tpos[cv + kk];
        const double qp = pr < 0 ? 0.0 : f ? Fa.v[bf + pr] : Ve.v[bv + pr];
        double *out = f ? Fa.v + cf + kk : Ve.v + cv + kk;
        *out = ordered_dot<P::ordered>(A, (size_t)(f ? rf : rv), f ? nkf : nkv, f ? xs : xs + nkf, pos, qp);
    }
}

template <class P> __global__ __launch_bounds__(NT_GEMV_MAX, GEMV_WAVES) void k_m2m(DevTree<P> t, int32_t g0, uint32_t mask)
{
    m2m_body(t, g0 + (int)blockIdx.x, mask);
}

template <class P> __device__ __forceinline__ void l2l_body(const DevTree<P> &t, int g, uint32_t mask)
{
    extern __shared__ double xs[]; // both families' parent locals
    constexpr bool ORD = P::ordered;
    const int tid = threadIdx.x, nt = blockDim.x;
    const auto &Fa = t.far;
    const auto &Ve = t.ver;
    const int cf = Fa.coef_off[g], rf = (mask & kFar) ? Fa.coef_off[g + 1] - cf : 0;
    const int cv = Ve.coef_off[g], rv = (mask & kVer) ? Ve.coef_off[g + 1] - cv : 0;
    const int bf = Fa.coef_off[t.box_cbeg[g]], Rf = rf ? Fa.coef_off[t.box_cend[g]] - bf : 0;
    const int bv = Ve.coef_off[t.box_cbeg[g]], Rv = rv ? Ve.coef_off[t.box_cend[g]] - bv : 0;
    for (int k = tid; k < rf; k += nt) xs[k] = Fa.u[cf + k];
    for (int k = tid; k < rv; k += nt) xs[rf + k] = Ve.u[cv + k];
    __syncthreads();
    // kept rows of the stacked transfer column-major (row j strided by the kept-row count); a
    // unit row e_a gives the local a itself
    const int nkf = rf ? Fa.tnk[g] : 0, nkv = rv ? Ve.tnk[g] : 0;
    for (int j = tid; j < Rf + Rv; j += nt) {
        const bool f = j < Rf;
        const int jj = f ? j : j - Rf;
        const int kj = f ? Fa.trow[bf + jj] : Ve.trow[bv + jj];
        const double *A = (f ? Fa.Tr_cm + Fa.troff[g] : Ve.Tr_cm + Ve.troff[g]) + (kj >= 0 ? kj : 0);
        const double *x = f ? xs : xs + rf;
        double *out = f ? Fa.u + bf + jj : Ve.u + bv + jj;
        // the parent's contribution added to the child's M2L result inside the one sum
        *out = kj >= 0 ? ordered_dot<ORD>(A, (size_t)(f ? nkf : nkv), f ? rf : rv, x, -1, 0.0, *out) : *out + x[~kj];
    }
}

template <class P> __global__ __launch_bounds__(NT_GEMV_MAX, GEMV_WAVES) void k_l2l(DevTree<P> t, int32_t g0, uint32_t mask)
{
    l2l_body(t, g0 + (int)blockIdx.x, mask);
}

// ---------------------------------------------------------------------------
// M2L: one target box per block.  Work item (a, Y): pivot a of X against
// source box Y, s_{aY} = sum_b K(t^{X,i}_a, t^{Y,i}_b) v_Y[b] in b order;
// then u_X[a] = sum_Y s_{aY} in list order.  Sources are staged in LDS a
// group of whole boxes at a time.  X and Y are distinct boxes of one level,
// and coincident points always fall in the same box, so r^2 > 0 here.
// ---------------------------------------------------------------------------
constexpr int NT_M2L = 128;
constexpr int M2L_SRC = 512;   // staged pivots per group (>= the largest rank)
constexpr int M2L_PART = 1024; // partial sums s_{aY} per group (>= 2 x the largest rank)
constexpr int M2L_BOX = 64;    // source boxes per group
constexpr int M2L_OWN = 4;     // targets per thread: rank <= NT_M2L * M2L_OWN

// In the FP32-M2L policy the far family uses float box-centred coordinates
// and, for log r, K = 0.5 log|c|^2 + 0.5 log(r^2 / |c|^2) with c the
// difference of the two box centres: the first term is taken in double once
// per source box, the second in float.
template <class P, bool FAR, int KIND, int D>
__global__ __launch_bounds__(NT_M2L) void k_m2l(DevTree<P> t, int32_t t0)
{
    constexpr bool LOWP = FAR && sizeof(typename P::far_t) == 4;
    using CT = std::conditional_t<LOWP, float, double>;
    constexpr bool CENTRED = LOWP && KIND == H2S_K_LOG_R;
    constexpr bool ORD = P::ordered;
    const auto &F = [&]() -> const auto & {
        if constexpr (FAR) return t.far;
        else return t.ver;
    }();
    __shared__ CT sx[M2L_SRC], sy[M2L_SRC], sz[D == 3 ? M2L_SRC : 1];
    __shared__ double sv[M2L_SRC];
    __shared__ double part[M2L_PART];
    __shared__ int ybeg[M2L_BOX], ylen[M2L_BOX];
    __shared__ double ylc[CENTRED ? M2L_BOX : 1];
    __shared__ float yic[CENTRED ? M2L_BOX : 1];
    __shared__ __align__(16) double ktab[kTabLen<KIND>];
    const int tid = threadIdx.x;
    if constexpr (!LOWP) stage_table<KIND>(t.ktab, ktab);
    const int g = F.targets[t0 + xcd_chunk_remap<kM2LChunk>(blockIdx.x, gridDim.x)]; // targets t0 .. t0 + gridDim.x - 1
    const int c0 = F.coef_off[g], r = F.coef_off[g + 1] - c0;
    const int e0 = F.il_off[g], e1 = F.il_off[g + 1];
    const CT diag = (CT)t.diag;
    const KPar<CT> kp = kpar<CT>(t);
    const KPar<double> kpd = kpar<double>(t);
    const double *cX = t.box_ctr + 3 * g;
    double uacc[M2L_OWN];
#pragma unroll
    for (int o = 0; o < M2L_OWN; ++o) uacc[o] = 0.0;
    int e = e0;
    while (e < e1) {
        // stage a group of whole source boxes (the loop bounds are uniform)
        int pos = 0, ny = 0;
        while (e < e1 && ny < M2L_BOX && (ny + 1) * r <= M2L_PART) {
            const int y = F.il_idx[e];
            const int cy = F.coef_off[y], ry = F.coef_off[y + 1] - cy;
            if (pos + ry > M2L_SRC) break;
            double dcx = 0, dcy = 0, dcz = 0;
            if constexpr (LOWP) {
                dcx = t.box_ctr[3 * y] - cX[0];
                dcy = t.box_ctr[3 * y + 1] - cX[1];
                dcz = t.box_ctr[3 * y + 2] - cX[2];
            }
            for (int j = tid; j < ry; j += NT_M2L) {
                if constexpr (LOWP) {
                    sx[pos + j] = (CT)(dcx + (double)F.pvx[cy + j]);
                    sy[pos + j] = (CT)(dcy + (double)F.pvy[cy + j]);
                    if constexpr (D == 3) sz[pos + j] = (CT)(dcz + (double)F.pvz[cy + j]);
                } else {
                    sx[pos + j] = F.pvx[cy + j];
                    sy[pos + j] = F.pvy[cy + j];
                    if constexpr (D == 3) sz[pos + j] = F.pvz[cy + j];
                }
                sv[pos + j] = F.v[cy + j];
            }
            if (tid == 0) {
                ybeg[ny] = pos;
                ylen[ny] = ry;
                if constexpr (CENTRED) {
                    const double c2 = dcx * dcx + dcy * dcy + dcz * dcz;
                    ylc[ny] = 0.5 * log(c2);
                    yic[ny] = (float)(1.0 / c2);
                }
            }
            pos += ry;
            ++ny;
            ++e;
        }
        __syncthreads();
        // partial sums s_{aY}, one work item per (target, source box)
        for (int w = tid; w < r * ny; w += NT_M2L) {
            const int a = w % r, yl = w / r;
            const CT xa = (CT)F.pvx[c0 + a], ya = (CT)F.pvy[c0 + a], za = D == 3 ? (CT)F.pvz[c0 + a] : CT(0);
            const int jb = ybeg[yl], je = jb + ylen[yl];
            double s = 0.0;
            if constexpr (CENTRED) {
                const float ic = yic[yl];
                float sf = 0.f;
                double vs = 0.0;
                for (int j = jb; j < je; ++j) {
                    const float r2 = dist2<false, D>(xa - sx[j], ya - sy[j], za - sz[D == 3 ? j : 0]);
                    sf += __log2f(r2 * ic) * 0.34657359027997264f * (float)sv[j];
                    vs += sv[j];
                }
                s = (double)sf + ylc[yl] * vs;
            } else if constexpr (LOWP) {
                float sf = 0.f;
                for (int j = jb; j < je; ++j) {
                    const float r2 = dist2<false, D>(xa - sx[j], ya - sy[j], za - sz[D == 3 ? j : 0]);
                    sf += kval<KIND>(r2, diag, kp) * (float)sv[j];
                }
                s = (double)sf;
            } else {
                int j = jb;
                for (; j + 4 <= je; j += 4) {
                    double kv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const double r2 = dist2<ORD, D>((double)xa - (double)sx[j + u], (double)ya - (double)sy[j + u],
                                                        D == 3 ? (double)za - (double)sz[j + u] : 0.0);
                        kv[u] = kval_pos<KIND>(r2, kpd, ktab);
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) s = madd<ORD>(s, kv[u], sv[j + u]);
                }
                for (; j < je; ++j) {
                    const double r2 = dist2<ORD, D>((double)xa - (double)sx[j], (double)ya - (double)sy[j],
                                                    D == 3 ? (double)za - (double)sz[j] : 0.0);
                    s = madd<ORD>(s, kval_pos<KIND>(r2, kpd, ktab), sv[j]);
                }
            }
            part[yl * r + a] = s;
        }
        __syncthreads();
        // u[a] += s_{aY} in list order
#pragma unroll
        for (int o = 0; o < M2L_OWN; ++o) {
            const int a = tid + o * NT_M2L;
            if (a < r)
                for (int yl = 0; yl < ny; ++yl)
                    uacc[o] = uacc[o] + part[yl * r + a];
        }
        __syncthreads();
    }
#pragma unroll
    for (int o = 0; o < M2L_OWN; ++o) {
        const int a = tid + o * NT_M2L;
        if (a < r) F.u[c0 + a] = uacc[o];
    }
}

// ---------------------------------------------------------------------------
// M2L in double, slice form: one target box X per block.  The pivots and
// multipoles of every box of IL(X) are staged in LDS (a group at a time) and
// split into source slices; each thread takes two target pivots (a and
// a + NP) against one slice, so every staged source serves two evaluations.
// u_X[a] = sum over slices (in slice order) of the slice's partial sums.
// X and its list boxes are distinct boxes of one level, so r^2 > 0.
// Each slice keeps two partial sums per target (even and odd sources of the
// slice), added after each staged group; the slices are added in slice order.
// Far field: chains of fused multiply-adds.  FP64 vertex field (FAR false,
// P::ordered): every partial sum is an accurate dot product kept as an
// unevaluated pair (hi, lo) (dot2_add), the pairs are added with dd_add and
// the result is rounded once, so u_X[a] is the sum over the whole list as if
// taken in twice the precision, of kernel values from the log rounded about
// once.
// ---------------------------------------------------------------------------
// block width and staged source pivots per group of k_m2l_slices / km_m2l, per family
constexpr int kM2LFarNT = 256, kM2LFarSRC = 512, kM2LVerNT = 256, kM2LVerSRC = 512;

template <class P, bool FAR, int KIND, int D, int NT, int SRC>
__device__ __forceinline__ void m2l_slices_body(const DevTree<P> &t, int ti)
{
    const auto &F = [&]() -> const auto & {
        if constexpr (FAR) return t.far;
        else return t.ver;
    }();
    constexpr bool XW = kExtraCoord<KIND>;
    // FP64 vertex field: accurate (hi, lo) sums of kernel values from log r rounded about once
    constexpr bool ACC = P::ordered && !FAR, ACC_SUM = ACC;
    constexpr int TL = ACC ? kTabLenAcc<KIND> : kTabLen<KIND>;
    // staged sources (x, y, v[, z][, w]); after the last group the same memory holds the slice partials
    constexpr int NSRC = (3 + (D == 3) + XW) * SRC;
    static_assert(NSRC >= 4 * NT, "the slice partials fit in the staging buffer");
    __shared__ double sbuf[NSRC];
    double *const sx = sbuf, *const sy = sx + SRC, *const sv = sy + SRC;
    double *const sz = sv + SRC;                 // used in 3D only
    double *const sw = sz + (D == 3 ? SRC : 0); // used by kernels of an extra coordinate only
    double *const red = sbuf;
    __shared__ int32_t boxoff[kMaxList], boxcoef[kMaxList], wsum[NT / 64];
    __shared__ __align__(16) double ktab[TL];
    const int tid = threadIdx.x;
    stage_table<KIND, TL>(t.ktab, ktab); // first used after a barrier
    const int g = F.targets[ti];
    const int c0 = F.coef_off[g], r = F.coef_off[g + 1] - c0;
    const int e0 = F.il_off[g], nil = F.il_off[g + 1] - e0; // nil <= kMaxList (checked at build)
    const KPar<double> kp = kpar<double>(t);
    // the sources of IL(X) in list order as slots 0 .. S-1: slot s lies in list box e with
    // boxoff[e] <= s < boxoff[e + 1], coefficient boxcoef[e] + s - boxoff[e].  A group of
    // SRC slots is staged with all its loads in flight at once.
    int S = 0;
    for (int eb = 0; eb < nil; eb += NT) { // NT list boxes at a time
        const int e = eb + tid;
        int cb = 0, nb = 0;
        if (e < nil) {
            const int y = F.il_idx[e0 + e];
            cb = F.coef_off[y];
            nb = F.coef_off[y + 1] - cb;
        }
        int tot;
        const int off = block_excl_scan<NT>(nb, wsum, tot);
        if (e < nil) {
            boxcoef[e] = cb;
            boxoff[e] = S + off;
        }
        S += tot;
        __syncthreads();
    }
    auto coef_of = [&](int sl) -> int {
        int lo = 0, hi = nil - 1; // largest e with boxoff[e] <= sl
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (boxoff[mid] <= sl) lo = mid;
            else hi = mid - 1;
        }
        return boxcoef[lo] + (sl - boxoff[lo]);
    };
    for (int a0 = 0; a0 < r; a0 += 2 * NT) {
        const int MT = min(r - a0, 2 * NT), NP = (MT + 1) / 2, NS = NT / NP;
        const int s = tid / NP, pa = tid % NP;
        const int ia = a0 + pa, ib = pa + NP < MT ? ia + NP : ia; // a lone last target is paired with itself
        const double xa = F.pvx[c0 + ia], ya = F.pvy[c0 + ia], za = D == 3 ? (double)F.pvz[c0 + ia] : 0.0;
        const double xb = F.pvx[c0 + ib], yb = F.pvy[c0 + ib], zb = D == 3 ? (double)F.pvz[c0 + ib] : 0.0;
        const double wa = XW ? (double)F.pvw[c0 + ia] : 0.0, wb = XW ? (double)F.pvw[c0 + ib] : 0.0;
        double acc_a = 0.0, acc_b = 0.0, lo_a = 0.0, lo_b = 0.0;
        int pos = 0;
        auto kv = [&](double x, double y, double z, double w, double x0, double y0, double z0, double w0) {
            return kval_pos<KIND, ACC>(add_extra<KIND>(dist2<false, D>(x - x0, y - y0, z - z0), w, w0), kp, ktab);
        };
        auto flush = [&]() {
            __syncthreads();
            if (ACC_SUM && s < NS) {
                // two independent (hi, lo) pairs per target keep two addition chains in flight
                double a0s = 0, a0c = 0, a1s = 0, a1c = 0, b0s = 0, b0c = 0, b1s = 0, b1c = 0;
                int j = s;
                for (; j + NS < pos; j += 2 * NS) {
                    const int j1 = j + NS;
                    const double x0 = sx[j], y0 = sy[j], z0 = D == 3 ? sz[j] : 0.0, v0 = sv[j];
                    const double x1 = sx[j1], y1 = sy[j1], z1 = D == 3 ? sz[j1] : 0.0, v1 = sv[j1];
                    const double w0 = XW ? sw[j] : 0.0, w1 = XW ? sw[j1] : 0.0;
                    dot2_add(a0s, a0c, kv(xa, ya, za, wa, x0, y0, z0, w0), v0);
                    dot2_add(b0s, b0c, kv(xb, yb, zb, wb, x0, y0, z0, w0), v0);
                    dot2_add(a1s, a1c, kv(xa, ya, za, wa, x1, y1, z1, w1), v1);
                    dot2_add(b1s, b1c, kv(xb, yb, zb, wb, x1, y1, z1, w1), v1);
                }
                if (j < pos) {
                    const double x0 = sx[j], y0 = sy[j], z0 = D == 3 ? sz[j] : 0.0, v0 = sv[j];
                    const double w0 = XW ? sw[j] : 0.0;
                    dot2_add(a0s, a0c, kv(xa, ya, za, wa, x0, y0, z0, w0), v0);
                    dot2_add(b0s, b0c, kv(xb, yb, zb, wb, x0, y0, z0, w0), v0);
                }
                dd_add(acc_a, lo_a, a0s, a0c);
                dd_add(acc_a, lo_a, a1s, a1c);
                dd_add(acc_b, lo_b, b0s, b0c);
                dd_add(acc_b, lo_b, b1s, b1c);
            } else if (s < NS) {
                double a0s = 0, a1s = 0, b0s = 0, b1s = 0;
                int j = s;
                for (; j + NS < pos; j += 2 * NS) {
                    const int j1 = j + NS;
                    const double x0 = sx[j], y0 = sy[j], z0 = D == 3 ? sz[j] : 0.0, v0 = sv[j];
                    const double x1 = sx[j1], y1 = sy[j1], z1 = D == 3 ? sz[j1] : 0.0, v1 = sv[j1];
                    const double w0 = XW ? sw[j] : 0.0, w1 = XW ? sw[j1] : 0.0;
                    a0s = fma(kv(xa, ya, za, wa, x0, y0, z0, w0), v0, a0s);
                    b0s = fma(kv(xb, yb, zb, wb, x0, y0, z0, w0), v0, b0s);
                    a1s = fma(kv(xa, ya, za, wa, x1, y1, z1, w1), v1, a1s);
                    b1s = fma(kv(xb, yb, zb, wb, x1, y1, z1, w1), v1, b1s);
                }
                if (j < pos) {
                    const double x0 = sx[j], y0 = sy[j], z0 = D == 3 ? sz[j] : 0.0, v0 = sv[j];
                    const double w0 = XW ? sw[j] : 0.0;
                    a0s = fma(kv(xa, ya, za, wa, x0, y0, z0, w0), v0, a0s);
                    b0s = fma(kv(xb, yb, zb, wb, x0, y0, z0, w0), v0, b0s);
                }
                acc_a += a0s + a1s;
                acc_b += b0s + b1s;
            }
            __syncthreads();
            pos = 0;
        };
        for (int base = 0; base < S; base += SRC) {
            const int take = min(S - base, SRC);
            for (int j = tid; j < take; j += NT) {
                const int c = coef_of(base + j);
                sx[j] = F.pvx[c];
                sy[j] = F.pvy[c];
                if constexpr (D == 3) sz[j] = F.pvz[c];
                if constexpr (XW) sw[j] = F.pvw[c];
                sv[j] = F.v[c];
            }
            pos = take;
            flush();
        }
        red[tid] = s < NS ? acc_a : 0.0;
        red[NT + tid] = s < NS ? acc_b : 0.0;
        if constexpr (ACC_SUM) {
            red[2 * NT + tid] = s < NS ? lo_a : 0.0;
            red[3 * NT + tid] = s < NS ? lo_b : 0.0;
        }
        __syncthreads();
        if (tid < NP) {
            double ua = 0.0, ub = 0.0, uac = 0.0, ubc = 0.0;
            for (int q = 0; q < NS; ++q) {
                if constexpr (ACC_SUM) {
                    dd_add(ua, uac, red[q * NP + tid], red[2 * NT + q * NP + tid]);
                    dd_add(ub, ubc, red[NT + q * NP + tid], red[3 * NT + q * NP + tid]);
                } else {
                    ua += red[q * NP + tid];
                    ub += red[NT + q * NP + tid];
                }
            }
            F.u[c0 + ia] = ua + uac;
            if (ib != ia) F.u[c0 + ib] = ub + ubc;
        }
        __syncthreads();
    }
}

// targets t0 .. t0 + gridDim.x - 1 of the family.  The 2D far field (fused sums, the one-ulp log,
// 18 KB of LDS) fits 8 blocks per CU in 64 registers; elsewhere LDS or registers allow about 6.
template <class P, bool FAR, int KIND, int D, int NT, int SRC>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(FAR && D == 2 ? 8 : 6))) void k_m2l_slices(DevTree<P> t,
                                                                                                            int32_t t0)
{
    m2l_slices_body<P, FAR, KIND, D, NT, SRC>(t, t0 + xcd_chunk_remap<kM2LChunk>(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// (H2+H)*: partial sums over one row chunk of G^T q, G = Vb over the rows of
// Y (side 0: w = Vb^T q_Y) or Ub over the rows of X (side 1: w' = Ub^T q_X).
// ---------------------------------------------------------------------------
template <class P> __global__ __launch_bounds__(256) void k_pair_part(DevTree<P> t)
{
    __shared__ double qs[2048]; // rows per chunk, set when the chunks are laid out
    const auto &Pr = t.pairs;
    const int c = blockIdx.x;
    const int p = Pr.chunk_pair[c], side = Pr.chunk_side[c];
    const int r = Pr.prank[p];
    const int box = side == 0 ? Pr.py[p] : Pr.px[p];
    const int nrows = t.box_end[box] - t.box_begin[box];
    const int r0 = Pr.chunk_begin[c], len = Pr.chunk_len[c];
    const double *q = t.qt + t.box_begin[box] + r0;
    for (int i = threadIdx.x; i < len; i += 256) qs[i] = q[i];
    __syncthreads();
    const auto *G = Pr.data + (side == 0 ? Pr.pv[p] : Pr.pu[p]) + r0; // column k contiguous over the rows
    double *out = Pr.partial + Pr.chunk_poff[c];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k = wave; k < r; k += 4) {
        double acc = 0.0;
        for (int i = lane; i < len; i += 64) acc += (double)G[(size_t)k * nrows + i] * qs[i];
        acc = wave_sum(acc);
        if (lane == 0) out[k] = acc;
    }
}

template <class P> __global__ __launch_bounds__(64) void k_pair_sum(DevTree<P> t)
{
    const auto &Pr = t.pairs;
    const int ps = blockIdx.x, p = ps >> 1, side = ps & 1;
    const int r = Pr.prank[p];
    const int c0 = Pr.side_chunk_off[ps], c1 = Pr.side_chunk_off[ps + 1];
    double *w = Pr.w + Pr.pw[p] + (size_t)side * r;
    for (int k = threadIdx.x; k < r; k += 64) {
        double s = 0.0;
        for (int c = c0; c < c1; ++c) s += Pr.partial[Pr.chunk_poff[c] + k];
        w[k] = s;
    }
}

// ---------------------------------------------------------------------------
// Near field: one target leaf per block, its near list N*(X) staged in LDS;
// yn[i] = sum_{j in N*(X)} K(x_i, x_j) q_j.  Each thread takes P2P_TPT
// targets (a, a + NP, a + 2 NP, ...) against one slice of the staged
// sources, so every source it reads from LDS serves P2P_TPT evaluations:
// the staged sources and the kernel-table gathers share the LDS bandwidth.
// ---------------------------------------------------------------------------
constexpr int NT_P2P = 256;
constexpr int P2P_SRC = 1024;     // staged source points per group
constexpr int P2P_TPT = 4;        // targets per thread

template <class P, int KIND, int D> __device__ __forceinline__ void p2p_body(const DevTree<P> &t, int leaf)
{
    using PT = typename P::pt_t;
    constexpr bool TAB = sizeof(PT) == 8;
    constexpr int TPT = P2P_TPT;
    constexpr bool XW = kExtraCoord<KIND>;
    // staged sources (x, y, q[, z][, w]); after the last group the same memory holds the slice partials
    constexpr size_t SRC_BYTES = (size_t)(3 + (D == 3) + XW) * P2P_SRC * sizeof(PT);
    constexpr size_t RED_BYTES = (size_t)TPT * NT_P2P * sizeof(double);
    __shared__ __align__(16) unsigned char sbuf[SRC_BYTES > RED_BYTES ? SRC_BYTES : RED_BYTES];
    PT *const sx = reinterpret_cast<PT *>(sbuf), *const sy = sx + P2P_SRC, *const sq = sy + P2P_SRC;
    PT *const sz = sq + P2P_SRC;                      // used in 3D only
    PT *const sw = sz + (D == 3 ? P2P_SRC : 0);       // used by kernels of an extra coordinate only
    double *const red = reinterpret_cast<double *>(sbuf);
    __shared__ __align__(16) double ktab[TAB ? kTabLen<KIND> : 2];
    // the near list's points in list order as slots 0 .. S-1: slot s lies in list box e with
    // nboff[e] <= s < nboff[e + 1], point nbbeg[e] + s - nboff[e]; nself = the leaf's own entry
    __shared__ int32_t nboff[kMaxList + 1], nbbeg[kMaxList], nself;
    const int tid = threadIdx.x;
    const PT diag = (PT)t.diag;
    const KPar<PT> kp = kpar<PT>(t);
    if constexpr (TAB) stage_table<KIND>(t.ktab, ktab); // first used after a barrier
    {
        const int g = t.leaf0 + leaf;
        const int b = t.box_begin[g], n = t.box_end[g] - b;
        const double *cX = t.box_ctr + 3 * g;
        const int ne0 = t.near_off[leaf], nne = t.near_off[leaf + 1] - ne0; // nne <= kMaxList (checked at build)
        for (int k = tid; k < nne; k += NT_P2P) {
            const int gs = t.leaf0 + t.near_idx[ne0 + k];
            nbbeg[k] = t.box_begin[gs];
            nboff[k + 1] = t.box_end[gs] - t.box_begin[gs];
        }
        __syncthreads();
        if (tid == 0) {
            nboff[0] = 0;
            nself = -1;
            for (int k = 0; k < nne; ++k) {
                nboff[k + 1] += nboff[k];
                if (t.leaf0 + t.near_idx[ne0 + k] == g) nself = k;
            }
        }
        __syncthreads();
        const int S = nboff[nne];
        auto box_of = [&](int sl) -> int {
            int lo = 0, hi = nne - 1; // largest e with nboff[e] <= sl
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (nboff[mid] <= sl) lo = mid;
                else hi = mid - 1;
            }
            return lo;
        };
        for (int i0 = 0; i0 < n; i0 += TPT * NT_P2P) {
            // MT targets this pass in NP groups (a, a + NP, ...); NS source slices
            const int MT = min(n - i0, TPT * NT_P2P), NP = (MT + TPT - 1) / TPT, NS = NT_P2P / NP;
            const int s = tid / NP, pa = tid % NP;
            int it[TPT];
            PT tx[TPT], ty[TPT], tz[TPT], tw[TPT];
            double acc[TPT];
#pragma unroll
            for (int k = 0; k < TPT; ++k) {
                it[k] = pa + k * NP < MT ? i0 + pa + k * NP : i0 + pa; // a missing target repeats the first
                tx[k] = t.px[b + it[k]];
                ty[k] = t.py[b + it[k]];
                tz[k] = D == 3 ? t.pz[b + it[k]] : PT(0);
                tw[k] = XW ? t.pw[b + it[k]] : PT(0);
                acc[k] = 0.0;
            }
            int pos = 0, self0 = 0, self1 = 0; // staged positions of the target leaf's own points
            // slice s takes the staged sources jb + s, jb + s + NS, ... below je
            auto slice_sum = [&](int jb, int je, auto check) {
                constexpr bool CHECK = decltype(check)::value;
                auto kv = [&](PT r2) -> PT {
                    if constexpr (sizeof(PT) == 8) {
                        if constexpr (CHECK) return kval<KIND>(r2, diag, kp, ktab);
                        else return kval_pos<KIND>(r2, kp, ktab);
                    } else {
                        return kval<KIND>(r2, diag, kp);
                    }
                };
                if constexpr (sizeof(PT) == 8) {
                    for (int j = jb + s; j < je; j += NS) {
                        const PT x0 = sx[j], y0 = sy[j], z0 = D == 3 ? sz[j] : PT(0), q0 = sq[j];
                        const PT w0 = XW ? sw[j] : PT(0);
#pragma unroll
                        for (int k = 0; k < TPT; ++k)
                            acc[k] = fma(kv(add_extra<KIND>(dist2<false, D>(tx[k] - x0, ty[k] - y0, tz[k] - z0), tw[k], w0)),
                                         q0, acc[k]);
                    }
                } else {
                    // float partial sums per slice, accumulated in double
                    PT a[TPT];
#pragma unroll
                    for (int k = 0; k < TPT; ++k) a[k] = PT(0);
                    for (int j = jb + s; j < je; j += NS) {
                        const PT x0 = sx[j], y0 = sy[j], z0 = D == 3 ? sz[j] : PT(0), q0 = sq[j];
                        const PT w0 = XW ? sw[j] : PT(0);
#pragma unroll
                        for (int k = 0; k < TPT; ++k)
                            a[k] += kv(add_extra<KIND>(dist2<false, D>(tx[k] - x0, ty[k] - y0, tz[k] - z0), tw[k], w0)) * q0;
                    }
#pragma unroll
                    for (int k = 0; k < TPT; ++k) acc[k] += (double)a[k];
                }
            };
            auto flush = [&]() {
                __syncthreads();
                if (s < NS) {
                    // only the target leaf's own points can coincide with a target
                    slice_sum(0, self0, std::false_type{});
                    slice_sum(self0, self1, std::true_type{});
                    slice_sum(self1, pos, std::false_type{});
                }
                __syncthreads();
                pos = self0 = self1 = 0;
            };
            // a group of P2P_SRC slots is staged with all its loads in flight at once
            for (int base = 0; base < S; base += P2P_SRC) {
                const int take = min(S - base, P2P_SRC);
                for (int j = tid; j < take; j += NT_P2P) {
                    const int e = box_of(base + j);
                    const int src = nbbeg[e] + (base + j - nboff[e]);
                    if constexpr (P::local) {
                        const int gs = t.leaf0 + t.near_idx[ne0 + e];
                        sx[j] = (PT)((t.box_ctr[3 * gs] - cX[0]) + (double)t.px[src]);
                        sy[j] = (PT)((t.box_ctr[3 * gs + 1] - cX[1]) + (double)t.py[src]);
                        if constexpr (D == 3) sz[j] = (PT)((t.box_ctr[3 * gs + 2] - cX[2]) + (double)t.pz[src]);
                    } else {
                        sx[j] = t.px[src];
                        sy[j] = t.py[src];
                        if constexpr (D == 3) sz[j] = t.pz[src];
                    }
                    sq[j] = (PT)t.qt[src];
                    if constexpr (XW) sw[j] = t.pw[src];
                }
                pos = take;
                if (nself >= 0) {
                    self0 = min(max(nboff[nself] - base, 0), take);
                    self1 = min(max(nboff[nself + 1] - base, 0), take);
                }
                flush();
            }
#pragma unroll
            for (int k = 0; k < TPT; ++k) red[k * NT_P2P + tid] = s < NS ? acc[k] : 0.0;
            __syncthreads();
            if (tid < NP) {
#pragma unroll
                for (int k = 0; k < TPT; ++k) {
                    double phi = 0.0;
                    for (int q = 0; q < NS; ++q) phi += red[k * NT_P2P + q * NP + tid];
                    if (k == 0 || it[k] != it[0]) t.yn[b + it[k]] = phi;
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Symmetric near field.  N* is symmetric (X' in N*(X) iff X in N*(X')) and so
// is K, so the block of leaf X evaluates its own block and the blocks of the
// near leaves above it once each:
//   yn_X[i]        = sum over X and upper X', j of K(x_i, x_j) q_j       (row sums)
//   w_{X->X'}[j]   = sum_i K(x_i, x_j) q_i  for the points j of upper X'  (column sums)
// the column sums going to the pair's slot in the near-field W; L2P adds to
// yn the slots of the near leaves below (in list order).  The layout is the
// one-sided near field's (TPT targets per thread against a slice of the
// staged sources); each thread leaves its targets' share of a source's
// column sum in LDS and the sums over the target groups are taken in order.
// ---------------------------------------------------------------------------
constexpr int P2PS_SPT = 4;    // staged sources per thread and group
constexpr int P2PS_GMAX = 256; // staged sources per group at most

template <class P, int KIND, int D> __device__ __forceinline__ void p2p_sym_body(const DevTree<P> &t, int leaf)
{
    using PT = typename P::pt_t;
    constexpr bool TAB = sizeof(PT) == 8;
    constexpr int TPT = P2P_TPT;
    constexpr bool XW = kExtraCoord<KIND>;
    __shared__ PT sx[P2PS_GMAX], sy[P2PS_GMAX], sz[D == 3 ? P2PS_GMAX : 1], sq[P2PS_GMAX], sw[XW ? P2PS_GMAX : 1];
    __shared__ int32_t sW[P2PS_GMAX]; // W position of a staged source of an upper leaf, -1 for the leaf's own
    __shared__ PT colpart[NT_P2P * P2PS_SPT];
    __shared__ double red[TPT * NT_P2P];
    __shared__ __align__(16) double ktab[TAB ? kTabLen<KIND> : 2];
    // the leaf itself and the near leaves above it in list order as slots 0 .. S-1 (slot s in
    // entry e: nboff[e] <= s < nboff[e + 1], point nbbeg[e] + s - nboff[e]); entry 0 is the leaf
    __shared__ int32_t nboff[kMaxList + 1], nbbeg[kMaxList], nbw[kMaxList], nbg[kMaxList];
    const int tid = threadIdx.x;
    const PT diag = (PT)t.diag;
    const KPar<PT> kp = kpar<PT>(t);
    if constexpr (TAB) stage_table<KIND>(t.ktab, ktab); // first used after a barrier
    const int g = t.leaf0 + leaf;
    const int b = t.box_begin[g], n = t.box_end[g] - b;
    const double *cX = t.box_ctr + 3 * g;
    const int eself = t.near_self[leaf], ne1 = t.near_off[leaf + 1];
    const int nne = ne1 - eself; // the leaf and the leaves above it (<= kMaxList, checked at build)
    for (int k = tid; k < nne; k += NT_P2P) {
        const int gs = t.leaf0 + t.near_idx[eself + k];
        nbbeg[k] = t.box_begin[gs];
        nboff[k + 1] = t.box_end[gs] - t.box_begin[gs];
        nbw[k] = k == 0 ? -1 : (int32_t)t.near_w[eself + k];
        nbg[k] = gs;
    }
    __syncthreads();
    if (tid == 0) {
        nboff[0] = 0;
        for (int k = 0; k < nne; ++k) nboff[k + 1] += nboff[k];
    }
    __syncthreads();
    const int S = nboff[nne], nown = nboff[1]; // slots [0, nown) are the leaf's own points
    auto box_of = [&](int sl) -> int {
        int lo = 0, hi = nne - 1; // largest e with nboff[e] <= sl
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (nboff[mid] <= sl) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    };
    for (int i0 = 0; i0 < n; i0 += TPT * NT_P2P) {
        // MT targets this pass in NP groups (a, a + NP, ...); NS source slices
        const int MT = min(n - i0, TPT * NT_P2P), NP = (MT + TPT - 1) / TPT, NS = NT_P2P / NP;
        const int G = min(NS * P2PS_SPT, P2PS_GMAX);
        const int s = tid / NP, pa = tid % NP;
        const bool act = s < NS;
        int it[TPT];
        PT tx[TPT], ty[TPT], tz[TPT], tw[TPT], tq[TPT];
        double acc[TPT];
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            const bool real = pa + k * NP < MT;
            it[k] = real ? i0 + pa + k * NP : i0 + pa; // a missing target repeats the first, with no charge
            tx[k] = t.px[b + it[k]];
            ty[k] = t.py[b + it[k]];
            tz[k] = D == 3 ? t.pz[b + it[k]] : PT(0);
            tw[k] = XW ? t.pw[b + it[k]] : PT(0);
            tq[k] = real ? (PT)t.qt[b + it[k]] : PT(0);
            acc[k] = 0.0;
        }
        for (int base = 0; base < S; base += G) {
            const int take = min(S - base, G);
            for (int j = tid; j < take; j += NT_P2P) {
                const int e = box_of(base + j);
                const int o = base + j - nboff[e], src = nbbeg[e] + o;
                if constexpr (P::local) {
                    const int gs = nbg[e];
                    sx[j] = (PT)((t.box_ctr[3 * gs] - cX[0]) + (double)t.px[src]);
                    sy[j] = (PT)((t.box_ctr[3 * gs + 1] - cX[1]) + (double)t.py[src]);
                    if constexpr (D == 3) sz[j] = (PT)((t.box_ctr[3 * gs + 2] - cX[2]) + (double)t.pz[src]);
                } else {
                    sx[j] = t.px[src];
                    sy[j] = t.py[src];
                    if constexpr (D == 3) sz[j] = t.pz[src];
                }
                sq[j] = (PT)t.qt[src];
                if constexpr (XW) sw[j] = t.pw[src];
                sW[j] = e == 0 ? -1 : nbw[e] + o;
            }
            __syncthreads();
            if (act) {
                const int own_end = min(max(nown - base, 0), take); // own points: staged [0, own_end)
                PT a[TPT]; // float policies: partial sums of the group in float, added to acc in double
#pragma unroll
                for (int k = 0; k < TPT; ++k) a[k] = PT(0);
                for (int j = s; j < take; j += NS) {
                    const PT x0 = sx[j], y0 = sy[j], z0 = D == 3 ? sz[j] : PT(0), q0 = sq[j];
                    const PT w0 = XW ? sw[j] : PT(0);
                    PT kv[TPT];
#pragma unroll
                    for (int k = 0; k < TPT; ++k) {
                        const PT r2 = add_extra<KIND>(dist2<false, D>(tx[k] - x0, ty[k] - y0, tz[k] - z0), tw[k], w0);
                        if constexpr (sizeof(PT) == 8) {
                            // only the leaf's own points can coincide with a target
                            kv[k] = j < own_end ? kval<KIND>(r2, diag, kp, ktab) : kval_pos<KIND>(r2, kp, ktab);
                        } else {
                            kv[k] = kval<KIND>(r2, diag, kp);
                        }
                    }
                    PT c = PT(0);
#pragma unroll
                    for (int k = 0; k < TPT; ++k) {
                        if constexpr (sizeof(PT) == 8) acc[k] = fma(kv[k], q0, acc[k]);
                        else a[k] += kv[k] * q0;
                        c = fma(kv[k], tq[k], c);
                    }
                    colpart[pa * G + j] = c;
                }
                if constexpr (sizeof(PT) != 8) {
#pragma unroll
                    for (int k = 0; k < TPT; ++k) acc[k] += (double)a[k];
                }
            }
            __syncthreads();
            for (int j = tid; j < take; j += NT_P2P) {
                if (sW[j] < 0) continue;
                double c = 0.0;
                for (int p = 0; p < NP; ++p) c += (double)colpart[p * G + j];
                // a leaf of more than TPT * NT_P2P points adds its later target passes to the first's
                const double prev = i0 == 0 ? 0.0 : t.near_wv[sW[j]];
                t.near_wv[sW[j]] = prev + c;
            }
            // the next group's staging writes sx .. sW only at indices this thread reads here, and
            // colpart only after its barrier
        }
#pragma unroll
        for (int k = 0; k < TPT; ++k) red[k * NT_P2P + tid] = act ? acc[k] : 0.0;
        __syncthreads();
        if (tid < NP) {
#pragma unroll
            for (int k = 0; k < TPT; ++k) {
                double phi = 0.0;
                for (int q = 0; q < NS; ++q) phi += red[k * NT_P2P + q * NP + tid];
                if (k == 0 || it[k] != it[0]) t.yn[b + it[k]] = phi;
            }
        }
        __syncthreads();
    }
}

// leaves leaf_begin .. leaf_begin + gridDim.x - 1, one per block
template <class P, int KIND, int D>
__global__ __launch_bounds__(NT_P2P) __attribute__((amdgpu_waves_per_eu(5))) void k_p2p(DevTree<P> t, int32_t leaf_begin, int32_t leaf_count)
{
    (void)leaf_count; // == gridDim.x
    p2p_sym_body<P, KIND, D>(t, leaf_begin + xcd_remap(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// Leaf pass down: near field + shift q, L2P (in index order), the (H2+H)*
// vertex blocks, sum and scatter to user order.  One thread per point.
// ---------------------------------------------------------------------------
constexpr int NT_LEAF = 128;

template <class P>
__device__ __forceinline__ void down_leaf_body(const DevTree<P> &t, int leaf, double *__restrict__ y, uint32_t mask)
{
    constexpr bool ORD = P::ordered;
    constexpr int HALF = NT_LEAF / 2;
    using BT = typename P::basis_t;
    __shared__ double ver_part[HALF];
    extern __shared__ double ucs[]; // the leaf's locals: far family, then vertex family
    const int g = t.leaf0 + leaf;
    const int b = t.box_begin[g], n = t.box_end[g] - b;
    const int cf = t.far.coef_off[g], cv = t.ver.coef_off[g];
    const int rf = (mask & kFar) && t.kappa >= t.far.lmin ? t.far.coef_off[g + 1] - cf : 0;
    const int rv = (mask & kVer) && t.kappa >= t.ver.lmin ? t.ver.coef_off[g + 1] - cv : 0;
    // threads [0, HALF) take the far family of point i, [HALF, NT_LEAF) the vertex family
    const int f = threadIdx.x < HALF ? 0 : 1, il = threadIdx.x - f * HALF;
    const int r = f == 0 ? rf : rv;
    // kept rows of U column-major (nk x r); a unit row e_a gives the local a itself
    const BT *U = f == 0 ? t.far.U_cm + t.far.uoff[leaf] : t.ver.U_cm + t.ver.uoff[leaf];
    const int16_t *urow = (f == 0 ? t.far.urow : t.ver.urow) + b;
    const int nk = r ? (f == 0 ? t.far.unk[leaf] : t.ver.unk[leaf]) : 0;
    const double *uc = f == 0 ? ucs : ucs + rf;
    // a point's row map and near-field values; the first chunk's are read before the barrier,
    // beside the locals
    int ki = 0, dst = 0;
    double yv = 0.0, qv = 0.0;
    const int ne0 = t.near_off[leaf], nes = t.near_self[leaf]; // near leaves below this one: [ne0, nes)
    auto point_loads = [&](int i) {
        if (i < n && r) ki = urow[i];
        if (f == 0 && i < n) {
            // the symmetric near field left the column sums of the near leaves below in W
            double v = t.yn[b + i];
            if (mask & kNear)
                for (int e = ne0; e < nes; ++e) v += t.near_wv[t.near_w[e] + i];
            yv = v;
            qv = t.qt[b + i];
            dst = t.perm[b + i];
        }
    };
    point_loads(il);
    for (int k = threadIdx.x; k < rf; k += NT_LEAF) ucs[k] = t.far.u[cf + k];
    for (int k = threadIdx.x; k < rv; k += NT_LEAF) ucs[rf + k] = t.ver.u[cv + k];
    __syncthreads();
    for (int i0 = 0; i0 < n; i0 += HALF) {
        const int i = i0 + il;
        if (i0 > 0) point_loads(i);
        double fam = 0.0;
        if (i < n && r) fam = ki >= 0 ? ordered_dot<ORD>(U + ki, (size_t)nk, r, uc) : uc[~ki];
        if (f == 1 && i < n) {
            double v = fam;
            if (t.variant == H2S_H2_PLUS_H && (mask & kVer)) {
                const auto &Pr = t.pairs;
                for (int l = 1; l <= t.kappa; ++l) {
                    const int X = t.leaf_anc[(size_t)leaf * (t.kappa + 1) + l];
                    const int off = b + i - t.box_begin[X];
                    const int nX = t.box_end[X] - t.box_begin[X];
                    for (int e = Pr.recv_off[X]; e < Pr.recv_off[X + 1]; ++e) {
                        const int ps = Pr.recv[e], p = ps >> 1, side = ps & 1;
                        const int rp = Pr.prank[p];
                        const auto *G = Pr.data + (side == 0 ? Pr.pu[p] : Pr.pv[p]);
                        const double *w = Pr.w + Pr.pw[p] + (size_t)side * rp;
                        v = v + ordered_dot<ORD>(G + off, (size_t)nX, rp, w);
                    }
                }
            }
            ver_part[il] = v;
        }
        __syncthreads();
        if (f == 0 && i < n) {
            double phi = 0.0;
            if (mask & kNear) phi = madd<ORD>(yv, t.shift, qv);
            if (mask & kFar) phi = phi + fam;
            if (mask & kVer) phi = phi + ver_part[il];
            y[dst] = phi;
        }
        __syncthreads();
    }
}

template <class P>
__global__ __launch_bounds__(NT_LEAF, LEAF_WAVES) void k_down_leaf(DevTree<P> t, double *__restrict__ y, uint32_t mask)
{
    down_leaf_body(t, xcd_remap(blockIdx.x, gridDim.x), y, mask);
}

// ---------------------------------------------------------------------------
// Many trees in one launch per step (MultiPlan): block b takes work item
// map[b].y of tree map[b].x; the tree's description is copied from device
// memory (uniform over the block, so it lands in scalar registers) and the
// single-tree body runs on it, so every output is the one h2s_apply gives.
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(256) void km_permute(const DevTree<P> *__restrict__ trees, const int2 *__restrict__ map,
                                                  const double *const *__restrict__ xs)
{
    const int2 w = map[blockIdx.x];
    const DevTree<P> t = trees[w.x];
    permute_body(t, xs[w.x], w.y);
}

template <class P>
__global__ __launch_bounds__(NT_GEMV_MAX, GEMV_WAVES) void km_up_leaf(const DevTree<P> *__restrict__ trees,
                                                                       const int2 *__restrict__ map)
{
    const int2 w = map[xcd_remap(blockIdx.x, gridDim.x)];
    const DevTree<P> t = trees[w.x];
    up_leaf_body(t, w.y, kFar | kVer);
}

template <class P>
__global__ __launch_bounds__(NT_GEMV_MAX, GEMV_WAVES) void km_m2m(const DevTree<P> *__restrict__ trees,
                                                                   const int2 *__restrict__ map)
{
    const int2 w = map[blockIdx.x];
    const DevTree<P> t = trees[w.x];
    m2m_body(t, w.y, kFar | kVer);
}

template <class P>
__global__ __launch_bounds__(NT_GEMV_MAX, GEMV_WAVES) void km_l2l(const DevTree<P> *__restrict__ trees,
                                                                   const int2 *__restrict__ map)
{
    const int2 w = map[blockIdx.x];
    const DevTree<P> t = trees[w.x];
    l2l_body(t, w.y, kFar | kVer);
}

template <class P, bool FAR, int KIND, int D, int NT, int SRC>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(5))) void km_m2l(const DevTree<P> *__restrict__ trees, const int2 *__restrict__ map)
{
    const int2 w = map[xcd_remap(blockIdx.x, gridDim.x)];
    const DevTree<P> t = trees[w.x];
    m2l_slices_body<P, FAR, KIND, D, NT, SRC>(t, w.y);
}

template <class P, int KIND, int D>
__global__ __launch_bounds__(NT_P2P) void km_p2p(const DevTree<P> *__restrict__ trees, const int2 *__restrict__ map)
{
    const int2 w = map[xcd_remap(blockIdx.x, gridDim.x)];
    const DevTree<P> t = trees[w.x];
    p2p_sym_body<P, KIND, D>(t, w.y);
}

// (no waves-per-SIMD bound: under the single-tree bound this one spills)
template <class P>
__global__ __launch_bounds__(NT_LEAF) void km_down_leaf(const DevTree<P> *__restrict__ trees, const int2 *__restrict__ map,
                                                        double *const *__restrict__ ys)
{
    const int2 w = map[xcd_remap(blockIdx.x, gridDim.x)];
    const DevTree<P> t = trees[w.x];
    down_leaf_body(t, w.y, ys[w.x], kNear | kFar | kVer);
}

// The steps of MultiPlan on st.main, the near field on st.aux (forked after
// the permutation, joined before L2P).
template <class P, int KIND, int D> hipError_t enqueue_multi(const MultiPlan<P> &mp, const Streams &st)
{
    hipStream_t s = (hipStream_t)st.main, aux = (hipStream_t)st.aux;
    hipError_t err;
    if (mp.n_perm) hipLaunchKernelGGL(km_permute<P>, dim3(mp.n_perm), dim3(256), 0, s, mp.trees, mp.perm_map, mp.xs);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if ((err = hipEventRecord((hipEvent_t)st.fork, s)) != hipSuccess) return err;
    if ((err = hipStreamWaitEvent(aux, (hipEvent_t)st.fork, 0)) != hipSuccess) return err;
    if (mp.n_leaf) hipLaunchKernelGGL((km_p2p<P, KIND, D>), dim3(mp.n_leaf), dim3(NT_P2P), 0, aux, mp.trees, mp.leaf_map);
    if ((err = hipEventRecord((hipEvent_t)st.join, aux)) != hipSuccess) return err;
    if (mp.n_up) hipLaunchKernelGGL(km_up_leaf<P>, dim3(mp.n_up), dim3(mp.w_up), mp.lds_leaf, s, mp.trees, mp.up_map);
    for (int k = 0; k < mp.steps; ++k)
        if (mp.n_m2m[k])
            hipLaunchKernelGGL(km_m2m<P>, dim3(mp.n_m2m[k]), dim3(mp.w_m2m[k]), mp.lds_rows, s, mp.trees, mp.m2m_map[k]);
    if (mp.n_far)
        hipLaunchKernelGGL((km_m2l<P, true, KIND, D, kM2LFarNT, kM2LFarSRC>), dim3(mp.n_far), dim3(kM2LFarNT), 0, s, mp.trees,
                           mp.far_map);
    if (mp.n_ver)
        hipLaunchKernelGGL((km_m2l<P, false, KIND, D, kM2LVerNT, kM2LVerSRC>), dim3(mp.n_ver), dim3(kM2LVerNT), 0, s,
                           mp.trees, mp.ver_map);
    for (int k = 0; k < mp.steps; ++k)
        if (mp.n_l2l[k])
            hipLaunchKernelGGL(km_l2l<P>, dim3(mp.n_l2l[k]), dim3(mp.w_l2l[k]), mp.lds_rank, s, mp.trees, mp.l2l_map[k]);
    if ((err = hipStreamWaitEvent(s, (hipEvent_t)st.join, 0)) != hipSuccess) return err;
    if (mp.n_leaf)
        hipLaunchKernelGGL(km_down_leaf<P>, dim3(mp.n_leaf), dim3(NT_LEAF), mp.lds_rank, s, mp.trees, mp.leaf_map, mp.ys);
    return hipGetLastError();
}

template <class P, int KIND, int D>
hipError_t enqueue(const DevTree<P> &t, const LaunchPlan &plan, const double *x, double *y, uint32_t mask,
                   const Streams &st, const ProfileHook *prof)
{
    hipStream_t s = (hipStream_t)st.main, aux = (hipStream_t)st.aux;
    auto mark = [&](int cls, int end, hipStream_t on) {
        if (prof) prof->mark(prof->ctx, cls, end, on);
    };
    const int32_t *lev_off = plan.lev_off;
    const size_t lds_leaf = sizeof(double) * (size_t)(2 * t.max_leaf);
    const size_t lds_rows = sizeof(double) * (size_t)(2 * t.max_rows);
    const size_t lds_rank = sizeof(double) * (size_t)(2 * t.max_rank);
    const bool fam_on = (mask & (kFar | kVer)) && t.kappa >= 1;
    mark(H2S_PROF_LEAF_UP, 0, s);
    hipLaunchKernelGGL(k_permute<P>, dim3((t.n + 255) / 256), dim3(256), 0, s, t, x);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    // The near field needs only the permuted charges.  It runs on the second
    // stream in two pieces: the first near_first of the leaves beside P2M and
    // M2M (HBM- and latency-bound), the rest beside L2L, so that it shares
    // the GPU with the memory-bound sweeps rather than with the ALU-bound
    // M2L.  The leaf-level M2L needs only the leaf multipoles: with
    // plan.m2l_stream it runs on a third stream from the end of P2M, beside
    // the coarse M2M levels (latency-bound, few boxes), and only the L2L into
    // the leaves waits for it.  With m2l_stream 2 the M2L of the level above
    // the leaves (most of the coarse M2L) runs on a fourth stream as soon as
    // M2M has made that level's multipoles, beside the rest of the M2M chain;
    // the coarser levels' M2L follows the chain on the main stream as one
    // launch per family (a launch per level would chain their latencies), and
    // the L2L chain waits for both.  Under the profiling hook everything runs on
    // the main stream instead, so that every kernel class is timed alone.
    const bool overlap = (mask & kNear) && !prof;
    const bool split = fam_on && !prof && plan.m2l_stream != 0;
    const bool pipe = split && plan.m2l_stream == 2;
    const int near1 = overlap && fam_on ? (int)(plan.near_first * t.nleaf) : t.nleaf;
    auto fork_near = [&](hipEvent_t ev, int lb, int le) -> hipError_t {
        hipError_t e2;
        if ((e2 = hipEventRecord(ev, s)) != hipSuccess) return e2;
        if ((e2 = hipStreamWaitEvent(aux, ev, 0)) != hipSuccess) return e2;
        if (le > lb) hipLaunchKernelGGL((k_p2p<P, KIND, D>), dim3(le - lb), dim3(NT_P2P), 0, aux, t, lb, le - lb);
        return hipEventRecord((hipEvent_t)st.join, aux);
    };
    // M2L of one family over its targets [tb, te) on stream `on`.  Targets of one level need
    // only that level's multipoles, and every level's targets are a contiguous range, so a range
    // split at a level boundary needs nothing from the other part.
    auto m2l = [&](bool far, int32_t tb, int32_t te, hipStream_t on) {
        if (te <= tb) return;
        if (far) {
            if constexpr (sizeof(typename P::far_t) == 4)
                hipLaunchKernelGGL((k_m2l<P, true, KIND, D>), dim3(te - tb), dim3(NT_M2L), 0, on, t, tb);
            else
                hipLaunchKernelGGL((k_m2l_slices<P, true, KIND, D, kM2LFarNT, kM2LFarSRC>), dim3(te - tb), dim3(kM2LFarNT), 0,
                                   on, t, tb);
        } else {
            hipLaunchKernelGGL((k_m2l_slices<P, false, KIND, D, kM2LVerNT, kM2LVerSRC>), dim3(te - tb), dim3(kM2LVerNT), 0,
                               on, t, tb);
        }
    };
    const bool far_on = (mask & kFar) != 0, ver_on = (mask & kVer) != 0;
    const int32_t far_split = split ? t.far.targets_leaf : t.far.ntargets;
    const int32_t ver_split = split ? t.ver.targets_leaf : t.ver.ntargets;
    if (overlap && (err = fork_near((hipEvent_t)st.fork, 0, near1)) != hipSuccess) return err;
    if (fam_on) hipLaunchKernelGGL(k_up_leaf<P>, dim3(t.nleaf), dim3(plan.up_threads[t.kappa]), lds_leaf, s, t, mask);
    mark(H2S_PROF_LEAF_UP, 1, s);
    if ((mask & kNear) && !overlap) {
        mark(H2S_PROF_NEAR, 0, s);
        hipLaunchKernelGGL((k_p2p<P, KIND, D>), dim3(t.nleaf), dim3(NT_P2P), 0, s, t, 0, t.nleaf);
        mark(H2S_PROF_NEAR, 1, s);
    }
    if (split) {
        hipStream_t aux2 = (hipStream_t)st.aux2;
        if ((err = hipEventRecord((hipEvent_t)st.fork3, s)) != hipSuccess) return err;
        if ((err = hipStreamWaitEvent(aux2, (hipEvent_t)st.fork3, 0)) != hipSuccess) return err;
        if (far_on) m2l(true, far_split, t.far.ntargets, aux2);
        if (ver_on) m2l(false, ver_split, t.ver.ntargets, aux2);
        if ((err = hipEventRecord((hipEvent_t)st.join2, aux2)) != hipSuccess) return err;
    }
    if (fam_on) {
        mark(H2S_PROF_M2M, 0, s);
        // with pipe, the M2L of level kappa - 1 goes to the fourth stream after its M2M
        const int lp = pipe && t.kappa >= 2 ? t.kappa - 1 : -1;
        const int32_t far_mid = lp > 0 ? plan.tlev[0][lp] : far_split, ver_mid = lp > 0 ? plan.tlev[1][lp] : ver_split;
        for (int l = t.kappa - 1; l >= 1; --l) {
            const int nb = lev_off[l + 1] - lev_off[l];
            if (nb)
                hipLaunchKernelGGL(k_m2m<P>, dim3(nb), dim3(plan.up_threads[l]), lds_rows, s, t, lev_off[l], mask);
            if (l == lp) {
                hipStream_t aux3 = (hipStream_t)st.aux3;
                if ((err = hipEventRecord((hipEvent_t)st.fork4, s)) != hipSuccess) return err;
                if ((err = hipStreamWaitEvent(aux3, (hipEvent_t)st.fork4, 0)) != hipSuccess) return err;
                if (far_on) m2l(true, far_mid, far_split, aux3);
                if (ver_on) m2l(false, ver_mid, ver_split, aux3);
                if ((err = hipEventRecord((hipEvent_t)st.join3, aux3)) != hipSuccess) return err;
            }
        }
        mark(H2S_PROF_M2M, 1, s);
        if (far_on && t.far.ntargets) {
            mark(H2S_PROF_M2L_FAR, 0, s);
            m2l(true, 0, far_mid, s);
            mark(H2S_PROF_M2L_FAR, 1, s);
        }
        if (ver_on && t.ver.ntargets) {
            mark(H2S_PROF_M2L_VER, 0, s);
            m2l(false, 0, ver_mid, s);
            mark(H2S_PROF_M2L_VER, 1, s);
        }
        if (lp > 0 && (err = hipStreamWaitEvent(s, (hipEvent_t)st.join3, 0)) != hipSuccess) return err;
        if (overlap && (err = fork_near((hipEvent_t)st.fork2, near1, t.nleaf)) != hipSuccess) return err;
        mark(H2S_PROF_L2L, 0, s);
        for (int l = 1; l <= t.kappa - 1; ++l) {
            // the L2L into the leaves adds to the leaf-level M2L results
            if (split && l == t.kappa - 1 && (err = hipStreamWaitEvent(s, (hipEvent_t)st.join2, 0)) != hipSuccess)
                return err;
            const int nb = lev_off[l + 1] - lev_off[l];
            if (nb)
                hipLaunchKernelGGL(k_l2l<P>, dim3(nb), dim3(plan.dn_threads[l]), lds_rank, s, t, lev_off[l], mask);
        }
        if (split && t.kappa < 2 && (err = hipStreamWaitEvent(s, (hipEvent_t)st.join2, 0)) != hipSuccess) return err;
        mark(H2S_PROF_L2L, 1, s);
    }
    if (t.variant == H2S_H2_PLUS_H && (mask & kVer) && t.pairs.npairs) {
        mark(H2S_PROF_PAIR_PART, 0, s);
        hipLaunchKernelGGL(k_pair_part<P>, dim3(t.pairs.nchunks), dim3(256), 0, s, t);
        mark(H2S_PROF_PAIR_PART, 1, s);
        mark(H2S_PROF_PAIR_SUM, 0, s);
        hipLaunchKernelGGL(k_pair_sum<P>, dim3(2 * t.pairs.npairs), dim3(64), 0, s, t);
        mark(H2S_PROF_PAIR_SUM, 1, s);
    }
    if (overlap)
        if ((err = hipStreamWaitEvent(s, (hipEvent_t)st.join, 0)) != hipSuccess) return err;
    mark(H2S_PROF_LEAF_DOWN, 0, s);
    hipLaunchKernelGGL(k_down_leaf<P>, dim3(t.nleaf), dim3(NT_LEAF), lds_rank, s, t, y, mask);
    mark(H2S_PROF_LEAF_DOWN, 1, s);
    return hipGetLastError();
}

} // namespace

template <class P>
int launch_mvp(const DevTree<P> &t, const LaunchPlan &plan, const double *x, double *y, uint32_t mask,
               const Streams &s, const ProfileHook *prof)
{
    const int key = t.kind * 2 + (t.d == 3);
    switch (key) {
    case 0: return (int)enqueue<P, H2S_K_LOG_R, 2>(t, plan, x, y, mask, s, prof);
    case 1: return (int)enqueue<P, H2S_K_LOG_R, 3>(t, plan, x, y, mask, s, prof);
    case 2: return (int)enqueue<P, H2S_K_INV_R, 2>(t, plan, x, y, mask, s, prof);
    case 3: return (int)enqueue<P, H2S_K_INV_R, 3>(t, plan, x, y, mask, s, prof);
    case 4: return (int)enqueue<P, H2S_K_GAUSSIAN, 2>(t, plan, x, y, mask, s, prof);
    case 5: return (int)enqueue<P, H2S_K_GAUSSIAN, 3>(t, plan, x, y, mask, s, prof);
    case 6: return (int)enqueue<P, H2S_K_EXP_R, 2>(t, plan, x, y, mask, s, prof);
    case 7: return (int)enqueue<P, H2S_K_EXP_R, 3>(t, plan, x, y, mask, s, prof);
    case 8: return (int)enqueue<P, H2S_K_RBF_AR, 2>(t, plan, x, y, mask, s, prof);
    case 9: return (int)enqueue<P, H2S_K_RBF_AR, 3>(t, plan, x, y, mask, s, prof);
    case 10: return (int)enqueue<P, H2S_K_RBF_LOG, 2>(t, plan, x, y, mask, s, prof);
    case 11: return (int)enqueue<P, H2S_K_RBF_LOG, 3>(t, plan, x, y, mask, s, prof);
    case 13: // the NTI multiquadric: 3D, not with the float far field of FP32_M2L
        if constexpr (std::is_same_v<P, P32M>) return (int)hipErrorInvalidValue;
        else return (int)enqueue<P, H2S_K_NTI_MQ, 3>(t, plan, x, y, mask, s, prof);
    default: return (int)hipErrorInvalidValue;
    }
}

template <class P> int launch_multi(int kind, int d, const MultiPlan<P> &mp, const Streams &s)
{
    switch (kind * 2 + (d == 3)) {
    case 0: return (int)enqueue_multi<P, H2S_K_LOG_R, 2>(mp, s);
    case 1: return (int)enqueue_multi<P, H2S_K_LOG_R, 3>(mp, s);
    case 2: return (int)enqueue_multi<P, H2S_K_INV_R, 2>(mp, s);
    case 3: return (int)enqueue_multi<P, H2S_K_INV_R, 3>(mp, s);
    case 4: return (int)enqueue_multi<P, H2S_K_GAUSSIAN, 2>(mp, s);
    case 5: return (int)enqueue_multi<P, H2S_K_GAUSSIAN, 3>(mp, s);
    case 6: return (int)enqueue_multi<P, H2S_K_EXP_R, 2>(mp, s);
    case 7: return (int)enqueue_multi<P, H2S_K_EXP_R, 3>(mp, s);
    case 8: return (int)enqueue_multi<P, H2S_K_RBF_AR, 2>(mp, s);
    case 9: return (int)enqueue_multi<P, H2S_K_RBF_AR, 3>(mp, s);
    case 10: return (int)enqueue_multi<P, H2S_K_RBF_LOG, 2>(mp, s);
    case 11: return (int)enqueue_multi<P, H2S_K_RBF_LOG, 3>(mp, s);
    case 13: return (int)enqueue_multi<P, H2S_K_NTI_MQ, 3>(mp, s);
    default: return (int)hipErrorInvalidValue;
    }
}

template int launch_multi<P64>(int, int, const MultiPlan<P64> &, const Streams &);
template int launch_multi<P32>(int, int, const MultiPlan<P32> &, const Streams &);

template int launch_mvp<P64>(const DevTree<P64> &, const LaunchPlan &, const double *, double *, uint32_t, const Streams &,
                             const ProfileHook *);
template int launch_mvp<P32>(const DevTree<P32> &, const LaunchPlan &, const double *, double *, uint32_t, const Streams &,
                             const ProfileHook *);
template int launch_mvp<P32M>(const DevTree<P32M> &, const LaunchPlan &, const double *, double *, uint32_t, const Streams &,
                              const ProfileHook *);

} // namespace h2s
