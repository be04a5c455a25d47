// h2s_kernels.hip -- HIP kernels of the H2* / (H2+H)* matrix-vector product
// for CDNA4 (gfx950), Khan & Ambikasaran (arXiv 2309.14085), Sec. 5.1.2 and
// Sec. 5.2.2:
//
//   k_up_leaf    charges to tree order + P2M   v_X = U_X^T q_X            (both families)
//   k_m2m        one level of M2M              v_X = sum_c U~_{X_c X}^T v_{X_c}
//   k_m2l        all levels of one family      u_X = sum_{Y in IL(X)} K(t^{X,i}, t^{Y,i}) v_Y
//   k_l2l        one level of L2L              u_{X_c} += U~_{X_c X} u_X
//   k_pair_part  (H2+H)*: partial products Vb^T q_Y, Ub^T q_X over row chunks
//   k_pair_sum   (H2+H)*: chunk sums in a fixed order
//   k_down_leaf  near field over N*(X) + L2P U_X u_X + (H2+H)* vertex blocks,
//                scattered back to user order
//
// Summation order.  The interpolative NCA operators have norms up to ~1e3 -
// 1e4 on coarse levels, so a rounding difference in a multipole or local
// coefficient is amplified on its way to the potential.  The steps whose
// results are amplified (P2M, M2M, the per-source-box M2L sums, L2L, L2P)
// therefore sum in the order of the definitions -- one output per thread,
// terms in index order, and under the FP64 policy with the product and the
// sum rounded separately -- so the GPU product tracks a plain sequential
// evaluation to within a few ulps of each coefficient.  The direct near field
// is a plain sum of kernel values (nothing amplifies it); it is split over
// source slices to fill the block.  No floating-point atomics are used.
//
// M2L and the near field evaluate the kernel on the fly from coordinates
// staged in LDS; the GEMV-shaped steps are HBM-bound and read each operator
// once, coalesced, from the copy laid out for them.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "h2s.h"
#include "h2s_device.hpp"

namespace h2s {

namespace {

constexpr unsigned kNear = 1u, kFar = 2u, kVer = 4u;

// Work items are dealt to the 8 XCDs round-robin by block index; remap so
// each XCD gets a contiguous (Morton-local, so L2-sharing) range of items.
__device__ __forceinline__ int xcd_remap(int bid, int nb)
{
    const int q = nb >> 3, rem = nb & 7, xcd = bid & 7, slot = bid >> 3;
    return xcd < rem ? xcd * (q + 1) + slot : rem * (q + 1) + (xcd - rem) * q + slot;
}

// s + a b: product and sum rounded separately (ORD) or fused.
template <bool ORD> __device__ __forceinline__ double madd(double s, double a, double b)
{
    if constexpr (ORD) return __dadd_rn(s, __dmul_rn(a, b));
    else return fma(a, b, s);
}

// 0.5 ln(x) for finite x > 0 in double, written from the mathematics:
// x = m 2^e with m in [sqrt(1/2), sqrt(2)) (frexp), ln m = 2 atanh(s) with
// s = (m - 1) / (m + 1), |s| <= 0.1716, and atanh(s) = s + s^3/3 + s^5/5 + ...
// summed through s^21 by Horner in s^2 (the next term is below 1e-19 of the
// result).  The quotient uses the hardware reciprocal refined by two Newton
// steps.  Error: a few ulps.
__device__ __forceinline__ double half_log(double x)
{
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752440) {
        m += m;
        e -= 1;
    }
    const double dn = m + 1.0;
    double rc = __builtin_amdgcn_rcp(dn);
    rc = fma(rc, fma(-dn, rc, 1.0), rc);
    rc = fma(rc, fma(-dn, rc, 1.0), rc);
    const double s = (m - 1.0) * rc;
    const double z = s * s;
    double p = 1.0 / 21;
    p = fma(p, z, 1.0 / 19);
    p = fma(p, z, 1.0 / 17);
    p = fma(p, z, 1.0 / 15);
    p = fma(p, z, 1.0 / 13);
    p = fma(p, z, 1.0 / 11);
    p = fma(p, z, 1.0 / 9);
    p = fma(p, z, 1.0 / 7);
    p = fma(p, z, 1.0 / 5);
    p = fma(p, z, 1.0 / 3);
    const double at = fma(s * z, p, s);
    return fma((double)e, 0.34657359027997264, at); // ln 2 / 2
}

// Which FP64 evaluation of log r the kernels use: the library's correctly
// rounded log(sqrt(r^2)), or half_log above.
constexpr bool kFastLog = true;

// Squared distance with products and sums rounded separately under ORD.
template <bool ORD, int D, typename T> __device__ __forceinline__ T dist2(T dx, T dy, T dz)
{
    if constexpr (ORD && sizeof(T) == 8) {
        double r2 = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
        if constexpr (D == 3) r2 = __dadd_rn(r2, __dmul_rn(dz, dz));
        return r2;
    } else {
        T r2 = dx * dx + dy * dy;
        if constexpr (D == 3) r2 += dz * dz;
        return r2;
    }
}

// Kernel value from the squared distance; r2 == 0 means coincident points.
// kp: h^2 for the Gaussian.
template <int KIND> __device__ __forceinline__ double kval(double r2, double diag, double kp)
{
    double v;
    if constexpr (KIND == H2S_K_LOG_R) v = kFastLog ? half_log(r2) : log(sqrt(r2));
    else if constexpr (KIND == H2S_K_INV_R) v = 1.0 / sqrt(r2);
    else if constexpr (KIND == H2S_K_GAUSSIAN) v = exp(-r2 / kp);
    else v = exp(-sqrt(r2));
    return r2 == 0.0 ? diag : v;
}

template <int KIND> __device__ __forceinline__ float kval(float r2, float diag, float kp)
{
    float v;
    if constexpr (KIND == H2S_K_LOG_R) v = __log2f(r2) * 0.34657359027997264f; // ln 2 / 2
    else if constexpr (KIND == H2S_K_INV_R) v = __frsqrt_rn(r2);
    else if constexpr (KIND == H2S_K_GAUSSIAN) v = __expf(-r2 / kp);
    else v = __expf(-__fsqrt_rn(r2));
    return r2 == 0.0f ? diag : v;
}

template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------------------
// P2M, M2M, L2L: one output per thread, terms in index order.
// ---------------------------------------------------------------------------
constexpr int NT_UP = 64; // P2M and M2M: ranks rarely exceed 64

// out[k] = sum_j A[j r + k] x[j] (A row-major R x r), one column k.
template <bool ORD, typename AT>
__device__ __forceinline__ void colsum(const AT *__restrict__ A, int R, int r, const double *xs, double *out, int k)
{
    double s = 0.0;
    for (int j = 0; j < R; ++j) s = madd<ORD>(s, (double)A[(size_t)j * r + k], xs[j]);
    out[k] = s;
}

template <class P>
__global__ __launch_bounds__(NT_UP) void k_up_leaf(DevTree<P> t, const double *__restrict__ x, uint32_t mask)
{
    extern __shared__ double qs[]; // largest leaf
    const int leaf = xcd_remap(blockIdx.x, gridDim.x), g = t.leaf0 + leaf, tid = threadIdx.x;
    const int b = t.box_begin[g], n = t.box_end[g] - b;
    for (int i = tid; i < n; i += NT_UP) {
        const double v = x[t.perm[b + i]];
        qs[i] = v;
        t.qt[b + i] = v;
    }
    __syncthreads();
    const int cf = t.far.coef_off[g], rf = (mask & kFar) && t.kappa >= t.far.lmin ? t.far.coef_off[g + 1] - cf : 0;
    const int cv = t.ver.coef_off[g], rv = (mask & kVer) && t.kappa >= t.ver.lmin ? t.ver.coef_off[g + 1] - cv : 0;
    // one column of the two families per thread
    for (int k = tid; k < rf + rv; k += NT_UP) {
        if (k < rf) colsum<P::ordered>(t.far.U_rm + t.far.uoff[leaf], n, rf, qs, t.far.v + cf, k);
        else colsum<P::ordered>(t.ver.U_rm + t.ver.uoff[leaf], n, rv, qs, t.ver.v + cv, k - rf);
    }
}

template <class P> __global__ __launch_bounds__(NT_UP) void k_m2m(DevTree<P> t, int32_t g0, uint32_t mask)
{
    extern __shared__ double xs[]; // both families' child coefficients
    const int g = g0 + blockIdx.x, tid = threadIdx.x;
    const auto &Fa = t.far;
    const auto &Ve = t.ver;
    const int cf = Fa.coef_off[g], rf = (mask & kFar) ? Fa.coef_off[g + 1] - cf : 0;
    const int cv = Ve.coef_off[g], rv = (mask & kVer) ? Ve.coef_off[g + 1] - cv : 0;
    const int bf = Fa.coef_off[t.box_cbeg[g]], Rf = rf ? Fa.coef_off[t.box_cend[g]] - bf : 0;
    const int bv = Ve.coef_off[t.box_cbeg[g]], Rv = rv ? Ve.coef_off[t.box_cend[g]] - bv : 0;
    for (int j = tid; j < Rf; j += NT_UP) xs[j] = Fa.v[bf + j];
    for (int j = tid; j < Rv; j += NT_UP) xs[Rf + j] = Ve.v[bv + j];
    __syncthreads();
    for (int k = tid; k < rf + rv; k += NT_UP) {
        if (k < rf) colsum<P::ordered>(Fa.Tr_rm + Fa.troff[g], Rf, rf, xs, Fa.v + cf, k);
        else colsum<P::ordered>(Ve.Tr_rm + Ve.troff[g], Rv, rv, xs + Rf, Ve.v + cv, k - rf);
    }
}

constexpr int NT_DN = 256; // L2L rows per box reach a few hundred

template <bool ORD, typename F>
__device__ __forceinline__ void l2l_family(const F &fam, const int32_t *cbeg, const int32_t *cend, int g, double *xs)
{
    const int c0 = fam.coef_off[g], r = fam.coef_off[g + 1] - c0;
    if (r == 0) return;
    const int cb = fam.coef_off[cbeg[g]], R = fam.coef_off[cend[g]] - cb;
    for (int k = threadIdx.x; k < r; k += NT_DN) xs[k] = fam.u[c0 + k];
    __syncthreads();
    const double *A = fam.Tr_cm + fam.troff[g];
    for (int j = threadIdx.x; j < R; j += NT_DN) {
        double s = 0.0;
        for (int k = 0; k < r; ++k) s = madd<ORD>(s, A[(size_t)k * R + j], xs[k]);
        fam.u[cb + j] = ORD ? __dadd_rn(fam.u[cb + j], s) : fam.u[cb + j] + s;
    }
    __syncthreads();
}

template <class P> __global__ __launch_bounds__(NT_DN) void k_l2l(DevTree<P> t, int32_t g0, uint32_t mask)
{
    extern __shared__ double xs[]; // largest rank
    const int g = g0 + blockIdx.x;
    if (mask & kFar) l2l_family<P::ordered>(t.far, t.box_cbeg, t.box_cend, g, xs);
    if (mask & kVer) l2l_family<P::ordered>(t.ver, t.box_cbeg, t.box_cend, g, xs);
}

// ---------------------------------------------------------------------------
// M2L: one target box per block.  Work item (a, Y): pivot a of X against
// source box Y, s_{aY} = sum_b K(t^{X,i}_a, t^{Y,i}_b) v_Y[b] in b order;
// then u_X[a] = sum_Y s_{aY} in list order.  Sources are staged in LDS a
// group of whole boxes at a time.
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
__global__ __launch_bounds__(NT_M2L) void k_m2l(DevTree<P> t)
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
    const int tid = threadIdx.x;
    const int g = F.targets[xcd_remap(blockIdx.x, gridDim.x)];
    const int c0 = F.coef_off[g], r = F.coef_off[g + 1] - c0;
    const int e0 = F.il_off[g], e1 = F.il_off[g + 1];
    const CT diag = (CT)t.diag, kp = (CT)t.kparam;
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
                for (int j = jb; j < je; ++j) {
                    const double r2 = dist2<ORD, D>((double)xa - (double)sx[j], (double)ya - (double)sy[j],
                                                    D == 3 ? (double)za - (double)sz[j] : 0.0);
                    s = madd<ORD>(s, kval<KIND>(r2, (double)diag, (double)kp), sv[j]);
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
                    uacc[o] = ORD ? __dadd_rn(uacc[o], part[yl * r + a]) : uacc[o] + part[yl * r + a];
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
// Leaf pass down: near field (source slices), L2P (in index order), the
// (H2+H)* vertex blocks, sum and scatter.
// ---------------------------------------------------------------------------
constexpr int NT_LEAF = 256;
constexpr int P2P_SRC = 1024; // staged source points per group

template <bool ORD, typename F>
__device__ __forceinline__ double l2p_family(const F &fam, int g, int leaf, int n, int i, int kappa)
{
    if (kappa < fam.lmin) return 0.0;
    const int c0 = fam.coef_off[g], r = fam.coef_off[g + 1] - c0;
    if (r == 0) return 0.0;
    const auto *U = fam.U_cm + fam.uoff[leaf];
    double s = 0.0;
    for (int k = 0; k < r; ++k) s = madd<ORD>(s, (double)U[(size_t)k * n + i], fam.u[c0 + k]);
    return s;
}

template <class P, int KIND, int D>
__global__ __launch_bounds__(NT_LEAF) void k_down_leaf(DevTree<P> t, double *__restrict__ y, uint32_t mask)
{
    using PT = typename P::pt_t;
    constexpr bool ORD = P::ordered;
    __shared__ PT sx[P2P_SRC], sy[P2P_SRC], sz[D == 3 ? P2P_SRC : 1], sq[P2P_SRC];
    __shared__ double red[NT_LEAF];
    const int tid = threadIdx.x;
    const int leaf = xcd_remap(blockIdx.x, gridDim.x), g = t.leaf0 + leaf;
    const int b = t.box_begin[g], n = t.box_end[g] - b;
    const PT diag = (PT)t.diag, kp = (PT)t.kparam;
    const double *cX = t.box_ctr + 3 * g;
    for (int i0 = 0; i0 < n; i0 += NT_LEAF) {
        const int m = min(n - i0, NT_LEAF), S = NT_LEAF / m, s = tid / m, i = i0 + tid % m;
        const PT xi = t.px[b + i], yi = t.py[b + i], zi = D == 3 ? t.pz[b + i] : PT(0);
        double acc = 0.0;
        if (mask & kNear) {
            int pos = 0;
            auto flush = [&]() {
                __syncthreads();
                if (s < S) {
                    PT part = 0;
                    for (int j = s; j < pos; j += S) {
                        const PT r2 = dist2<false, D>(xi - sx[j], yi - sy[j], zi - sz[D == 3 ? j : 0]);
                        part += kval<KIND>(r2, diag, kp) * sq[j];
                    }
                    acc += (double)part;
                }
                __syncthreads();
                pos = 0;
            };
            for (int e = t.near_off[leaf]; e < t.near_off[leaf + 1]; ++e) {
                const int gs = t.leaf0 + t.near_idx[e];
                const int sb = t.box_begin[gs], sn = t.box_end[gs] - sb;
                double dcx = 0, dcy = 0, dcz = 0;
                if constexpr (P::local) {
                    dcx = t.box_ctr[3 * gs] - cX[0];
                    dcy = t.box_ctr[3 * gs + 1] - cX[1];
                    dcz = t.box_ctr[3 * gs + 2] - cX[2];
                }
                for (int j0 = 0; j0 < sn;) {
                    const int take = min(sn - j0, P2P_SRC - pos);
                    for (int j = tid; j < take; j += NT_LEAF) {
                        const int src = sb + j0 + j;
                        if constexpr (P::local) {
                            sx[pos + j] = (PT)(dcx + (double)t.px[src]);
                            sy[pos + j] = (PT)(dcy + (double)t.py[src]);
                            if constexpr (D == 3) sz[pos + j] = (PT)(dcz + (double)t.pz[src]);
                        } else {
                            sx[pos + j] = t.px[src];
                            sy[pos + j] = t.py[src];
                            if constexpr (D == 3) sz[pos + j] = t.pz[src];
                        }
                        sq[pos + j] = (PT)t.qt[src];
                    }
                    pos += take;
                    j0 += take;
                    if (pos == P2P_SRC) flush();
                }
            }
            if (pos > 0) flush();
        }
        red[tid] = s < S ? acc : 0.0;
        __syncthreads();
        if (tid < m) {
            double phi = 0.0;
            for (int q = 0; q < S; ++q) phi += red[q * m + tid];
            if (mask & kNear) phi = madd<ORD>(phi, t.shift, t.qt[b + i]);
            if (mask & kFar) {
                const double f = l2p_family<ORD>(t.far, g, leaf, n, i, t.kappa);
                phi = ORD ? __dadd_rn(phi, f) : phi + f;
            }
            if (mask & kVer) {
                double v = l2p_family<ORD>(t.ver, g, leaf, n, i, t.kappa);
                if (t.variant == H2S_H2_PLUS_H) {
                    const auto &Pr = t.pairs;
                    for (int l = 1; l <= t.kappa; ++l) {
                        const int X = t.leaf_anc[(size_t)leaf * (t.kappa + 1) + l];
                        const int off = b + i - t.box_begin[X];
                        const int nX = t.box_end[X] - t.box_begin[X];
                        for (int e = Pr.recv_off[X]; e < Pr.recv_off[X + 1]; ++e) {
                            const int ps = Pr.recv[e], p = ps >> 1, side = ps & 1;
                            const int r = Pr.prank[p];
                            const auto *G = Pr.data + (side == 0 ? Pr.pu[p] : Pr.pv[p]);
                            const double *w = Pr.w + Pr.pw[p] + (size_t)side * r;
                            for (int k = 0; k < r; ++k) v = madd<ORD>(v, (double)G[(size_t)k * nX + off], w[k]);
                        }
                    }
                }
                phi = ORD ? __dadd_rn(phi, v) : phi + v;
            }
            y[t.perm[b + i]] = phi;
        }
        __syncthreads();
    }
}

template <class P, int KIND, int D>
hipError_t enqueue(const DevTree<P> &t, const int32_t *lev_off, const double *x, double *y, uint32_t mask,
                   hipStream_t s, const ProfileHook *prof)
{
    auto mark = [&](int cls, int end) {
        if (prof) prof->mark(prof->ctx, cls, end);
    };
    const size_t lds_leaf = sizeof(double) * (size_t)t.max_leaf;
    const size_t lds_rows = sizeof(double) * (size_t)(2 * t.max_rows);
    const size_t lds_rank = sizeof(double) * (size_t)t.max_rank;
    mark(H2S_PROF_LEAF_UP, 0);
    hipLaunchKernelGGL(k_up_leaf<P>, dim3(t.nleaf), dim3(NT_UP), lds_leaf, s, t, x, mask);
    mark(H2S_PROF_LEAF_UP, 1);
    const bool fam_on = (mask & (kFar | kVer)) && t.kappa >= 1;
    if (fam_on) {
        mark(H2S_PROF_M2M, 0);
        for (int l = t.kappa - 1; l >= 1; --l) {
            const int nb = lev_off[l + 1] - lev_off[l];
            if (nb) hipLaunchKernelGGL(k_m2m<P>, dim3(nb), dim3(NT_UP), lds_rows, s, t, lev_off[l], mask);
        }
        mark(H2S_PROF_M2M, 1);
        mark(H2S_PROF_M2L, 0);
        if ((mask & kFar) && t.far.ntargets)
            hipLaunchKernelGGL((k_m2l<P, true, KIND, D>), dim3(t.far.ntargets), dim3(NT_M2L), 0, s, t);
        if ((mask & kVer) && t.ver.ntargets)
            hipLaunchKernelGGL((k_m2l<P, false, KIND, D>), dim3(t.ver.ntargets), dim3(NT_M2L), 0, s, t);
        mark(H2S_PROF_M2L, 1);
        mark(H2S_PROF_L2L, 0);
        for (int l = 1; l <= t.kappa - 1; ++l) {
            const int nb = lev_off[l + 1] - lev_off[l];
            if (nb) hipLaunchKernelGGL(k_l2l<P>, dim3(nb), dim3(NT_DN), lds_rank, s, t, lev_off[l], mask);
        }
        mark(H2S_PROF_L2L, 1);
    }
    if (t.variant == H2S_H2_PLUS_H && (mask & kVer) && t.pairs.npairs) {
        mark(H2S_PROF_PAIR_PART, 0);
        hipLaunchKernelGGL(k_pair_part<P>, dim3(t.pairs.nchunks), dim3(256), 0, s, t);
        mark(H2S_PROF_PAIR_PART, 1);
        mark(H2S_PROF_PAIR_SUM, 0);
        hipLaunchKernelGGL(k_pair_sum<P>, dim3(2 * t.pairs.npairs), dim3(64), 0, s, t);
        mark(H2S_PROF_PAIR_SUM, 1);
    }
    mark(H2S_PROF_LEAF_DOWN, 0);
    hipLaunchKernelGGL((k_down_leaf<P, KIND, D>), dim3(t.nleaf), dim3(NT_LEAF), 0, s, t, y, mask);
    mark(H2S_PROF_LEAF_DOWN, 1);
    return hipGetLastError();
}

} // namespace

template <class P>
int launch_mvp(const DevTree<P> &t, const int32_t *lev_off, const double *x, double *y, uint32_t mask, void *stream,
               const ProfileHook *prof)
{
    hipStream_t s = (hipStream_t)stream;
    const int key = t.kind * 2 + (t.d == 3);
    switch (key) {
    case 0: return (int)enqueue<P, H2S_K_LOG_R, 2>(t, lev_off, x, y, mask, s, prof);
    case 1: return (int)enqueue<P, H2S_K_LOG_R, 3>(t, lev_off, x, y, mask, s, prof);
    case 2: return (int)enqueue<P, H2S_K_INV_R, 2>(t, lev_off, x, y, mask, s, prof);
    case 3: return (int)enqueue<P, H2S_K_INV_R, 3>(t, lev_off, x, y, mask, s, prof);
    case 4: return (int)enqueue<P, H2S_K_GAUSSIAN, 2>(t, lev_off, x, y, mask, s, prof);
    case 5: return (int)enqueue<P, H2S_K_GAUSSIAN, 3>(t, lev_off, x, y, mask, s, prof);
    case 6: return (int)enqueue<P, H2S_K_EXP_R, 2>(t, lev_off, x, y, mask, s, prof);
    default: return (int)enqueue<P, H2S_K_EXP_R, 3>(t, lev_off, x, y, mask, s, prof);
    }
}

template int launch_mvp<P64>(const DevTree<P64> &, const int32_t *, const double *, double *, uint32_t, void *,
                             const ProfileHook *);
template int launch_mvp<P32>(const DevTree<P32> &, const int32_t *, const double *, double *, uint32_t, void *,
                             const ProfileHook *);
template int launch_mvp<P32M>(const DevTree<P32M> &, const int32_t *, const double *, double *, uint32_t, void *,
                              const ProfileHook *);

} // namespace h2s
