// h2s_kernels.hip -- HIP kernels of the H2* / (H2+H)* matrix-vector product
// for CDNA4 (gfx950), Khan & Ambikasaran (arXiv 2309.14085), Sec. 5.1.2 and
// Sec. 5.2.2:
//
//   k_leaf_up     charges to tree order + P2M at the leaves   v_X = U_X^T q_X
//   k_m2m         one level of the upward pass               v_X = sum_c U~_{X_c X}^T v_{X_c}
//   k_m2l         all levels, all boxes                      u_X = sum_{Y in IL(X)} K(t^{X,i}, t^{Y,i}) v_Y
//   k_l2l         one level of the downward pass             u_{X_c} += U~_{X_c X} u_X
//   k_pair_part   (H2+H)*: partial products Vb^T q_Y, Ub^T q_X over row chunks
//   k_pair_sum    (H2+H)*: chunk sums in a fixed order
//   k_leaf_down   L2P U_X u_X for both families, (H2+H)* vertex blocks, the
//                 direct near field over N*(X) and the scatter to user order
//
// Every kernel is one 64-lane wavefront per work item.  M2L and the near field
// evaluate the kernel on the fly: source coordinates (and coefficients or
// charges) are staged through LDS 64 at a time and each lane owns one target.
// No floating-point atomics are used, so results are reproducible run to run.
#include <hip/hip_runtime.h>

#include "h2s.h"
#include "h2s_device.hpp"

namespace h2s {

namespace {

constexpr unsigned kNear = 1u, kFar = 2u, kVer = 4u;

template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Kernel value from the squared distance; r2 == 0 means coincident points.
template <int KIND> __device__ __forceinline__ double kval(double r2, double diag, double kp)
{
    double v;
    if constexpr (KIND == H2S_K_LOG_R) v = 0.5 * log(r2);
    else if constexpr (KIND == H2S_K_INV_R) v = 1.0 / sqrt(r2);
    else if constexpr (KIND == H2S_K_GAUSSIAN) v = exp(-r2 * kp);
    else v = exp(-sqrt(r2));
    return r2 == 0.0 ? diag : v;
}

template <int KIND> __device__ __forceinline__ float kval(float r2, float diag, float kp)
{
    float v;
    if constexpr (KIND == H2S_K_LOG_R) v = __log2f(r2) * 0.34657359027997264f; // ln 2 / 2
    else if constexpr (KIND == H2S_K_INV_R) v = __frsqrt_rn(r2);
    else if constexpr (KIND == H2S_K_GAUSSIAN) v = __expf(-r2 * kp);
    else v = __expf(-__fsqrt_rn(r2));
    return r2 == 0.0f ? diag : v;
}

// FP64 stores absolute coordinates (the centre difference is 0).  FP32 stores
// offsets from box centres; the difference of two centres is taken in double
// and rounded once, so close pairs keep their relative accuracy.
template <typename T>
__device__ __forceinline__ void centre_diff(const DevTree<T> &t, int32_t gx, int32_t gy, T &cx, T &cy, T &cz)
{
    if constexpr (sizeof(T) == 8) {
        cx = cy = cz = 0;
    } else {
        cx = (T)(t.box_ctr[3 * gx] - t.box_ctr[3 * gy]);
        cy = (T)(t.box_ctr[3 * gx + 1] - t.box_ctr[3 * gy + 1]);
        cz = (T)(t.box_ctr[3 * gx + 2] - t.box_ctr[3 * gy + 2]);
    }
}

template <typename T>
__global__ __launch_bounds__(64) void k_leaf_up(DevTree<T> t, const double *__restrict__ x, uint32_t mask)
{
    const int leaf = blockIdx.x, g = t.leaf0 + leaf, lane = threadIdx.x;
    const int b = t.box_begin[g], n = t.box_end[g] - b;
    for (int i = lane; i < n; i += 64) t.qt[b + i] = (T)x[t.perm[b + i]];
    // each lane reads back only the charges it wrote itself
    for (int f = 0; f < 2; ++f) {
        if (!(mask & (f == 0 ? kFar : kVer))) continue;
        const DevFamily<T> &F = t.fam[f];
        if (t.kappa < F.lmin) continue;
        const int c0 = F.coef_off[g], r = F.coef_off[g + 1] - c0;
        if (r == 0) continue;
        const T *U = F.U + F.uoff[leaf];
        for (int k = 0; k < r; ++k) {
            T s = 0;
            for (int i = lane; i < n; i += 64) s += U[(size_t)k * n + i] * t.qt[b + i];
            s = wave_sum(s);
            if (lane == 0) F.v[c0 + k] = s;
        }
    }
}

template <typename T> __global__ __launch_bounds__(64) void k_m2m(DevTree<T> t, int32_t g0, uint32_t mask)
{
    const int f = blockIdx.y;
    if (!(mask & (f == 0 ? kFar : kVer))) return;
    const DevFamily<T> &F = t.fam[f];
    const int g = g0 + blockIdx.x;
    const int c0 = F.coef_off[g], r = F.coef_off[g + 1] - c0;
    if (r == 0) return;
    const int cb = F.coef_off[t.box_cbeg[g]], rows = F.coef_off[t.box_cend[g]] - cb;
    const T *Tr = F.Tr + F.troff[g];
    for (int k = threadIdx.x; k < r; k += 64) {
        T s = 0;
        for (int j = 0; j < rows; ++j) s += Tr[(size_t)j * r + k] * F.v[cb + j];
        F.v[c0 + k] = s;
    }
}

template <typename T, int KIND, int D>
__global__ __launch_bounds__(64) void k_m2l(DevTree<T> t, uint32_t mask)
{
    int idx = blockIdx.x, f = 0;
    if (idx >= t.fam[0].ntargets) {
        idx -= t.fam[0].ntargets;
        f = 1;
    }
    if (!(mask & (f == 0 ? kFar : kVer))) return;
    const DevFamily<T> &F = t.fam[f];
    const int g = F.targets[idx];
    const int c0 = F.coef_off[g], r = F.coef_off[g + 1] - c0;
    const int lane = threadIdx.x;
    __shared__ T sx[64], sy[64], sz[64], sv[64];
    const T diag = (T)t.diag, kp = (T)t.kparam;
    for (int k0 = 0; k0 < r; k0 += 64) {
        const int k = k0 + lane;
        const bool act = k < r;
        const T xi = act ? F.pvx[c0 + k] : T(0);
        const T yi = act ? F.pvy[c0 + k] : T(0);
        const T zi = (D == 3 && act) ? F.pvz[c0 + k] : T(0);
        T acc = 0;
        for (int e = F.il_off[g]; e < F.il_off[g + 1]; ++e) {
            const int y = F.il_idx[e];
            const int cy = F.coef_off[y], ry = F.coef_off[y + 1] - cy;
            T cdx, cdy, cdz;
            centre_diff(t, g, y, cdx, cdy, cdz);
            for (int j0 = 0; j0 < ry; j0 += 64) {
                __syncthreads();
                if (j0 + lane < ry) {
                    sx[lane] = F.pvx[cy + j0 + lane];
                    sy[lane] = F.pvy[cy + j0 + lane];
                    if (D == 3) sz[lane] = F.pvz[cy + j0 + lane];
                    sv[lane] = F.v[cy + j0 + lane];
                }
                __syncthreads();
                const int nj = min(64, ry - j0);
                for (int j = 0; j < nj; ++j) {
                    const T dx = cdx + (xi - sx[j]), dy = cdy + (yi - sy[j]);
                    T r2 = dx * dx + dy * dy;
                    if (D == 3) {
                        const T dz = cdz + (zi - sz[j]);
                        r2 += dz * dz;
                    }
                    acc += kval<KIND>(r2, diag, kp) * sv[j];
                }
            }
        }
        if (act) F.u[c0 + k] = acc;
    }
}

template <typename T> __global__ __launch_bounds__(64) void k_l2l(DevTree<T> t, int32_t g0, uint32_t mask)
{
    const int f = blockIdx.y;
    if (!(mask & (f == 0 ? kFar : kVer))) return;
    const DevFamily<T> &F = t.fam[f];
    const int g = g0 + blockIdx.x;
    const int c0 = F.coef_off[g], r = F.coef_off[g + 1] - c0;
    if (r == 0) return;
    const int cb = F.coef_off[t.box_cbeg[g]], rows = F.coef_off[t.box_cend[g]] - cb;
    const T *Tr = F.Tr + F.troff[g];
    for (int j = threadIdx.x; j < rows; j += 64) {
        const T *row = Tr + (size_t)j * r;
        T s = 0;
        for (int k = 0; k < r; ++k) s += row[k] * F.u[c0 + k];
        F.u[cb + j] += s;
    }
}

// (H2+H)*: partial sums over one row chunk of G^T q, with G = Vb over the
// rows of Y (side 0: w = Vb^T q_Y) or G = Ub over the rows of X (side 1:
// w' = Ub^T q_X).
template <typename T> __global__ __launch_bounds__(64) void k_pair_part(DevTree<T> t)
{
    const DevPairs<T> &P = t.pairs;
    const int c = blockIdx.x, lane = threadIdx.x;
    const int p = P.chunk_pair[c], side = P.chunk_side[c];
    const int r = P.prank[p];
    const int box = side == 0 ? P.py[p] : P.px[p];
    const int nrows = t.box_end[box] - t.box_begin[box];
    const T *G = P.data + (side == 0 ? P.pv[p] : P.pu[p]);
    const T *q = t.qt + t.box_begin[box];
    const int r0 = P.chunk_begin[c], r1 = r0 + P.chunk_len[c];
    T *out = P.partial + P.chunk_poff[c];
    for (int k = 0; k < r; ++k) {
        T s = 0;
        for (int i = r0 + lane; i < r1; i += 64) s += G[(size_t)k * nrows + i] * q[i];
        s = wave_sum(s);
        if (lane == 0) out[k] = s;
    }
}

template <typename T> __global__ __launch_bounds__(64) void k_pair_sum(DevTree<T> t)
{
    const DevPairs<T> &P = t.pairs;
    const int ps = blockIdx.x, p = ps >> 1, side = ps & 1;
    const int r = P.prank[p];
    const int c0 = P.side_chunk_off[ps], c1 = P.side_chunk_off[ps + 1];
    T *w = P.w + P.pw[p] + (size_t)side * r;
    for (int k = threadIdx.x; k < r; k += 64) {
        T s = 0;
        for (int c = c0; c < c1; ++c) s += P.partial[P.chunk_poff[c] + k];
        w[k] = s;
    }
}

template <typename T, int KIND, int D>
__global__ __launch_bounds__(64) void k_leaf_down(DevTree<T> t, double *__restrict__ y, uint32_t mask)
{
    const int leaf = blockIdx.x, g = t.leaf0 + leaf, lane = threadIdx.x;
    const int b = t.box_begin[g], n = t.box_end[g] - b;
    __shared__ T sx[64], sy[64], sz[64], sq[64];
    const T diag = (T)t.diag, kp = (T)t.kparam;
    for (int i0 = 0; i0 < n; i0 += 64) {
        const int i = i0 + lane;
        const bool act = i < n;
        T phi = 0;
        if (mask & kNear) {
            const T xi = act ? t.px[b + i] : T(0);
            const T yi = act ? t.py[b + i] : T(0);
            const T zi = (D == 3 && act) ? t.pz[b + i] : T(0);
            for (int e = t.near_off[leaf]; e < t.near_off[leaf + 1]; ++e) {
                const int gs = t.leaf0 + t.near_idx[e];
                const int sb = t.box_begin[gs], sn = t.box_end[gs] - sb;
                T cdx, cdy, cdz;
                centre_diff(t, g, gs, cdx, cdy, cdz);
                for (int j0 = 0; j0 < sn; j0 += 64) {
                    __syncthreads();
                    if (j0 + lane < sn) {
                        sx[lane] = t.px[sb + j0 + lane];
                        sy[lane] = t.py[sb + j0 + lane];
                        if (D == 3) sz[lane] = t.pz[sb + j0 + lane];
                        sq[lane] = t.qt[sb + j0 + lane];
                    }
                    __syncthreads();
                    const int nj = min(64, sn - j0);
                    for (int j = 0; j < nj; ++j) {
                        const T dx = cdx + (xi - sx[j]), dy = cdy + (yi - sy[j]);
                        T r2 = dx * dx + dy * dy;
                        if (D == 3) {
                            const T dz = cdz + (zi - sz[j]);
                            r2 += dz * dz;
                        }
                        phi += kval<KIND>(r2, diag, kp) * sq[j];
                    }
                }
            }
            if (act) phi += (T)t.shift * t.qt[b + i];
        }
        if (act) {
            for (int f = 0; f < 2; ++f) {
                if (!(mask & (f == 0 ? kFar : kVer))) continue;
                const DevFamily<T> &F = t.fam[f];
                if (t.kappa < F.lmin) continue;
                const int c0 = F.coef_off[g], r = F.coef_off[g + 1] - c0;
                const T *U = F.U + (r ? F.uoff[leaf] : 0);
                for (int k = 0; k < r; ++k) phi += U[(size_t)k * n + i] * F.u[c0 + k];
            }
            if (t.variant == H2S_H2_PLUS_H && (mask & kVer)) {
                const DevPairs<T> &P = t.pairs;
                for (int l = 1; l <= t.kappa; ++l) {
                    const int X = t.leaf_anc[(size_t)leaf * (t.kappa + 1) + l];
                    const int off = b + i - t.box_begin[X];
                    const int nX = t.box_end[X] - t.box_begin[X];
                    for (int e = P.recv_off[X]; e < P.recv_off[X + 1]; ++e) {
                        const int ps = P.recv[e], p = ps >> 1, side = ps & 1;
                        const int r = P.prank[p];
                        const T *G = P.data + (side == 0 ? P.pu[p] : P.pv[p]);
                        const T *w = P.w + P.pw[p] + (size_t)side * r;
                        for (int k = 0; k < r; ++k) phi += G[(size_t)k * nX + off] * w[k];
                    }
                }
            }
            y[t.perm[b + i]] = (double)phi;
        }
    }
}

template <typename T, int KIND, int D>
hipError_t enqueue(const DevTree<T> &t, const int32_t *lev_off, const double *x, double *y, uint32_t mask,
                   hipStream_t s, const ProfileHook *prof)
{
    auto mark = [&](int cls, int end) {
        if (prof) prof->mark(prof->ctx, cls, end);
    };
    mark(H2S_PROF_LEAF_UP, 0);
    hipLaunchKernelGGL(k_leaf_up<T>, dim3(t.nleaf), dim3(64), 0, s, t, x, mask);
    mark(H2S_PROF_LEAF_UP, 1);
    const bool fam_on = (mask & (kFar | kVer)) && t.kappa >= 1;
    if (fam_on) {
        mark(H2S_PROF_M2M, 0);
        for (int l = t.kappa - 1; l >= 1; --l) {
            const int nb = lev_off[l + 1] - lev_off[l];
            if (nb) hipLaunchKernelGGL(k_m2m<T>, dim3(nb, 2), dim3(64), 0, s, t, lev_off[l], mask);
        }
        mark(H2S_PROF_M2M, 1);
        const int nt = t.fam[0].ntargets + t.fam[1].ntargets;
        mark(H2S_PROF_M2L, 0);
        if (nt) hipLaunchKernelGGL((k_m2l<T, KIND, D>), dim3(nt), dim3(64), 0, s, t, mask);
        mark(H2S_PROF_M2L, 1);
        mark(H2S_PROF_L2L, 0);
        for (int l = 1; l <= t.kappa - 1; ++l) {
            const int nb = lev_off[l + 1] - lev_off[l];
            if (nb) hipLaunchKernelGGL(k_l2l<T>, dim3(nb, 2), dim3(64), 0, s, t, lev_off[l], mask);
        }
        mark(H2S_PROF_L2L, 1);
    }
    if (t.variant == H2S_H2_PLUS_H && (mask & kVer) && t.pairs.npairs) {
        mark(H2S_PROF_PAIR_PART, 0);
        hipLaunchKernelGGL(k_pair_part<T>, dim3(t.pairs.nchunks), dim3(64), 0, s, t);
        mark(H2S_PROF_PAIR_PART, 1);
        mark(H2S_PROF_PAIR_SUM, 0);
        hipLaunchKernelGGL(k_pair_sum<T>, dim3(2 * t.pairs.npairs), dim3(64), 0, s, t);
        mark(H2S_PROF_PAIR_SUM, 1);
    }
    mark(H2S_PROF_LEAF_DOWN, 0);
    hipLaunchKernelGGL((k_leaf_down<T, KIND, D>), dim3(t.nleaf), dim3(64), 0, s, t, y, mask);
    mark(H2S_PROF_LEAF_DOWN, 1);
    return hipGetLastError();
}

} // namespace

template <typename T>
int launch_mvp(const DevTree<T> &t, const int32_t *lev_off, const double *x, double *y, uint32_t mask,
               void *stream, const ProfileHook *prof)
{
    hipStream_t s = (hipStream_t)stream;
    const int key = t.kind * 2 + (t.d == 3);
    switch (key) {
    case 0: return (int)enqueue<T, H2S_K_LOG_R, 2>(t, lev_off, x, y, mask, s, prof);
    case 1: return (int)enqueue<T, H2S_K_LOG_R, 3>(t, lev_off, x, y, mask, s, prof);
    case 2: return (int)enqueue<T, H2S_K_INV_R, 2>(t, lev_off, x, y, mask, s, prof);
    case 3: return (int)enqueue<T, H2S_K_INV_R, 3>(t, lev_off, x, y, mask, s, prof);
    case 4: return (int)enqueue<T, H2S_K_GAUSSIAN, 2>(t, lev_off, x, y, mask, s, prof);
    case 5: return (int)enqueue<T, H2S_K_GAUSSIAN, 3>(t, lev_off, x, y, mask, s, prof);
    case 6: return (int)enqueue<T, H2S_K_EXP_R, 2>(t, lev_off, x, y, mask, s, prof);
    default: return (int)enqueue<T, H2S_K_EXP_R, 3>(t, lev_off, x, y, mask, s, prof);
    }
}

template int launch_mvp<double>(const DevTree<double> &, const int32_t *, const double *, double *, uint32_t, void *,
                                const ProfileHook *);
template int launch_mvp<float>(const DevTree<float> &, const int32_t *, const double *, double *, uint32_t, void *,
                               const ProfileHook *);

} // namespace h2s
