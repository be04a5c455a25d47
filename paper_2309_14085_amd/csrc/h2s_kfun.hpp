// h2s_kfun.hpp -- device helpers shared by the product kernels
// (h2s_kernels.hip, h2s_kernels_batch.hip): phase masks, the XCD block
// remap, separately rounded multiply-add, the FP64 kernel functions (table-
// driven log and exp, Newton-refined 1/sqrt), the kernel value from a squared
// distance, wavefront sums and the pipelined ordered dot product.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "h2s.h"

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

// The same for items of uneven cost sorted by cost class (M2L targets: coarse
// levels first, their boxes several times the work of a leaf's): the items
// are cut into chunks of C, and chunk c goes to XCD c mod 8, so each XCD gets
// Morton-local runs of C items from every part of the range.  Block bid = 8 j
// + x (XCD x) takes item (8 (j / C) + x) C + j mod C while whole rows of 8
// chunks remain; the items of the last, partial row map to themselves.  A
// bijection of [0, nb).
constexpr int kM2LChunk = 32; // the run length the M2L kernels use
template <int C> __device__ __forceinline__ int xcd_chunk_remap(int bid, int nb)
{
    const int rows = nb / (8 * C);
    if (bid >= rows * 8 * C) return bid;
    const int x = bid & 7, j = bid >> 3;
    return (8 * (j / C) + x) * C + j % C;
}

// s + a b.  ORD: the product and the sum rounded separately, as a plain
// sequential evaluation does (the HBM-bound sums can afford it); otherwise
// one fused multiply-add.
template <bool ORD> __device__ __forceinline__ double madd(double s, double a, double b)
{
    if constexpr (ORD) {
#pragma clang fp contract(off)
        const double p = a * b;
        return s + p;
    } else {
        return fma(a, b, s);
    }
}

// 0.5 ln(x) for finite x > 0 in double, table-driven (Tang's reduction):
// x = m 2^e with m in [1/2, 1) (frexp); the top 8 fraction bits of m select
// a subinterval i of width 1/512 with centre z_i, c_i ~ 1/z_i; then
// r = m c_i - 1 (|r| < 2^-9, one rounding) and
//   0.5 ln x = 0.5 e ln 2 - 0.5 ln c_i + 0.5 ln(1 + r),
// the last term by its Taylor series through r^5 (truncation below 1e-17).
// tab holds (c_i, -0.5 ln c_i) for the 256 subintervals (built on the host
// in extended precision).  Absolute error about one ulp of the result.
__device__ __forceinline__ double half_log(double x, const double2 *tab)
{
    int e;
    const double m = frexp(x, &e);
    const int i = (__double2hiint(m) >> 12) & 255;
    const double2 c = tab[i];
    const double r = fma(m, c.x, -1.0);
    double p = 1.0 / 10;
    p = fma(p, r, -1.0 / 8);
    p = fma(p, r, 1.0 / 6);
    p = fma(p, r, -1.0 / 4);
    p = fma(p, r, 1.0 / 2);
    return fma(r, p, fma((double)e, 0.34657359027997264, c.y)); // ln 2 / 2
}

// The same logarithm rounded almost always correctly, for the M2L sums, whose
// result the interpolation operators amplify: ln 2 / 2 = Lh + Ll and
// -0.5 ln c_i = Th_i + Tl_i with Lh and Th_i multiples of 2^-43 (Lh has 42
// significant bits), so e Lh + Th_i is exact for |e| < 2^10; the small rest
// e Ll + Tl_i + 0.5 ln(1 + r) carries an absolute error near 2e-19, and the
// one final addition rounds.  tab[256 + i] holds (Th_i, Tl_i).
__device__ __forceinline__ double half_log_acc(double x, const double2 *tab)
{
    constexpr double kLh = 0x1.62e42fefa3800p-2, kLl = 0x1.ef35793c76730p-46;
    int e;
    const double m = frexp(x, &e);
    const int i = (__double2hiint(m) >> 12) & 255;
    const double2 c = tab[i], th = tab[256 + i];
    const double r = fma(m, c.x, -1.0);
    double p = 1.0 / 10;
    p = fma(p, r, -1.0 / 8);
    p = fma(p, r, 1.0 / 6);
    p = fma(p, r, -1.0 / 4);
    p = fma(p, r, 1.0 / 2);
    const double ed = (double)e;
    double hi, lo;
    {
#pragma clang fp contract(off) // e Lh + Th is exact only as a separate product and sum
        hi = ed * kLh + th.x;
    }
    lo = fma(r, p, fma(ed, kLl, th.y));
    return hi + lo;
}

// exp(x) in double, table-driven (Tang's reduction): k = nearest integer to
// 64 x / ln 2, r = x - k ln2/64 (|r| <= ln2/128, with ln2/64 split into an
// exactly multipliable head and a tail), k = 64 m + j, and
//   exp(x) = 2^m 2^(j/64) exp(r),
// exp(r) by its Taylor series through r^6 (truncation below 3e-20).  tab
// holds 2^(j/64), j < 64 (extended precision on the host).  Arguments below
// -1000 are clamped (the result is 0 in double either way).  Relative error
// about two ulps.
__device__ __forceinline__ double exp_tab(double x, const double *tab)
{
    x = fmax(x, -1000.0);
    const double kd = rint(x * 92.332482616893656877); // 64 / ln 2
    const int k = (int)kd;
    double r = fma(-kd, 0.010830417275428772, x);     // head of ln2/64
    r = fma(-kd, 7.420820373487167e-09, r);           // tail of ln2/64
    double p = 1.0 / 720;
    p = fma(p, r, 1.0 / 120);
    p = fma(p, r, 1.0 / 24);
    p = fma(p, r, 1.0 / 6);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(tab[k & 63] * p, k >> 6);
}

// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton steps
// y <- y + y (1 - x y^2) / 2.  Relative error about one ulp.
__device__ __forceinline__ double inv_sqrt(double x)
{
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double t = x * y;
        const double e = fma(-t, y, 1.0);
        y = fma(y * 0.5, e, y);
    }
    return y;
}

// Lookup tables of the kernel functions, in doubles: log r and the log RBF
// 256 pairs (c_i, -0.5 ln c_i) followed by 256 pairs (Th_i, Tl_i), the
// exponential kernels 2^(j/64).  Staged in LDS per block.
template <int KIND>
constexpr int kTabLen = KIND == H2S_K_LOG_R || KIND == H2S_K_RBF_LOG
                            ? 512
                            : (KIND == H2S_K_GAUSSIAN || KIND == H2S_K_EXP_R ? 64 : 2);
// With the (Th_i, Tl_i) pairs of the accurate logarithm behind.
template <int KIND>
constexpr int kTabLenAcc = KIND == H2S_K_LOG_R || KIND == H2S_K_RBF_LOG ? 1024 : kTabLen<KIND>;

// Stage the first LEN doubles of the table in LDS (whole block; the caller
// synchronises).
template <int KIND, int LEN = kTabLen<KIND>> __device__ __forceinline__ void stage_table(const double *g, double *tab)
{
    if constexpr (KIND != H2S_K_INV_R && KIND != H2S_K_RBF_AR)
        for (int i = threadIdx.x; i < LEN; i += blockDim.x) tab[i] = g[i];
}

// Kernels of an extra per-point coordinate w besides the position: the NTI
// multiquadric stages w = c(x) = exp(-(x_1 + x_3)) with the coordinates and
// adds (w_x - w_y)^2 to r^2.
template <int KIND> constexpr bool kExtraCoord = KIND == H2S_K_NTI_MQ;

template <int KIND, typename T> __device__ __forceinline__ T add_extra(T r2, T wa, T wb)
{
    if constexpr (kExtraCoord<KIND>) {
        const T dw = wa - wb;
        return r2 + dw * dw;
    } else {
        return r2;
    }
}

// Scalar parameters of the kernel function (uniform over the grid, so they
// live in scalar registers): kp = -1/h^2 for the Gaussian; for the piecewise
// RBFs of radius a, c0 = a^2 and the branch factors c1, c2 (a, 1/a for
// a/r | r/a; 1/log a, 1/(a log a - 1) for log r | r log r - 1).
template <typename T> struct KPar {
    T kp, c0, c1, c2;
};

template <typename T, class Tree> __device__ __forceinline__ KPar<T> kpar(const Tree &t)
{
    return KPar<T>{(T)t.kparam, (T)t.kc[0], (T)t.kc[1], (T)t.kc[2]};
}

// Squared distance (ORD is accepted for symmetry with madd).
template <bool ORD, int D, typename T> __device__ __forceinline__ T dist2(T dx, T dy, T dz)
{
    T r2 = dx * dx + dy * dy;
    if constexpr (D == 3) r2 += dz * dz;
    return r2;
}

// Kernel value from a squared distance r2 > 0.  The branch of the piecewise
// RBFs is taken on r2 >= a^2 (the functions are continuous at r = a).
template <int KIND, bool ACC = false>
__device__ __forceinline__ double kval_pos(double r2, const KPar<double> &kp, const double *tab)
{
    if constexpr (KIND == H2S_K_LOG_R && ACC) return half_log_acc(r2, (const double2 *)tab);
    else if constexpr (KIND == H2S_K_LOG_R) return half_log(r2, (const double2 *)tab);
    else if constexpr (KIND == H2S_K_INV_R) return inv_sqrt(r2);
    else if constexpr (KIND == H2S_K_GAUSSIAN) return exp_tab(r2 * kp.kp, tab);
    else if constexpr (KIND == H2S_K_EXP_R) return exp_tab(-sqrt(r2), tab);
    else if constexpr (KIND == H2S_K_RBF_AR) {
        const double rs = inv_sqrt(r2); // 1/r
        return r2 >= kp.c0 ? kp.c1 * rs : (r2 * rs) * kp.c2;
    } else if constexpr (KIND == H2S_K_RBF_LOG) {
        const double lr = ACC ? half_log_acc(r2, (const double2 *)tab) : half_log(r2, (const double2 *)tab); // log r
        return r2 >= kp.c0 ? lr * kp.c1 : fma(sqrt(r2), lr, -1.0) * kp.c2;
    } else { // H2S_K_NTI_MQ: r2 already holds |x - y|^2 + (c(x) - c(y))^2
        const double t = r2 + 1.0;
        return t * sqrt(t);
    }
}

// Kernel value from the squared distance; r2 == 0 means coincident points.
template <int KIND>
__device__ __forceinline__ double kval(double r2, double diag, const KPar<double> &kp, const double *tab)
{
    const double v = kval_pos<KIND>(r2, kp, tab);
    return r2 == 0.0 ? diag : v;
}

template <int KIND> __device__ __forceinline__ float kval(float r2, float diag, const KPar<float> &kp)
{
    float v;
    if constexpr (KIND == H2S_K_LOG_R) v = __log2f(r2) * 0.34657359027997264f; // ln 2 / 2
    else if constexpr (KIND == H2S_K_INV_R) v = __frsqrt_rn(r2);
    else if constexpr (KIND == H2S_K_GAUSSIAN) v = __expf(r2 * kp.kp);
    else if constexpr (KIND == H2S_K_EXP_R) v = __expf(-__fsqrt_rn(r2));
    else if constexpr (KIND == H2S_K_RBF_AR) {
        const float rs = __frsqrt_rn(r2);
        v = r2 >= kp.c0 ? kp.c1 * rs : (r2 * rs) * kp.c2;
    } else if constexpr (KIND == H2S_K_RBF_LOG) {
        const float lr = __log2f(r2) * 0.34657359027997264f;
        v = r2 >= kp.c0 ? lr * kp.c1 : fmaf(__fsqrt_rn(r2), lr, -1.0f) * kp.c2;
    } else {
        const float t = r2 + 1.0f;
        v = t * __fsqrt_rn(t);
    }
    return r2 == 0.0f ? diag : v;
}

// Exclusive prefix sum of one value per thread over a block of NT threads (wave
// scans by shuffles, then the waves' totals); wsum: NT / 64 ints of LDS.  All
// threads must call it; it ends with the block synchronised.
template <int NT> __device__ __forceinline__ int block_excl_scan(int v, int *wsum, int &total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        const int sw = wsum[w];
        before += w < wave ? sw : 0;
        total += sw;
    }
    return before + x - v;
}

template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Error-free transformations (Ogita, Rump and Oishi, "Accurate sum and dot
// product", 2005) on an unevaluated pair (s, c), the value s + c:
// (s, c) += a b -- the product's rounding error from an fma, the addition's
// from TwoSum, both gathered in c.
__device__ __forceinline__ void dot2_add(double &s, double &c, double a, double b)
{
#pragma clang fp contract(off) // the error terms need the separately rounded product and sums
    const double p = a * b, ep = fma(a, b, -p);
    const double t = s + p, z = t - s, es = (s - (t - z)) + (p - z);
    s = t;
    c += ep + es;
}

// (s, c) += (h, l)
__device__ __forceinline__ void dd_add(double &s, double &c, double h, double l)
{
#pragma clang fp contract(off)
    const double t = s + h, z = t - s, es = (s - (t - z)) + (h - z);
    s = t;
    c += es + l;
}

// Dot product init + sum_j a(j) x[j], a(j) = A[j stride], with qp added just
// before term pos (pos == R: after the last; pos < 0: never), in index order.
// ORD (the FP64 path): an accurate dot product -- the sum as if taken in
// twice the working precision, rounded once -- because the interpolation
// operators (norms up to ~1e3 - 1e4 on coarse levels) amplify the rounding
// error of a plain sum, eps sum |a x|, into the potential; otherwise plain
// fused multiply-adds.  The operator loads are software-pipelined two
// batches of UNR deep so that a batch is in flight while the previous one is
// accumulated.
constexpr int UNR = 4;

template <bool ORD, typename AT>
__device__ __forceinline__ double ordered_dot(const AT *__restrict__ A, size_t stride, int R, const double *xs,
                                              int pos = -1, double qp = 0.0, double init = 0.0)
{
    double s = init, c = 0.0;
    auto step = [&](int j, double a) {
        if constexpr (ORD) {
            if (j == pos) dd_add(s, c, qp, 0.0);
            dot2_add(s, c, a, xs[j]);
        } else {
            s = fma(a, xs[j], j == pos ? s + qp : s);
        }
    };
    int j = 0;
    if (R >= 2 * UNR) {
        double a[UNR], b[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) a[u] = (double)A[(size_t)u * stride];
        for (; j + 3 * UNR <= R; j += 2 * UNR) {
#pragma unroll
            for (int u = 0; u < UNR; ++u) b[u] = (double)A[(size_t)(j + UNR + u) * stride];
#pragma unroll
            for (int u = 0; u < UNR; ++u) step(j + u, a[u]);
#pragma unroll
            for (int u = 0; u < UNR; ++u) a[u] = (double)A[(size_t)(j + 2 * UNR + u) * stride];
#pragma unroll
            for (int u = 0; u < UNR; ++u) step(j + UNR + u, b[u]);
        }
        // a holds rows j .. j + UNR - 1 (fewer than 3 UNR rows were left)
#pragma unroll
        for (int u = 0; u < UNR; ++u) step(j + u, a[u]);
        j += UNR;
    }
    // the remaining rows, one predicated batch of loads at a time
    for (; j < R; j += UNR) {
        double c[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) c[u] = j + u < R ? (double)A[(size_t)(j + u) * stride] : 0.0;
#pragma unroll
        for (int u = 0; u < UNR; ++u)
            if (j + u < R) step(j + u, c[u]);
    }
    if (pos == R) {
        if constexpr (ORD) dd_add(s, c, qp, 0.0);
        else s += qp;
    }
    return ORD ? s + c : s;
}

} // namespace
} // namespace h2s
