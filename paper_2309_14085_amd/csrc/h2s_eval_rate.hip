// h2s_eval_rate.hip -- register-resident peak rate of the kernel function.
//
// The roofline of the evaluation-bound phases (near field and M2L, whose
// kernel values are computed on the fly) needs the rate at which the chip can
// evaluate the same kernel formula when nothing else limits it.  Each thread
// keeps 4 targets and 8 sources (coordinates and charges) in registers and
// sums K(x_a, y_b) q_b over them pass after pass, moving the sources by a tiny
// step per pass so that no pass repeats the last; the lookup table of the
// table-driven functions sits in LDS exactly as in the product kernels.
#include <hip/hip_runtime.h>

#include "h2s_eval_rate.hpp"
#include "h2s_kfun.hpp"

namespace h2s {
namespace {

constexpr int kTargets = 4, kSources = 8, kThreads = 256;

__device__ __forceinline__ double unit_hash(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return (double)x * (1.0 / 4294967296.0); // [0, 1)
}

template <typename T, int KIND, int D>
__global__ __launch_bounds__(kThreads) void k_eval_rate(const double *__restrict__ ktab_g, KPar<double> kp64,
                                                        double step, int passes, double *__restrict__ out)
{
    __shared__ __align__(16) double ktab[kTabLen<KIND>];
    stage_table<KIND>(ktab_g, ktab);
    __syncthreads();
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    // targets in [-1, 1]^d, sources in [1, 3] x [-1, 1]^(d-1): every distance is at least 0
    // and spreads over (0, ~4.5], so table indices differ from lane to lane as in the product
    T xa[kTargets], ya[kTargets], za[kTargets], wa[kTargets], acc[kTargets];
    T xs[kSources], ys[kSources], zs[kSources], ws[kSources], vs[kSources];
#pragma unroll
    for (int a = 0; a < kTargets; ++a) {
        const uint32_t h = gid * 64u + (uint32_t)a * 4u;
        xa[a] = (T)(2.0 * unit_hash(h) - 1.0);
        ya[a] = (T)(2.0 * unit_hash(h + 1) - 1.0);
        za[a] = (T)(2.0 * unit_hash(h + 2) - 1.0);
        wa[a] = (T)unit_hash(h + 3);
        acc[a] = (T)0;
    }
#pragma unroll
    for (int b = 0; b < kSources; ++b) {
        const uint32_t h = gid * 64u + 16u + (uint32_t)b * 5u;
        xs[b] = (T)(1.01 + 2.0 * unit_hash(h));
        ys[b] = (T)(2.0 * unit_hash(h + 1) - 1.0);
        zs[b] = (T)(2.0 * unit_hash(h + 2) - 1.0);
        ws[b] = (T)unit_hash(h + 3);
        vs[b] = (T)(unit_hash(h + 4) - 0.5);
    }
    const T st = (T)step;
    for (int p = 0; p < passes; ++p) {
#pragma unroll
        for (int b = 0; b < kSources; ++b) {
#pragma unroll
            for (int a = 0; a < kTargets; ++a) {
                const T r2 = add_extra<KIND>(dist2<false, D>(xa[a] - xs[b], ya[a] - ys[b], za[a] - zs[b]), wa[a], ws[b]);
                if constexpr (sizeof(T) == 8) {
                    acc[a] = fma(kval_pos<KIND>(r2, kp64, ktab), vs[b], acc[a]);
                } else {
                    const KPar<float> kp{(float)kp64.kp, (float)kp64.c0, (float)kp64.c1, (float)kp64.c2};
                    acc[a] = fmaf(kval<KIND>(r2, 0.0f, kp), vs[b], acc[a]);
                }
            }
            xs[b] += st;
        }
    }
    T s = (T)0;
#pragma unroll
    for (int a = 0; a < kTargets; ++a) s += acc[a];
    out[gid] = (double)s;
}

template <typename T, int KIND>
hipError_t launch_kind(int d, int blocks, const double *tab, const KPar<double> &kp, int passes, double *out,
                       hipStream_t s)
{
    if (d == 2) {
        if constexpr (kExtraCoord<KIND>) return hipErrorInvalidValue; // the NTI kernel is 3D only
        else k_eval_rate<T, KIND, 2><<<blocks, kThreads, 0, s>>>(tab, kp, 1e-9, passes, out);
    } else {
        k_eval_rate<T, KIND, 3><<<blocks, kThreads, 0, s>>>(tab, kp, 1e-9, passes, out);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prec(int kind, int d, int blocks, const double *tab, const KPar<double> &kp, int passes,
                       double *out, hipStream_t s)
{
    switch (kind) {
    case H2S_K_LOG_R: return launch_kind<T, H2S_K_LOG_R>(d, blocks, tab, kp, passes, out, s);
    case H2S_K_INV_R: return launch_kind<T, H2S_K_INV_R>(d, blocks, tab, kp, passes, out, s);
    case H2S_K_GAUSSIAN: return launch_kind<T, H2S_K_GAUSSIAN>(d, blocks, tab, kp, passes, out, s);
    case H2S_K_EXP_R: return launch_kind<T, H2S_K_EXP_R>(d, blocks, tab, kp, passes, out, s);
    case H2S_K_RBF_AR: return launch_kind<T, H2S_K_RBF_AR>(d, blocks, tab, kp, passes, out, s);
    case H2S_K_RBF_LOG: return launch_kind<T, H2S_K_RBF_LOG>(d, blocks, tab, kp, passes, out, s);
    case H2S_K_NTI_MQ: return launch_kind<T, H2S_K_NTI_MQ>(d, blocks, tab, kp, passes, out, s);
    default: return hipErrorInvalidValue;
    }
}

} // namespace

int64_t eval_rate_evals(int blocks, int passes)
{
    return (int64_t)blocks * kThreads * passes * kTargets * kSources;
}

int64_t eval_rate_outputs(int blocks) { return (int64_t)blocks * kThreads; }

hipError_t launch_eval_rate(int kind, int d, bool fp32, int blocks, const double *tab, double kparam,
                            const double kc[3], int passes, double *out, hipStream_t s)
{
    const KPar<double> kp{kparam, kc[0], kc[1], kc[2]};
    return fp32 ? launch_prec<float>(kind, d, blocks, tab, kp, passes, out, s)
                : launch_prec<double>(kind, d, blocks, tab, kp, passes, out, s);
}

} // namespace h2s
