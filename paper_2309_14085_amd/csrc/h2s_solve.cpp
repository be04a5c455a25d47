// h2s_solve.cpp -- GMRES with iterative refinement for K~ x = b (the solve of
// Khan & Ambikasaran, arXiv 2309.14085, Sec. 6: GMRES to a relative residual
// tolerance with the fast product as the operator).
//
// Each refinement step runs one GMRES(m) cycle on K~ d = r for the current
// FP64 residual r, with the Krylov products in the inner precision (FP32 by
// default) and everything else in FP64 on the device: Arnoldi vectors, the
// classical Gram-Schmidt projections applied twice, norms, the correction
// x += V y and the residual r = b - K~ x with the FP64 product.  The
// (m + 1) x m Hessenberg matrix, its Givens rotations and the triangular
// solve live on the host; one small device-to-host copy per Arnoldi step
// brings back the projection coefficients and the new norm.
#include "h2s_solve.hpp"

#include <hip/hip_runtime_api.h>

#include <cmath>
#include <limits>
#include <vector>

#include "h2s_blas.hpp"

namespace h2s {

namespace {

struct Fail {
    int code;
};

inline void ck(int rc)
{
    if (rc != 0) throw Fail{rc};
}

} // namespace

int gmres_ir(const SolveOps &ops, const SolveWork &wk, const SolveParams &prm, int64_t n, const double *b, double *x,
             void *stream, SolveResult *res)
{
    hipStream_t s = (hipStream_t)stream;
    const int m = prm.restart;
    double *h1 = wk.small, *h2 = wk.small + (m + 1), *nrm2 = wk.small + 2 * (m + 1);
    const double *h1h = wk.small_host, *h2h = wk.small_host + (m + 1), *nrm2h = wk.small_host + 2 * (m + 1);
    *res = SolveResult{0, 0, 0, std::numeric_limits<double>::quiet_NaN()};
    try {
        auto to_host = [&](int count) {
            ck((int)hipMemcpyAsync(wk.small_host, wk.small, sizeof(double) * count, hipMemcpyDeviceToHost, s));
            ck((int)hipStreamSynchronize(s));
        };
        auto norm = [&](const double *v) {
            ck(blas_dots(v, n, 1, v, n, wk.part, nrm2, s));
            to_host(2 * (m + 1) + 1);
            return std::sqrt(*nrm2h);
        };
        const double bnorm = norm(b);
        if (bnorm == 0.0) {
            ck(blas_fill(x, 0.0, n, s));
            *res = SolveResult{0, 0, 1, 0.0};
            return 0;
        }
        if (prm.use_x0) {
            ck(ops.apply_outer(ops.ctx, x, wk.y));
            ck(blas_sub(b, wk.y, wk.r, n, s));
        } else {
            ck(blas_fill(x, 0.0, n, s));
            ck((int)hipMemcpyAsync(wk.r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        }
        double rnorm = norm(wk.r);
        std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), yv(m);
        auto Hat = [&](int i, int j) -> double & { return H[(size_t)i * m + j]; };
        int its = 0, refs = 0, stall = 0;
        while (true) {
            if (rnorm / bnorm <= prm.rtol) {
                res->converged = 1;
                break;
            }
            if (its >= prm.max_iter || refs >= prm.max_refine || stall >= 3) break;
            // one GMRES(m) cycle on K~ d = r, d = V_k y
            ck(blas_scale(wk.r, rnorm, wk.V, n, s));
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = rnorm;
            int k = 0;
            for (int j = 0; j < m; ++j) {
                const double *vj = wk.V + (int64_t)j * n;
                ck(ops.apply_inner(ops.ctx, vj, wk.w));
                ck(blas_dots(wk.V, n, j + 1, wk.w, n, wk.part, h1, s));
                ck(blas_gemv_acc(wk.V, n, j + 1, h1, -1.0, wk.w, n, s));
                ck(blas_dots(wk.V, n, j + 1, wk.w, n, wk.part, h2, s));
                ck(blas_gemv_acc(wk.V, n, j + 1, h2, -1.0, wk.w, n, s));
                ck(blas_dots(wk.w, n, 1, wk.w, n, wk.part, nrm2, s));
                ck(blas_normalise(wk.w, nrm2, wk.V + (int64_t)(j + 1) * n, n, s));
                to_host(2 * (m + 1) + 1);
                for (int i = 0; i <= j; ++i) Hat(i, j) = h1h[i] + h2h[i];
                const double hn = std::sqrt(*nrm2h);
                Hat(j + 1, j) = hn;
                for (int i = 0; i < j; ++i) {
                    const double t = cs[i] * Hat(i, j) + sn[i] * Hat(i + 1, j);
                    Hat(i + 1, j) = -sn[i] * Hat(i, j) + cs[i] * Hat(i + 1, j);
                    Hat(i, j) = t;
                }
                const double den = std::hypot(Hat(j, j), Hat(j + 1, j));
                cs[j] = den != 0.0 ? Hat(j, j) / den : 1.0;
                sn[j] = den != 0.0 ? Hat(j + 1, j) / den : 0.0;
                Hat(j, j) = cs[j] * Hat(j, j) + sn[j] * Hat(j + 1, j);
                Hat(j + 1, j) = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                ++its;
                k = j + 1;
                if (std::fabs(g[j + 1]) <= prm.inner_rtol * rnorm || its >= prm.max_iter || hn == 0.0 || den == 0.0)
                    break;
            }
            // back substitution H_k y = g_k, then x += V_k y
            for (int i = k - 1; i >= 0; --i) {
                double t = g[i];
                for (int c = i + 1; c < k; ++c) t -= Hat(i, c) * yv[c];
                yv[i] = Hat(i, i) != 0.0 ? t / Hat(i, i) : 0.0;
            }
            for (int i = 0; i < k; ++i) wk.small_host[i] = yv[i];
            ck((int)hipMemcpyAsync(h1, wk.small_host, sizeof(double) * k, hipMemcpyHostToDevice, s));
            ck(blas_gemv_acc(wk.V, n, k, h1, 1.0, x, n, s));
            ++refs;
            // FP64 residual
            ck(ops.apply_outer(ops.ctx, x, wk.y));
            ck(blas_sub(b, wk.y, wk.r, n, s));
            const double prev = rnorm;
            rnorm = norm(wk.r);
            stall = rnorm >= 0.999 * prev ? stall + 1 : 0;
        }
        res->iterations = its;
        res->refinements = refs;
        res->residual = rnorm / bnorm;
    } catch (const Fail &f) {
        return f.code;
    }
    return 0;
}

} // namespace h2s
