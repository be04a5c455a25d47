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
// solve live on the device too (h2s_blas.hip): a cycle is enqueued step by
// step without waiting, the host reads back the cycle's state only every
// kCheck steps (to stop at the inner tolerance) and the new residual norm
// once per cycle.
#include "h2s_solve.hpp"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <limits>

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

// Arnoldi steps enqueued between two looks at the cycle's state.
constexpr int kCheck = 4;

int gmres_ir(const SolveOps &ops, const SolveWork &wk, const SolveParams &prm, int64_t n, const double *b, double *x,
             void *stream, SolveResult *res)
{
    hipStream_t s = (hipStream_t)stream;
    const int m = prm.restart;
    // layout of wk.small (solve_small_doubles)
    double *h1 = wk.small, *h2 = h1 + (m + 1), *nrm2 = h2 + (m + 1), *st = nrm2 + 1;
    double *H = st + 2, *cs = H + (int64_t)(m + 1) * m, *sn = cs + m, *g = sn + m, *yv = g + (m + 1);
    const int64_t o_nrm2 = nrm2 - wk.small;
    const double *nrm2h = wk.small_host + o_nrm2, *sth = nrm2h + 1;
    *res = SolveResult{0, 0, 0, std::numeric_limits<double>::quiet_NaN()};
    try {
        // the new norm and the cycle state to the host
        auto to_host = [&]() {
            ck((int)hipMemcpyAsync(wk.small_host + o_nrm2, nrm2, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
            ck((int)hipStreamSynchronize(s));
        };
        auto norm = [&](const double *v) {
            ck(blas_dots(v, n, 1, v, n, wk.part, nrm2, s));
            to_host();
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
        int its = 0, refs = 0, stall = 0;
        while (true) {
            if (rnorm / bnorm <= prm.rtol) {
                res->converged = 1;
                break;
            }
            if (its >= prm.max_iter || refs >= prm.max_refine || stall >= 3) break;
            // one GMRES(m) cycle on K~ d = r, d = V_k y, with the Hessenberg work on the device
            ck(blas_scale(wk.r, rnorm, wk.V, n, s));
            ck(blas_cycle_start(g, st, m, rnorm, s));
            const double tol = prm.inner_rtol * rnorm;
            const int steps = std::min(m, prm.max_iter - its);
            for (int j = 0; j < steps; ++j) {
                const double *vj = wk.V + (int64_t)j * n;
                ck(ops.apply_inner(ops.ctx, vj, wk.w));
                ck(blas_dots(wk.V, n, j + 1, wk.w, n, wk.part, h1, s));
                ck(blas_gemv_acc(wk.V, n, j + 1, h1, -1.0, wk.w, n, s));
                ck(blas_dots(wk.V, n, j + 1, wk.w, n, wk.part, h2, s));
                ck(blas_gemv_acc(wk.V, n, j + 1, h2, -1.0, wk.w, n, s));
                ck(blas_dots(wk.w, n, 1, wk.w, n, wk.part, nrm2, s));
                ck(blas_normalise(wk.w, nrm2, wk.V + (int64_t)(j + 1) * n, n, s));
                ck(blas_givens(j, m, h1, h2, nrm2, H, cs, sn, g, tol, st, s));
                if ((j + 1) % kCheck == 0 && j + 1 < steps) {
                    to_host();
                    if (sth[0] != 0.0) break;
                }
            }
            to_host();
            const int k = (int)sth[1];
            its += k;
            // back substitution H_k y = g_k, then x += V_k y
            ck(blas_backsolve(m, H, g, st, yv, s));
            ck(blas_gemv_acc(wk.V, n, k, yv, 1.0, x, n, s));
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
