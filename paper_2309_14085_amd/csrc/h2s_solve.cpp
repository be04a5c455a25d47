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

int gmres_ir_many(const SolveOpsMany &ops, const SolveWorkMany &wk, const SolveParams &prm, int64_t n, int ncols,
                  const double *b, int64_t ldb, double *x, int64_t ldx, void *stream, SolveResult *res)
{
    hipStream_t s = (hipStream_t)stream;
    const int m = prm.restart, nc = ncols;
    const SmallLayout L = small_layout(m);
    const int64_t S = solve_small_doubles(m), sV = (int64_t)(m + 1) * n, sP = blas_dots_blocks(n) * (m + 1);
    // vec: the gathered states (3 per column), then per column the cycle's start norm, inner
    // tolerance and step limit
    double *beta_d = wk.vec + 3 * (int64_t)wk.cols, *tol_d = beta_d + wk.cols, *lim_d = tol_d + wk.cols;
    double *beta_h = wk.host + 3 * (int64_t)wk.cols, *tol_h = beta_h + wk.cols, *lim_h = tol_h + wk.cols;
    std::vector<double> bnorm(nc), rnorm(nc);
    std::vector<int> its(nc, 0), refs(nc, 0), stall(nc, 0), done(nc, 0), conv(nc, 0);
    for (int c = 0; c < nc; ++c) res[c] = SolveResult{0, 0, 0, std::numeric_limits<double>::quiet_NaN()};
    try {
        int na = 0; // active columns, listed in wk.idx
        auto set_active = [&](const std::vector<int> &cols) {
            na = (int)cols.size();
            for (int i = 0; i < na; ++i) wk.host_idx[i] = cols[i];
            if (na) ck((int)hipMemcpyAsync(wk.idx, wk.host_idx, sizeof(int) * na, hipMemcpyHostToDevice, s));
        };
        // every column's new norm and cycle state to the host
        auto to_host = [&]() {
            ck(blas_gather_state(wk.small, S, L, nc, wk.vec, s));
            ck((int)hipMemcpyAsync(wk.host, wk.vec, sizeof(double) * 3 * nc, hipMemcpyDeviceToHost, s));
            ck((int)hipStreamSynchronize(s));
        };
        // squared norms of the listed columns of a (ld, stride sv) matrix into their nrm2 slots
        auto norms = [&](const double *v, int64_t sv) {
            ck(blas_dots_m(v, n, sv, 1, v, sv, n, wk.part, sP, wk.small + L.nrm2, S, wk.idx, na, s));
            to_host();
        };
        std::vector<int> all(nc);
        for (int c = 0; c < nc; ++c) all[c] = c;
        set_active(all);
        norms(b, ldb);
        for (int c = 0; c < nc; ++c) bnorm[c] = std::sqrt(wk.host[3 * c]);
        if (prm.use_x0) {
            ck(ops.apply_outer(ops.ctx, x, ldx, wk.Y, n, nc));
            ck(blas_sub_m(b, ldb, wk.Y, n, wk.R, n, n, wk.idx, na, s));
        } else {
            for (int c = 0; c < nc; ++c) {
                ck(blas_fill(x + c * ldx, 0.0, n, s));
                ck((int)hipMemcpyAsync(wk.R + c * n, b + c * ldb, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            }
        }
        norms(wk.R, n);
        for (int c = 0; c < nc; ++c) {
            rnorm[c] = std::sqrt(wk.host[3 * c]);
            if (bnorm[c] == 0.0) { // b = 0: x = 0 exactly
                ck(blas_fill(x + c * ldx, 0.0, n, s));
                done[c] = conv[c] = 1;
                rnorm[c] = 0.0;
            }
        }
        while (true) {
            std::vector<int> act;
            for (int c = 0; c < nc; ++c) {
                if (done[c]) continue;
                if (rnorm[c] / bnorm[c] <= prm.rtol) {
                    done[c] = conv[c] = 1;
                    continue;
                }
                if (its[c] >= prm.max_iter || refs[c] >= prm.max_refine || stall[c] >= 3) {
                    done[c] = 1;
                    continue;
                }
                act.push_back(c);
            }
            if (act.empty()) break;
            set_active(act);
            // one GMRES(m) cycle per active column on K~ d = r, d = V_k y, in lockstep
            int steps = 0;
            for (int c : act) {
                beta_h[c] = rnorm[c];
                tol_h[c] = prm.inner_rtol * rnorm[c];
                lim_h[c] = (double)std::min(m, prm.max_iter - its[c]);
                steps = std::max(steps, (int)lim_h[c]);
            }
            ck((int)hipMemcpyAsync(beta_d, beta_h, sizeof(double) * 3 * wk.cols, hipMemcpyHostToDevice, s));
            ck(blas_scale_m(wk.R, n, beta_d, wk.V, sV, n, wk.idx, na, s));
            ck(blas_cycle_start_m(wk.small, S, L, m, beta_d, wk.idx, na, s));
            for (int j = 0; j < steps; ++j) {
                // the step's products for every column at once (inactive columns ride along)
                ck(ops.apply_inner(ops.ctx, wk.V + (int64_t)j * n, sV, wk.W, n, nc));
                const double *Vj = wk.V;
                ck(blas_dots_m(Vj, n, sV, j + 1, wk.W, n, n, wk.part, sP, wk.small + L.h1, S, wk.idx, na, s));
                ck(blas_gemv_acc_m(Vj, n, sV, j + 1, wk.small + L.h1, S, -1.0, wk.W, n, n, wk.idx, na, s));
                ck(blas_dots_m(Vj, n, sV, j + 1, wk.W, n, n, wk.part, sP, wk.small + L.h2, S, wk.idx, na, s));
                ck(blas_gemv_acc_m(Vj, n, sV, j + 1, wk.small + L.h2, S, -1.0, wk.W, n, n, wk.idx, na, s));
                ck(blas_dots_m(wk.W, n, n, 1, wk.W, n, n, wk.part, sP, wk.small + L.nrm2, S, wk.idx, na, s));
                ck(blas_normalise_m(wk.W, n, wk.small + L.nrm2, S, wk.V + (int64_t)(j + 1) * n, sV, n, wk.idx, na, s));
                // a column past its own step limit takes no more steps into its Hessenberg matrix
                ck(blas_givens_m(j, m, wk.small, S, L, tol_d, lim_d, wk.idx, na, s));
                if ((j + 1) % kCheck == 0 && j + 1 < steps) {
                    to_host();
                    bool all_done = true;
                    for (int c : act) all_done = all_done && (wk.host[3 * c + 1] != 0.0 || j + 1 >= (int)lim_h[c]);
                    if (all_done) break;
                }
            }
            to_host();
            for (int c : act) its[c] += (int)wk.host[3 * c + 2];
            // back substitution H_k y = g_k, then x += V_k y, per column
            ck(blas_backsolve_m(m, wk.small, S, L, wk.idx, na, s));
            ck(blas_xupdate_m(wk.V, n, sV, wk.small, S, L, x, ldx, n, wk.idx, na, s));
            for (int c : act) ++refs[c];
            // FP64 residuals of every column at once
            ck(ops.apply_outer(ops.ctx, x, ldx, wk.Y, n, nc));
            ck(blas_sub_m(b, ldb, wk.Y, n, wk.R, n, n, wk.idx, na, s));
            norms(wk.R, n);
            for (int c : act) {
                const double prev = rnorm[c];
                rnorm[c] = std::sqrt(wk.host[3 * c]);
                stall[c] = rnorm[c] >= 0.999 * prev ? stall[c] + 1 : 0;
            }
        }
        for (int c = 0; c < nc; ++c)
            res[c] = SolveResult{its[c], refs[c], conv[c], bnorm[c] == 0.0 ? 0.0 : rnorm[c] / bnorm[c]};
    } catch (const Fail &f) {
        return f.code;
    }
    return 0;
}

} // namespace h2s
