// h2s_blas.hpp -- FP64 vector kernels of the GMRES solve (h2s_blas.hip).
// All pointers are device memory; every call is asynchronous on `stream` and
// returns a hipError_t as int.  Reductions run in a fixed order.
#pragma once

#include <cstdint>

namespace h2s {

constexpr int kMaxCols = 1024; // columns of V in one GEMV (restart + 1)

// Partial-sum rows used by blas_dots for n rows (one per wavefront).
int64_t blas_dots_blocks(int64_t n);
// out[k] = sum_i V[i + k ldv] w[i], k < ncols; part holds blas_dots_blocks(n) * ncols doubles.
int blas_dots(const double *V, int64_t ldv, int ncols, const double *w, int64_t n, double *part, double *out,
              void *stream);
// y += alpha V c (V n x ncols, column-major with leading dimension ldv; ncols <= kMaxCols).
int blas_gemv_acc(const double *V, int64_t ldv, int ncols, const double *c, double alpha, double *y, int64_t n,
                  void *stream);
// v = w / sqrt(nrm2[0]) (0 where nrm2[0] == 0); v may equal w.
int blas_normalise(const double *w, const double *nrm2, double *v, int64_t n, void *stream);
// v = w / beta; v may equal w.
int blas_scale(const double *w, double beta, double *v, int64_t n, void *stream);
// r = b - y.
int blas_sub(const double *b, const double *y, double *r, int64_t n, void *stream);
// v = c.
int blas_fill(double *v, double c, int64_t n, void *stream);

// The Hessenberg part of a GMRES(m) cycle on the device.  H: (m + 1) x m row-major; cs, sn: m;
// g: m + 1; st: 2 (st[0] = 1 once the cycle is done, st[1] = steps kept).
// Start a cycle: g = beta e_1, st = 0.
int blas_cycle_start(double *g, double *st, int m, double beta, void *stream);
// Step j: H(:, j) = h1 + h2 (rows 0..j), H(j+1, j) = sqrt(nrm2[0]), the earlier rotations, a new
// rotation zeroing H(j+1, j), g rotated; done when |g[j+1]| <= tol or on a breakdown.
int blas_givens(int j, int m, const double *h1, const double *h2, const double *nrm2, double *H, double *cs, double *sn,
                double *g, double tol, double *st, void *stream);
// y = H_k^{-1} g_k, k = st[1], by back substitution.
int blas_backsolve(int m, const double *H, const double *g, const double *st, double *y, void *stream);

// Layout of one column's small solve state (SolveWork::small, solve_small_doubles(m) doubles):
// offsets of the two Gram-Schmidt projections, the new norm, the cycle state, the Hessenberg
// matrix, the rotations, the rotated right-hand side and the least-squares solution.
struct SmallLayout {
    int64_t h1, h2, nrm2, st, H, cs, sn, g, yv;
};
inline SmallLayout small_layout(int m)
{
    SmallLayout L{};
    L.h1 = 0;
    L.h2 = L.h1 + (m + 1);
    L.nrm2 = L.h2 + (m + 1);
    L.st = L.nrm2 + 1;
    L.H = L.st + 2;
    L.cs = L.H + (int64_t)(m + 1) * m;
    L.sn = L.cs + m;
    L.g = L.sn + m;
    L.yv = L.g + (m + 1);
    return L;
}

// Column-batched forms for the lockstep solve of several right-hand sides: the same operation
// on the columns idx[0 .. nc) (a device list of column numbers), column c's operands at
// base + c * stride (strides in doubles).  Each column's results equal the single-column call's.
int blas_dots_m(const double *V, int64_t ldv, int64_t sV, int ncols, const double *w, int64_t sw, int64_t n,
                double *part, int64_t sp, double *out, int64_t so, const int *idx, int nc, void *stream);
int blas_gemv_acc_m(const double *V, int64_t ldv, int64_t sV, int ncols, const double *c, int64_t sc, double alpha,
                    double *y, int64_t sy, int64_t n, const int *idx, int nc, void *stream);
int blas_normalise_m(const double *w, int64_t sw, const double *nrm2, int64_t sn, double *v, int64_t sv, int64_t n,
                     const int *idx, int nc, void *stream);
// v_c = w_c / beta[c]
int blas_scale_m(const double *w, int64_t sw, const double *beta, double *v, int64_t sv, int64_t n, const int *idx,
                 int nc, void *stream);
// r_c = b_c - y_c
int blas_sub_m(const double *b, int64_t sb, const double *y, int64_t sy, double *r, int64_t sr, int64_t n,
               const int *idx, int nc, void *stream);
// The Hessenberg steps of blas_cycle_start / blas_givens / blas_backsolve for every listed column;
// small: the columns' states, S doubles apart (layout L); beta[c], tol[c]: the column's cycle
// start norm and inner tolerance.
int blas_cycle_start_m(double *small, int64_t S, SmallLayout L, int m, const double *beta, const int *idx, int nc,
                       void *stream);
int blas_givens_m(int j, int m, double *small, int64_t S, SmallLayout L, const double *tol, const double *lim,
                  const int *idx, int nc, void *stream); // steps j >= lim[c] are ignored
int blas_backsolve_m(int m, double *small, int64_t S, SmallLayout L, const int *idx, int nc, void *stream);
// x_c += V_c y_c over the k_c = st_c[1] steps the cycle kept
int blas_xupdate_m(const double *V, int64_t ldv, int64_t sV, const double *small, int64_t S, SmallLayout L, double *x,
                   int64_t sx, int64_t n, const int *idx, int nc, void *stream);
// out[3 c + i] = small[c S + L.nrm2 + i], i < 3, c < ncols: every column's new norm and cycle state
int blas_gather_state(const double *small, int64_t S, SmallLayout L, int ncols, double *out, void *stream);

} // namespace h2s
