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

} // namespace h2s
