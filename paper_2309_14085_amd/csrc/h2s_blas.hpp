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

} // namespace h2s
