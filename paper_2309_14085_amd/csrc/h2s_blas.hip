// h2s_blas.hip -- FP64 vector kernels of the GMRES solve (Arnoldi with
// classical Gram-Schmidt applied twice, the correction x += V y and the
// residual b - K~ x).  Every reduction runs in a fixed order (partial sums
// per wavefront, then a fixed tree over them), so a solve is bitwise
// reproducible run to run.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "h2s_blas.hpp"

namespace h2s {

namespace {

constexpr int NT = 256;
constexpr int ROWS_PER_THREAD = 2;
constexpr int ROWS_PER_BLOCK = NT * ROWS_PER_THREAD;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int WAVES = NT / 64;

// part[(blk WAVES + wave) ncols + k] = sum over the wave's rows i of
// V[i + k ldv] w[i]: wave-level reductions only, no block barriers.
__global__ __launch_bounds__(NT) void k_dots_part(const double *__restrict__ V, int64_t ldv, int ncols,
                                                  const double *__restrict__ w, int64_t n, double *__restrict__ part)
{
    const int64_t base = (int64_t)blockIdx.x * ROWS_PER_BLOCK + threadIdx.x;
    double wr[ROWS_PER_THREAD];
#pragma unroll
    for (int u = 0; u < ROWS_PER_THREAD; ++u) {
        const int64_t i = base + (int64_t)u * NT;
        wr[u] = i < n ? w[i] : 0.0;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double *out = part + ((int64_t)blockIdx.x * WAVES + wave) * ncols;
    // KB columns at a time keep KB x ROWS_PER_THREAD loads in flight per thread
    constexpr int KB = 8;
    for (int k0 = 0; k0 < ncols; k0 += KB) {
        double s[KB];
#pragma unroll
        for (int c = 0; c < KB; ++c) {
            s[c] = 0.0;
            if (k0 + c < ncols) {
                const double *col = V + (int64_t)(k0 + c) * ldv;
#pragma unroll
                for (int u = 0; u < ROWS_PER_THREAD; ++u) {
                    const int64_t i = base + (int64_t)u * NT;
                    if (i < n) s[c] = fma(col[i], wr[u], s[c]);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < KB; ++c) {
            const double t = wave_sum(s[c]);
            if (lane == 0 && k0 + c < ncols) out[k0 + c] = t;
        }
    }
}

// out[k] = sum_p part[p ncols + k] over the np partial rows: one block per k,
// thread t sums rows t, t + NT, ... in order, then a fixed reduction tree.
__global__ __launch_bounds__(NT) void k_dots_final(const double *__restrict__ part, int np, int ncols,
                                                   double *__restrict__ out)
{
    __shared__ double red[WAVES];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int p = threadIdx.x; p < np; p += NT) s += part[(int64_t)p * ncols + k];
    s = wave_sum(s);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < WAVES; ++q) t += red[q];
        out[k] = t;
    }
}

// y[i] += alpha sum_k V[i + k ldv] c[k]   (c in device memory, ncols <= kMaxCols)
__global__ __launch_bounds__(NT) void k_gemv_acc(const double *__restrict__ V, int64_t ldv, int ncols,
                                                 const double *__restrict__ c, double alpha, double *__restrict__ y,
                                                 int64_t n)
{
    __shared__ double cs[kMaxCols];
    for (int k = threadIdx.x; k < ncols; k += NT) cs[k] = c[k];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < ncols; ++k) s = fma(V[i + (int64_t)k * ldv], cs[k], s);
    y[i] = fma(alpha, s, y[i]);
}

// v = w / sqrt(nrm2[0]), or 0 when the norm is zero (breakdown).
__global__ __launch_bounds__(NT) void k_normalise(const double *__restrict__ w, const double *__restrict__ nrm2,
                                                  double *__restrict__ v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    const double s = nrm2[0];
    v[i] = s > 0.0 ? w[i] / sqrt(s) : 0.0;
}

// v = w / beta (beta a host scalar > 0).
__global__ __launch_bounds__(NT) void k_scale(const double *__restrict__ w, double beta, double *__restrict__ v,
                                              int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) v[i] = w[i] / beta;
}

// r = b - y
__global__ __launch_bounds__(NT) void k_sub(const double *__restrict__ b, const double *__restrict__ y,
                                            double *__restrict__ r, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) r[i] = b[i] - y[i];
}

// v = c (fill)
__global__ __launch_bounds__(NT) void k_fill(double *__restrict__ v, double c, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) v[i] = c;
}

inline unsigned grid(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

// ---------------------------------------------------------------------------
// Column-batched forms: blockIdx.y picks the column c = idx[blockIdx.y]; the
// arithmetic of each column is that of the single-column kernels above.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_dots_part_m(const double *__restrict__ V0, int64_t ldv, int64_t sV, int ncols,
                                                    const double *__restrict__ w0, int64_t sw, int64_t n,
                                                    double *__restrict__ part0, int64_t sp, const int *__restrict__ idx)
{
    const int64_t c = idx[blockIdx.y];
    const double *V = V0 + c * sV, *w = w0 + c * sw;
    double *part = part0 + c * sp;
    const int64_t base = (int64_t)blockIdx.x * ROWS_PER_BLOCK + threadIdx.x;
    double wr[ROWS_PER_THREAD];
#pragma unroll
    for (int u = 0; u < ROWS_PER_THREAD; ++u) {
        const int64_t i = base + (int64_t)u * NT;
        wr[u] = i < n ? w[i] : 0.0;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double *out = part + ((int64_t)blockIdx.x * WAVES + wave) * ncols;
    constexpr int KB = 8;
    for (int k0 = 0; k0 < ncols; k0 += KB) {
        double s[KB];
#pragma unroll
        for (int cc = 0; cc < KB; ++cc) {
            s[cc] = 0.0;
            if (k0 + cc < ncols) {
                const double *col = V + (int64_t)(k0 + cc) * ldv;
#pragma unroll
                for (int u = 0; u < ROWS_PER_THREAD; ++u) {
                    const int64_t i = base + (int64_t)u * NT;
                    if (i < n) s[cc] = fma(col[i], wr[u], s[cc]);
                }
            }
        }
#pragma unroll
        for (int cc = 0; cc < KB; ++cc) {
            const double t = wave_sum(s[cc]);
            if (lane == 0 && k0 + cc < ncols) out[k0 + cc] = t;
        }
    }
}

__global__ __launch_bounds__(NT) void k_dots_final_m(const double *__restrict__ part0, int64_t sp, int np, int ncols,
                                                     double *__restrict__ out0, int64_t so, const int *__restrict__ idx)
{
    __shared__ double red[WAVES];
    const int64_t c = idx[blockIdx.y];
    const double *part = part0 + c * sp;
    const int k = blockIdx.x;
    double s = 0.0;
    for (int p = threadIdx.x; p < np; p += NT) s += part[(int64_t)p * ncols + k];
    s = wave_sum(s);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < WAVES; ++q) t += red[q];
        out0[c * so + k] = t;
    }
}

__global__ __launch_bounds__(NT) void k_gemv_acc_m(const double *__restrict__ V0, int64_t ldv, int64_t sV, int ncols,
                                                   const double *__restrict__ c0, int64_t sc, double alpha,
                                                   double *__restrict__ y0, int64_t sy, int64_t n,
                                                   const int *__restrict__ idx)
{
    __shared__ double cs[kMaxCols];
    const int64_t col = idx[blockIdx.y];
    const double *V = V0 + col * sV, *cv = c0 + col * sc;
    double *y = y0 + col * sy;
    for (int k = threadIdx.x; k < ncols; k += NT) cs[k] = cv[k];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < ncols; ++k) s = fma(V[i + (int64_t)k * ldv], cs[k], s);
    y[i] = fma(alpha, s, y[i]);
}

__global__ __launch_bounds__(NT) void k_normalise_m(const double *__restrict__ w0, int64_t sw,
                                                    const double *__restrict__ nrm0, int64_t sn,
                                                    double *__restrict__ v0, int64_t sv, int64_t n,
                                                    const int *__restrict__ idx)
{
    const int64_t c = idx[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    const double s = nrm0[c * sn];
    v0[c * sv + i] = s > 0.0 ? w0[c * sw + i] / sqrt(s) : 0.0;
}

__global__ __launch_bounds__(NT) void k_scale_m(const double *__restrict__ w0, int64_t sw, const double *__restrict__ beta,
                                                double *__restrict__ v0, int64_t sv, int64_t n,
                                                const int *__restrict__ idx)
{
    const int64_t c = idx[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) v0[c * sv + i] = w0[c * sw + i] / beta[c];
}

__global__ __launch_bounds__(NT) void k_sub_m(const double *__restrict__ b0, int64_t sb, const double *__restrict__ y0,
                                              int64_t sy, double *__restrict__ r0, int64_t sr, int64_t n,
                                              const int *__restrict__ idx)
{
    const int64_t c = idx[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) r0[c * sr + i] = b0[c * sb + i] - y0[c * sy + i];
}

__global__ void k_gather_state(const double *__restrict__ small, int64_t S, int64_t off, int ncols,
                               double *__restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 3 * ncols) out[t] = small[(int64_t)(t / 3) * S + off + t % 3];
}

} // namespace

int64_t blas_dots_blocks(int64_t n) { return WAVES * ((n + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK); }

int blas_dots(const double *V, int64_t ldv, int ncols, const double *w, int64_t n, double *part, double *out,
              void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int64_t nb = (n + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK;
    if (ncols <= 0 || n <= 0) return 0;
    hipLaunchKernelGGL(k_dots_part, dim3((unsigned)nb), dim3(NT), 0, s, V, ldv, ncols, w, n, part);
    hipLaunchKernelGGL(k_dots_final, dim3((unsigned)ncols), dim3(NT), 0, s, part, (int)(nb * WAVES), ncols, out);
    return (int)hipGetLastError();
}

int blas_gemv_acc(const double *V, int64_t ldv, int ncols, const double *c, double alpha, double *y, int64_t n,
                  void *stream)
{
    if (ncols <= 0 || n <= 0) return 0;
    if (ncols > kMaxCols) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gemv_acc, dim3(grid(n, NT)), dim3(NT), 0, (hipStream_t)stream, V, ldv, ncols, c, alpha, y, n);
    return (int)hipGetLastError();
}

namespace {

// ---------------------------------------------------------------------------
// The small dense part of a GMRES(m) cycle on the device (one thread: at most
// m + 1 = 1001 entries per column, a few microseconds).  H is (m + 1) x m,
// row-major; st[0] = 1 once the cycle is done, st[1] = the steps it kept.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cycle_start_body(double *g, double *st, int m, double beta)
{
    for (int i = 0; i <= m; ++i) g[i] = 0.0;
    g[0] = beta;
    st[0] = 0.0;
    st[1] = 0.0;
}

__global__ void k_cycle_start(double *g, double *st, int m, double beta)
{
    if (threadIdx.x == 0) cycle_start_body(g, st, m, beta);
}

// Step j: column j of H from the two Gram-Schmidt passes (h1 + h2) and the new norm, the
// rotations of steps 0 .. j-1 in order, then the rotation that zeroes H(j+1, j), applied to g.
// The cycle is done when |g[j+1]| <= tol, or on a breakdown (zero norm or zero pivot); a done
// cycle ignores later steps.
__device__ __forceinline__ void givens_body(int j, int m, const double *h1, const double *h2, const double *nrm2,
                                            double *H, double *cs, double *sn, double *g, double tol, double *st)
{
    if (st[0] != 0.0) return;
    auto Hat = [&](int i, int c) -> double & { return H[(int64_t)i * m + c]; };
    for (int i = 0; i <= j; ++i) Hat(i, j) = h1[i] + h2[i];
    const double hn = sqrt(nrm2[0]);
    Hat(j + 1, j) = hn;
    for (int i = 0; i < j; ++i) {
        const double t = cs[i] * Hat(i, j) + sn[i] * Hat(i + 1, j);
        Hat(i + 1, j) = -sn[i] * Hat(i, j) + cs[i] * Hat(i + 1, j);
        Hat(i, j) = t;
    }
    const double den = hypot(Hat(j, j), Hat(j + 1, j));
    cs[j] = den != 0.0 ? Hat(j, j) / den : 1.0;
    sn[j] = den != 0.0 ? Hat(j + 1, j) / den : 0.0;
    Hat(j, j) = cs[j] * Hat(j, j) + sn[j] * Hat(j + 1, j);
    Hat(j + 1, j) = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    st[1] = (double)(j + 1);
    if (fabs(g[j + 1]) <= tol || hn == 0.0 || den == 0.0) st[0] = 1.0;
}

__global__ void k_givens(int j, int m, const double *h1, const double *h2, const double *nrm2, double *H, double *cs,
                         double *sn, double *g, double tol, double *st)
{
    if (threadIdx.x == 0) givens_body(j, m, h1, h2, nrm2, H, cs, sn, g, tol, st);
}

// y = H_k^{-1} g_k by back substitution, k = st[1] steps.
__device__ __forceinline__ void backsolve_body(int m, const double *H, const double *g, const double *st, double *y)
{
    const int k = (int)st[1];
    for (int i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int c = i + 1; c < k; ++c) t -= H[(int64_t)i * m + c] * y[c];
        const double d = H[(int64_t)i * m + i];
        y[i] = d != 0.0 ? t / d : 0.0;
    }
}

__global__ void k_backsolve(int m, const double *H, const double *g, const double *st, double *y)
{
    if (threadIdx.x == 0) backsolve_body(m, H, g, st, y);
}

// the same for the listed columns, one block each
__global__ void k_cycle_start_m(double *small, int64_t S, SmallLayout L, int m, const double *beta, const int *idx)
{
    const int64_t c = idx[blockIdx.x];
    if (threadIdx.x == 0) cycle_start_body(small + c * S + L.g, small + c * S + L.st, m, beta[c]);
}

__global__ void k_givens_m(int j, int m, double *small, int64_t S, SmallLayout L, const double *tol, const double *lim,
                           const int *idx)
{
    const int64_t c = idx[blockIdx.x];
    double *b = small + c * S;
    if (threadIdx.x == 0 && (double)j < lim[c])
        givens_body(j, m, b + L.h1, b + L.h2, b + L.nrm2, b + L.H, b + L.cs, b + L.sn, b + L.g, tol[c], b + L.st);
}

__global__ void k_backsolve_m(int m, double *small, int64_t S, SmallLayout L, const int *idx)
{
    const int64_t c = idx[blockIdx.x];
    double *b = small + c * S;
    if (threadIdx.x == 0) backsolve_body(m, b + L.H, b + L.g, b + L.st, b + L.yv);
}

// x_c += V_c y_c over k_c = st_c[1] columns of V_c
__global__ __launch_bounds__(256) void k_xupdate_m(const double *__restrict__ V0, int64_t ldv, int64_t sV,
                                                   const double *__restrict__ small, int64_t S, SmallLayout L,
                                                   double *__restrict__ x0, int64_t sx, int64_t n,
                                                   const int *__restrict__ idx)
{
    __shared__ double ys[kMaxCols];
    const int64_t c = idx[blockIdx.y];
    const double *b = small + c * S, *V = V0 + c * sV;
    const int k = (int)b[L.st + 1];
    for (int q = threadIdx.x; q < k; q += 256) ys[q] = b[L.yv + q];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int q = 0; q < k; ++q) s = fma(V[i + (int64_t)q * ldv], ys[q], s);
    x0[c * sx + i] = fma(1.0, s, x0[c * sx + i]);
}

} // namespace

int blas_cycle_start(double *g, double *st, int m, double beta, void *stream)
{
    hipLaunchKernelGGL(k_cycle_start, dim3(1), dim3(64), 0, (hipStream_t)stream, g, st, m, beta);
    return (int)hipGetLastError();
}

int blas_givens(int j, int m, const double *h1, const double *h2, const double *nrm2, double *H, double *cs, double *sn,
                double *g, double tol, double *st, void *stream)
{
    hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, (hipStream_t)stream, j, m, h1, h2, nrm2, H, cs, sn, g, tol, st);
    return (int)hipGetLastError();
}

int blas_backsolve(int m, const double *H, const double *g, const double *st, double *y, void *stream)
{
    hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(64), 0, (hipStream_t)stream, m, H, g, st, y);
    return (int)hipGetLastError();
}

int blas_normalise(const double *w, const double *nrm2, double *v, int64_t n, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_normalise, dim3(grid(n, NT)), dim3(NT), 0, (hipStream_t)stream, w, nrm2, v, n);
    return (int)hipGetLastError();
}

int blas_scale(const double *w, double beta, double *v, int64_t n, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_scale, dim3(grid(n, NT)), dim3(NT), 0, (hipStream_t)stream, w, beta, v, n);
    return (int)hipGetLastError();
}

int blas_sub(const double *b, const double *y, double *r, int64_t n, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_sub, dim3(grid(n, NT)), dim3(NT), 0, (hipStream_t)stream, b, y, r, n);
    return (int)hipGetLastError();
}

int blas_fill(double *v, double c, int64_t n, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_fill, dim3(grid(n, NT)), dim3(NT), 0, (hipStream_t)stream, v, c, n);
    return (int)hipGetLastError();
}

int blas_dots_m(const double *V, int64_t ldv, int64_t sV, int ncols, const double *w, int64_t sw, int64_t n,
                double *part, int64_t sp, double *out, int64_t so, const int *idx, int nc, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int64_t nb = (n + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK;
    if (ncols <= 0 || n <= 0 || nc <= 0) return 0;
    hipLaunchKernelGGL(k_dots_part_m, dim3((unsigned)nb, (unsigned)nc), dim3(NT), 0, s, V, ldv, sV, ncols, w, sw, n,
                       part, sp, idx);
    hipLaunchKernelGGL(k_dots_final_m, dim3((unsigned)ncols, (unsigned)nc), dim3(NT), 0, s, part, sp,
                       (int)(nb * WAVES), ncols, out, so, idx);
    return (int)hipGetLastError();
}

int blas_gemv_acc_m(const double *V, int64_t ldv, int64_t sV, int ncols, const double *c, int64_t sc, double alpha,
                    double *y, int64_t sy, int64_t n, const int *idx, int nc, void *stream)
{
    if (ncols <= 0 || n <= 0 || nc <= 0) return 0;
    if (ncols > kMaxCols) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gemv_acc_m, dim3(grid(n, NT), (unsigned)nc), dim3(NT), 0, (hipStream_t)stream, V, ldv, sV,
                       ncols, c, sc, alpha, y, sy, n, idx);
    return (int)hipGetLastError();
}

int blas_normalise_m(const double *w, int64_t sw, const double *nrm2, int64_t sn, double *v, int64_t sv, int64_t n,
                     const int *idx, int nc, void *stream)
{
    if (n <= 0 || nc <= 0) return 0;
    hipLaunchKernelGGL(k_normalise_m, dim3(grid(n, NT), (unsigned)nc), dim3(NT), 0, (hipStream_t)stream, w, sw, nrm2,
                       sn, v, sv, n, idx);
    return (int)hipGetLastError();
}

int blas_scale_m(const double *w, int64_t sw, const double *beta, double *v, int64_t sv, int64_t n, const int *idx,
                 int nc, void *stream)
{
    if (n <= 0 || nc <= 0) return 0;
    hipLaunchKernelGGL(k_scale_m, dim3(grid(n, NT), (unsigned)nc), dim3(NT), 0, (hipStream_t)stream, w, sw, beta, v,
                       sv, n, idx);
    return (int)hipGetLastError();
}

int blas_sub_m(const double *b, int64_t sb, const double *y, int64_t sy, double *r, int64_t sr, int64_t n,
               const int *idx, int nc, void *stream)
{
    if (n <= 0 || nc <= 0) return 0;
    hipLaunchKernelGGL(k_sub_m, dim3(grid(n, NT), (unsigned)nc), dim3(NT), 0, (hipStream_t)stream, b, sb, y, sy, r, sr,
                       n, idx);
    return (int)hipGetLastError();
}

int blas_cycle_start_m(double *small, int64_t S, SmallLayout L, int m, const double *beta, const int *idx, int nc,
                       void *stream)
{
    if (nc <= 0) return 0;
    hipLaunchKernelGGL(k_cycle_start_m, dim3((unsigned)nc), dim3(64), 0, (hipStream_t)stream, small, S, L, m, beta, idx);
    return (int)hipGetLastError();
}

int blas_givens_m(int j, int m, double *small, int64_t S, SmallLayout L, const double *tol, const double *lim,
                  const int *idx, int nc, void *stream)
{
    if (nc <= 0) return 0;
    hipLaunchKernelGGL(k_givens_m, dim3((unsigned)nc), dim3(64), 0, (hipStream_t)stream, j, m, small, S, L, tol, lim,
                       idx);
    return (int)hipGetLastError();
}

int blas_backsolve_m(int m, double *small, int64_t S, SmallLayout L, const int *idx, int nc, void *stream)
{
    if (nc <= 0) return 0;
    hipLaunchKernelGGL(k_backsolve_m, dim3((unsigned)nc), dim3(64), 0, (hipStream_t)stream, m, small, S, L, idx);
    return (int)hipGetLastError();
}

int blas_xupdate_m(const double *V, int64_t ldv, int64_t sV, const double *small, int64_t S, SmallLayout L, double *x,
                   int64_t sx, int64_t n, const int *idx, int nc, void *stream)
{
    if (n <= 0 || nc <= 0) return 0;
    hipLaunchKernelGGL(k_xupdate_m, dim3(grid(n, 256), (unsigned)nc), dim3(256), 0, (hipStream_t)stream, V, ldv, sV,
                       small, S, L, x, sx, n, idx);
    return (int)hipGetLastError();
}

int blas_gather_state(const double *small, int64_t S, SmallLayout L, int ncols, double *out, void *stream)
{
    if (ncols <= 0) return 0;
    hipLaunchKernelGGL(k_gather_state, dim3(grid(3 * (int64_t)ncols, 64)), dim3(64), 0, (hipStream_t)stream, small, S,
                       L.nrm2, ncols, out);
    return (int)hipGetLastError();
}

} // namespace h2s
