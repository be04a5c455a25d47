// h2s_solve.hpp -- mixed-precision GMRES with iterative refinement on the
// device (h2s_solve.cpp).  The driver knows nothing about trees: the two
// products come in as callbacks.
#pragma once

#include <cstdint>

namespace h2s {

struct SolveOps {
    void *ctx;
    // y = K~ x with x, y device vectors of length n, ordered on the solve's stream
    int (*apply_inner)(void *ctx, const double *x, double *y); // precision of the Krylov iterations
    int (*apply_outer)(void *ctx, const double *x, double *y); // FP64: residuals of the refinement
};

// Device workspace (owned by the caller) for restart length m.
struct SolveWork {
    double *V;          // n x (m + 1), column-major, ld = n
    double *w, *r, *y;  // n each
    double *part;       // blas_dots_blocks(n) * (m + 1)
    double *small;      // device, solve_small_doubles(m): see gmres_ir for the layout
    double *small_host; // pinned host mirror of `small`
};

// Doubles of SolveWork::small for restart length m: the two Gram-Schmidt projections (m + 1
// each), the new norm and the cycle state (3), the Hessenberg matrix ((m + 1) m), the rotations
// (2 m), the rotated right-hand side (m + 1) and the least-squares solution (m).
inline int64_t solve_small_doubles(int m) { return 2 * (int64_t)(m + 1) + 3 + (int64_t)(m + 1) * m + 2 * (int64_t)m + (m + 1) + m; }

struct SolveParams {
    int restart, max_iter, max_refine;
    double rtol, inner_rtol;
    int use_x0;
};

struct SolveResult {
    int iterations, refinements, converged;
    double residual; // ||b - K~ x|| / ||b|| with the FP64 product
};

// Solve K~ x = b (b, x device, length n).  Returns 0 or a hipError_t.
int gmres_ir(const SolveOps &ops, const SolveWork &wk, const SolveParams &prm, int64_t n, const double *b, double *x,
             void *stream, SolveResult *res);

// Several right-hand sides in lockstep: every Krylov step applies the operator to all columns
// at once (the batched product), and the vector work of the columns runs in column-batched
// kernels; each column keeps its own Krylov space, cycle and refinement, and stops on its own.
struct SolveOpsMany {
    void *ctx;
    // Y = K~ X for ncols columns (device, column-major, leading dimensions ldx, ldy)
    int (*apply_inner)(void *ctx, const double *x, int64_t ldx, double *y, int64_t ldy, int ncols);
    int (*apply_outer)(void *ctx, const double *x, int64_t ldx, double *y, int64_t ldy, int ncols);
};

// Device workspace for up to `cols` columns and restart length m (owned by the caller).
struct SolveWorkMany {
    int cols;
    double *V;          // cols x n x (m + 1): column c's basis at V + c (m + 1) n, ld = n
    double *W, *R, *Y;  // n x cols each, ld = n
    double *part;       // cols x blas_dots_blocks(n) (m + 1)
    double *small;      // cols x solve_small_doubles(m)
    double *vec;        // 6 cols: the gathered states (3 per column), then beta, tol, step limit per column
    int *idx;           // cols: the active columns
    double *host;       // pinned mirror of vec
    int *host_idx;      // pinned mirror of idx
};

int gmres_ir_many(const SolveOpsMany &ops, const SolveWorkMany &wk, const SolveParams &prm, int64_t n, int ncols,
                  const double *b, int64_t ldb, double *x, int64_t ldx, void *stream, SolveResult *res);

} // namespace h2s
