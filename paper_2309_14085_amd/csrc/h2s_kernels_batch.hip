// h2s_kernels_batch.hip -- the H2* product for a block of kBatch right-hand
// sides at once (Sec. 5.1.2 applied column by column).  Every operator entry
// read from HBM and every kernel value evaluated serves all kBatch columns:
// the transfer and basis GEMVs become skinny GEMMs and the near field and M2L
// evaluate K(x_i, x_j) once per pair.  Per column, the GEMV sums (P2M, M2M,
// L2L, L2P) are those of the single-column kernels (h2s_kernels.hip): index
// order, separately rounded products and sums.  The kernel sums (near field,
// M2L) run in slice order with their own slicing, so they agree with the
// single-column results to rounding.
//
// Layout: charges, near-field potentials and coefficients of a block are
// row-major with the kBatch columns contiguous (qb[i kBatch + c]); columns
// past the block's active count are zero.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "h2s.h"
#include "h2s_device.hpp"
#include "h2s_kfun.hpp"

// Batch buffers for callers that cannot allocate (h2s_apply_noalloc): one
// array per device, alive until the process ends.  Host code never uses this
// name as an address; it takes the device address from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[H2S_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace h2s {

namespace {

constexpr int NB = kBatch;
constexpr int NT_BG = 256; // GEMV blocks (one output of a box per thread, looping if needed)

// qb[i][c] = x[c ldx + perm[i]] for the block's active columns, 0 beyond.
template <class P>
__global__ __launch_bounds__(256) void kb_permute(DevTree<P> t, const double *__restrict__ x, int64_t ldx, int na)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= t.n) return;
    const int src = t.perm[i];
#pragma unroll
    for (int c = 0; c < NB; ++c) t.qb[(size_t)i * NB + c] = c < na ? x[(size_t)c * ldx + src] : 0.0;
}

// acc[c] = sum_j A[j stride] xs[j NB + c], j in index order, for every column c.
template <bool ORD, typename AT>
__device__ __forceinline__ void ordered_dot_b(const AT *__restrict__ A, size_t stride, int R, const double *xs,
                                              double (&acc)[NB])
{
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[c] = 0.0;
    int j = 0;
    for (; j + 4 <= R; j += 4) {
        double a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = (double)A[(size_t)(j + u) * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < NB; ++c) acc[c] = madd<ORD>(acc[c], a[u], xs[(j + u) * NB + c]);
    }
    for (; j < R; ++j) {
        const double a = (double)A[(size_t)j * stride];
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[c] = madd<ORD>(acc[c], a, xs[j * NB + c]);
    }
}

// P2M: the leaf's charges are read by every thread at the same index, so they
// are read in place through the caches rather than staged.  Kept row j of U
// holds local row keep[j]; the column's unit row adds the pivot's charges where
// its row lies among the kept rows (before kept row pos).
template <class P> __global__ __launch_bounds__(NT_BG) void kb_up_leaf(DevTree<P> t, uint32_t mask)
{
    constexpr bool ORD = P::ordered;
    const int leaf = xcd_remap(blockIdx.x, gridDim.x), g = t.leaf0 + leaf, tid = threadIdx.x;
    const int b = t.box_begin[g];
    const double *qs = t.qb + (size_t)b * NB;
    const int cf = t.far.coef_off[g], rf = (mask & kFar) && t.kappa >= t.far.lmin ? t.far.coef_off[g + 1] - cf : 0;
    const int cv = t.ver.coef_off[g], rv = (mask & kVer) && t.kappa >= t.ver.lmin ? t.ver.coef_off[g + 1] - cv : 0;
    for (int k = tid; k < rf + rv; k += NT_BG) {
        const bool f = k < rf;
        const int kk = f ? k : k - rf;
        const auto *A = f ? t.far.U_rm + t.far.uoff[leaf] + kk : t.ver.U_rm + t.ver.uoff[leaf] + kk;
        const size_t stride = (size_t)(f ? rf : rv);
        const int nk = f ? t.far.unk[leaf] : t.ver.unk[leaf];
        const uint16_t *keep = (f ? t.far.ukeep : t.ver.ukeep) + b;
        const int pr = f ? t.far.uprow[cf + kk] : t.ver.uprow[cv + kk];
        const int pos = pr < 0 ? -1 : f ? t.far.upos[cf + kk] : t.ver.upos[cv + kk];
        const double *qp = qs + (size_t)(pr < 0 ? 0 : pr) * NB;
        double *out = (f ? t.far.vb + (size_t)(cf + kk) * NB : t.ver.vb + (size_t)(cv + kk) * NB);
        double acc[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[c] = 0.0;
        int j = 0;
        for (; j + 4 <= nk; j += 4) {
            double a[4];
            const double *x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = (double)A[(size_t)(j + u) * stride];
                x[u] = qs + (size_t)keep[j + u] * NB;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < NB; ++c) acc[c] = madd<ORD>(j + u == pos ? acc[c] + qp[c] : acc[c], a[u], x[u][c]);
        }
        for (; j < nk; ++j) {
            const double a = (double)A[(size_t)j * stride];
            const double *x = qs + (size_t)keep[j] * NB;
#pragma unroll
            for (int c = 0; c < NB; ++c) acc[c] = madd<ORD>(j == pos ? acc[c] + qp[c] : acc[c], a, x[c]);
        }
#pragma unroll
        for (int c = 0; c < NB; ++c) out[c] = pos == nk ? acc[c] + qp[c] : acc[c];
    }
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// M2M and L2L of every column block at once, on the FP64 matrix cores: one wave per (box, row
// tile of 16 outputs), 16x16x4 products over the contraction index in index order, one 16-column
// tile per product (two for more than 16 columns).  A transfer is read once for all columns; the
// column blocks share it.  Operand layouts: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16];
// the result holds rows l / 16 + 4 q of column l % 16.
constexpr int NT_BT = 64;

// out (rows x cols) = A (rows x K) * B (K x cols), A[i][k] = a[k * lda_k + i * lda_i], B[k] of
// column n at b_n[brow(k) * NB] (brow = bidx, or k itself); output row i goes to row orow(i) of
// out (oidx, or i); an output row i with unit[i] >= 0 also adds B row unit[i] (a unit row of the
// operator that is not stored).  Rows past `rows` and columns of absent blocks are neither read
// nor written.
struct TileIO {
    const double *a;
    size_t lda_k, lda_i;
    const double *b;         // the first column block's B[0][0]
    double *out;             // the first column block's out[0][0]
    size_t bstride;          // one column block to the next, in B and out
    int rows, K, nblk;
    bool add;                // out += A B instead of out = A B
    const uint16_t *bidx;    // or null
    const uint16_t *oidx;    // or null
    const int16_t *unit;     // or null
};

// Every load is issued unconditionally (absent rows and column blocks read row 0 and block 0)
// and masked after, so that the unrolled steps keep their loads in flight together.
template <bool TWO> __device__ __forceinline__ void tile_product_t(const TileIO &io, int tile)
{
    constexpr int U = 4; // 4-term steps per iteration
    const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
    const int i = tile * 16 + li;
    const bool iok = i < io.rows;
    const int n0 = li, n1 = 16 + li; // columns of the two tiles
    const bool ok0 = n0 / NB < io.nblk, ok1 = TWO && n1 / NB < io.nblk;
    const double *B0 = io.b + (ok0 ? (size_t)(n0 / NB) * io.bstride : 0) + n0 % NB;
    const double *B1 = io.b + (ok1 ? (size_t)(n1 / NB) * io.bstride : 0) + n1 % NB;
    const double *A = io.a + (size_t)(iok ? i : 0) * io.lda_i;
    auto brow = [&](int k) -> size_t { return (size_t)(io.bidx ? io.bidx[k] : k); };
    dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
    const int Kf = io.K & ~(4 * U - 1);
    for (int k0 = 0; k0 < Kf; k0 += 4 * U) {
        double a[U], b0[U], b1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + 4 * u + lk;
            const size_t kb = brow(k);
            a[u] = A[(size_t)k * io.lda_k];
            b0[u] = B0[kb * NB];
            if constexpr (TWO) b1[u] = B1[kb * NB];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double au = iok ? a[u] : 0.0;
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(au, ok0 ? b0[u] : 0.0, acc0, 0, 0, 0);
            if constexpr (TWO) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(au, ok1 ? b1[u] : 0.0, acc1, 0, 0, 0);
        }
    }
    for (int k0 = Kf; k0 < io.K; k0 += 4) { // the remaining terms, 4 at a time
        const int k = k0 + lk;
        const bool kok = k < io.K;
        const int kc = kok ? k : 0;
        const size_t kb = brow(kc);
        const double a = A[(size_t)kc * io.lda_k], b0 = B0[kb * NB];
        const double au = iok && kok ? a : 0.0;
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(au, ok0 ? b0 : 0.0, acc0, 0, 0, 0);
        if constexpr (TWO) {
            const double b1 = B1[kb * NB];
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(au, ok1 ? b1 : 0.0, acc1, 0, 0, 0);
        }
    }
    double *O0 = io.out + (size_t)(n0 / NB) * io.bstride + n0 % NB;
    double *O1 = io.out + (size_t)(n1 / NB) * io.bstride + n1 % NB;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int row = tile * 16 + lk + 4 * q;
        if (row < io.rows) {
            const size_t o = (size_t)(io.oidx ? io.oidx[row] : row) * NB;
            const int ur = io.unit ? io.unit[row] : -1;
            double v0 = acc0[q], v1 = acc1[q];
            if (ur >= 0) {
                v0 = v0 + B0[(size_t)ur * NB];
                if (ok1) v1 = v1 + B1[(size_t)ur * NB];
            }
            if (ok0) O0[o] = io.add ? O0[o] + v0 : v0;
            if (ok1) O1[o] = io.add ? O1[o] + v1 : v1;
        }
    }
}

__device__ __forceinline__ void tile_product(const TileIO &io, int tile)
{
    if (io.nblk * NB > 16) tile_product_t<true>(io, tile);
    else tile_product_t<false>(io, tile);
}

// M2M: the parent's multipoles (rank rows) = transfer^T (rank x kept rows) times the children's
// multipoles of the kept rows, plus the child coefficient of each unit row.  Grid: (boxes of
// the level, row tiles of the largest rank).
template <class P, bool FAR> __global__ __launch_bounds__(NT_BT) void kb_m2m_mfma(DevTree<P> t, int32_t g0, int nblk)
{
    const auto &F = [&]() -> const auto & {
        if constexpr (FAR) return t.far;
        else return t.ver;
    }();
    const int g = g0 + blockIdx.x, tile = blockIdx.y;
    const int c0 = F.coef_off[g], r = F.coef_off[g + 1] - c0;
    if (tile * 16 >= r) return; // whole wave
    const int b0 = F.coef_off[t.box_cbeg[g]];
    TileIO io;
    io.a = F.Tr_rm + F.troff[g]; // kept rows x r row-major: transfer^T[i][k] at k * r + i
    io.lda_k = (size_t)r;
    io.lda_i = 1;
    io.b = F.vb + (size_t)b0 * NB;
    io.out = F.vb + (size_t)c0 * NB;
    io.bstride = (size_t)F.ncoef * NB;
    io.rows = r;
    io.K = F.tnk[g];
    io.nblk = nblk;
    io.add = false;
    io.bidx = F.tkeep + b0;
    io.oidx = nullptr;
    io.unit = F.tprow + c0;
    tile_product(io, tile);
}

// L2L: the children's locals of the kept rows += transfer (kept rows x rank) times the parent's
// locals; the wave of tile 0 also adds the parent's local a to the child coefficient of each
// unit row e_a.  Grid: (boxes of the level, row tiles of the largest stacked transfer).
template <class P, bool FAR> __global__ __launch_bounds__(NT_BT) void kb_l2l_mfma(DevTree<P> t, int32_t g0, int nblk)
{
    const auto &F = [&]() -> const auto & {
        if constexpr (FAR) return t.far;
        else return t.ver;
    }();
    const int g = g0 + blockIdx.x, tile = blockIdx.y;
    const int c0 = F.coef_off[g], r = F.coef_off[g + 1] - c0;
    if (r == 0) return;
    const int b0 = F.coef_off[t.box_cbeg[g]], nk = F.tnk[g];
    const size_t bstride = (size_t)F.ncoef * NB;
    if (tile == 0) // unit rows: rows disjoint from the kept rows the tiles write
        for (int e = threadIdx.x; e < r * nblk * NB; e += NT_BT) {
            const int a = e / (nblk * NB), col = e % (nblk * NB), pr = F.tprow[c0 + a];
            if (pr < 0) continue;
            double *o = F.ub + (size_t)(col / NB) * bstride + (size_t)(b0 + pr) * NB + col % NB;
            *o = *o + F.ub[(size_t)(col / NB) * bstride + (size_t)(c0 + a) * NB + col % NB];
        }
    if (tile * 16 >= nk) return; // whole wave
    TileIO io;
    io.a = F.Tr_cm + F.troff[g]; // column-major kept rows x r: transfer[i][k] at k * nk + i
    io.lda_k = (size_t)nk;
    io.lda_i = 1;
    io.b = F.ub + (size_t)c0 * NB;
    io.out = F.ub + (size_t)b0 * NB;
    io.bstride = bstride;
    io.rows = nk;
    io.K = r;
    io.nblk = nblk;
    io.add = true;
    io.bidx = nullptr;
    io.oidx = F.tkeep + b0;
    io.unit = nullptr;
    tile_product(io, tile);
}

// M2L in double, slice form, kBatch columns per evaluation.  Each thread takes
// BM_TPT target pivots (a, a + NP, ...) against one slice of the staged
// sources, so the coordinates and the kBatch multipoles of a source, read
// once from LDS, serve BM_TPT evaluations and BM_TPT x kBatch multiply-adds.
constexpr int NT_BM = 256;
constexpr int BM_SRC = 512;
constexpr int BM_TPT = 4;

template <class P, bool FAR, int KIND, int D> __global__ __launch_bounds__(NT_BM) void kb_m2l(DevTree<P> t)
{
    const auto &F = [&]() -> const auto & {
        if constexpr (FAR) return t.far;
        else return t.ver;
    }();
    constexpr int TPT = BM_TPT;
    constexpr bool XW = kExtraCoord<KIND>;
    __shared__ double sx[BM_SRC], sy[BM_SRC], sz[D == 3 ? BM_SRC : 1], sw[XW ? BM_SRC : 1];
    __shared__ double sv[BM_SRC * NB]; // after the last group: the slice partials of one column
    __shared__ __align__(16) double ktab[kTabLen<KIND>];
    static_assert(BM_SRC * NB >= TPT * NT_BM, "slice partials fit in the multipole buffer");
    const int tid = threadIdx.x;
    stage_table<KIND>(t.ktab, ktab); // first used after a barrier
    const int g = F.targets[xcd_chunk_remap<kM2LChunk>(blockIdx.x, gridDim.x)];
    const int c0 = F.coef_off[g], r = F.coef_off[g + 1] - c0;
    const int e0 = F.il_off[g], e1 = F.il_off[g + 1];
    const KPar<double> kp = kpar<double>(t);
    for (int a0 = 0; a0 < r; a0 += TPT * NT_BM) {
        const int MT = min(r - a0, TPT * NT_BM), NP = (MT + TPT - 1) / TPT, NS = NT_BM / NP;
        const int s = tid / NP, pa = tid % NP;
        int it[TPT];
        double tx[TPT], ty[TPT], tz[TPT], tw[TPT];
        double acc[TPT][NB];
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            it[k] = pa + k * NP < MT ? a0 + pa + k * NP : a0 + pa; // a missing target repeats the first
            tx[k] = F.pvx[c0 + it[k]];
            ty[k] = F.pvy[c0 + it[k]];
            tz[k] = D == 3 ? (double)F.pvz[c0 + it[k]] : 0.0;
            tw[k] = XW ? (double)F.pvw[c0 + it[k]] : 0.0;
#pragma unroll
            for (int c = 0; c < NB; ++c) acc[k][c] = 0.0;
        }
        int pos = 0;
        auto flush = [&]() {
            __syncthreads();
            if (s < NS) {
                for (int j = s; j < pos; j += NS) {
                    const double x0 = sx[j], y0 = sy[j], z0 = D == 3 ? sz[j] : 0.0, w0 = XW ? sw[j] : 0.0;
                    double kv[TPT];
#pragma unroll
                    for (int k = 0; k < TPT; ++k)
                        kv[k] = kval_pos<KIND>(
                            add_extra<KIND>(dist2<false, D>(tx[k] - x0, ty[k] - y0, tz[k] - z0), tw[k], w0), kp, ktab);
#pragma unroll
                    for (int c = 0; c < NB; ++c) {
                        const double v = sv[j * NB + c];
#pragma unroll
                        for (int k = 0; k < TPT; ++k) acc[k][c] = fma(kv[k], v, acc[k][c]);
                    }
                }
            }
            __syncthreads();
            pos = 0;
        };
        for (int e = e0; e < e1; ++e) {
            const int y = F.il_idx[e];
            const int cy = F.coef_off[y], ry = F.coef_off[y + 1] - cy;
            for (int j0 = 0; j0 < ry;) {
                const int take = min(ry - j0, BM_SRC - pos);
                for (int j = tid; j < take; j += NT_BM) {
                    sx[pos + j] = F.pvx[cy + j0 + j];
                    sy[pos + j] = F.pvy[cy + j0 + j];
                    if constexpr (D == 3) sz[pos + j] = F.pvz[cy + j0 + j];
                    if constexpr (XW) sw[pos + j] = F.pvw[cy + j0 + j];
                }
                for (int e2 = tid; e2 < take * NB; e2 += NT_BM) sv[pos * NB + e2] = F.vb[(size_t)(cy + j0) * NB + e2];
                pos += take;
                j0 += take;
                if (pos == BM_SRC) flush();
            }
        }
        if (pos > 0) flush(); // ends with a barrier (or nothing was staged): sv is free
        // slice partials, one column at a time, summed in slice order
        double *const red = sv;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
#pragma unroll
            for (int k = 0; k < TPT; ++k) red[k * NT_BM + tid] = s < NS ? acc[k][c] : 0.0;
            __syncthreads();
            if (tid < NP) {
#pragma unroll
                for (int k = 0; k < TPT; ++k) {
                    double u = 0.0;
                    for (int q = 0; q < NS; ++q) u += red[k * NT_BM + q * NP + tid];
                    if (k == 0 || it[k] != it[0]) F.ub[(size_t)(c0 + it[k]) * NB + c] = u;
                }
            }
            __syncthreads();
        }
    }
}

// M2L in double on the matrix cores for up to kGroupBlocks blocks of kBatch
// columns at once: u_X (r_X x cols) += sum over Y in IL(X) of T_XY V_Y, tiled
// for v_mfma_f64_16x16x4f64 (D 16 x 16 += A 16 x 4 . B 4 x 16 per wave).  A
// holds the kernel values of 16 target pivots against 4 staged sources, one
// evaluation per lane (target lane % 16, source lane / 16); B the multipoles
// of those sources for 16 columns (column lane % 16); D is 16 targets x 16
// columns, lane l holding rows l / 16 + 4 q (q = 0..3) of column l % 16.  Two
// column tiles share every evaluation, so one kernel value serves up to 32
// columns: the vector units evaluate, the matrix cores multiply-add.  Tiles
// of 16 targets go to the 4 waves; with fewer than 4 tiles the waves of a
// tile split the 4-source steps and add their partial tiles in wave order.
// Two accumulators per column tile take alternate steps (independent MFMAs).
constexpr int NT_BMM = 256;  // 4 waves
constexpr int BMM_SRC = 64;  // staged source pivots per group
constexpr int BMM_STEPS = 4; // 4-source product steps per iteration

template <class P, bool FAR, int KIND, int D>
__global__ __launch_bounds__(NT_BMM) __attribute__((amdgpu_waves_per_eu(5))) void kb_m2l_mfma(DevTree<P> t, int nblk)
{
    constexpr int GC = kGroupCols;
    constexpr int TPS = NT_BMM / BMM_SRC, CPT = GC / TPS; // staging: threads per source, columns per thread
    static_assert(GC == 32 && TPS * BMM_SRC == NT_BMM && CPT * TPS == GC, "staging covers a group exactly");
    static_assert(BMM_SRC % (16 * BMM_STEPS) == 0 && BMM_STEPS % 2 == 0, "an iteration's steps stay inside a group");
    const auto &F = [&]() -> const auto & {
        if constexpr (FAR) return t.far;
        else return t.ver;
    }();
    constexpr bool XW = kExtraCoord<KIND>;
    __shared__ double sx[BMM_SRC], sy[BMM_SRC], sz[D == 3 ? BMM_SRC : 1], sw[XW ? BMM_SRC : 1];
    constexpr int SVS = GC + 16; // row stride of sv: rows j and j + 1 in different bank halves
    __shared__ double sv[BMM_SRC * SVS]; // after the last group: the waves' partial tiles
    __shared__ int32_t boxoff[kMaxList + 1], boxcoef[kMaxList];
    __shared__ double tx[64], ty[64], tz[D == 3 ? 64 : 1], tw[XW ? 64 : 1]; // the round's target pivots
    __shared__ __align__(16) double ktab[kTabLen<KIND>];
    static_assert(BMM_SRC * SVS >= 4 * 64 * 8, "partial tiles fit in the multipole buffer");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    stage_table<KIND>(t.ktab, ktab); // first used after a barrier
    const int g = F.targets[xcd_chunk_remap<kM2LChunk>(blockIdx.x, gridDim.x)];
    const int c0 = F.coef_off[g], r = F.coef_off[g + 1] - c0;
    const int e0 = F.il_off[g], nil = F.il_off[g + 1] - e0; // nil <= kMaxList (checked at build)
    const KPar<double> kp = kpar<double>(t);
    const size_t bstride = (size_t)F.ncoef * NB; // one block's coefficients
    const bool two = nblk * NB > 16;             // the second column tile holds active columns
    const int ntiles = (r + 15) / 16;
    if (ntiles == 0) return; // uniform over the block, before any barrier
    // the sources of IL(X) in list order as slots 0 .. S-1: slot s lies in list box e with
    // boxoff[e] <= s < boxoff[e + 1], coefficient boxcoef[e] + s - boxoff[e]
    for (int k = tid; k < nil; k += NT_BMM) {
        const int y = F.il_idx[e0 + k];
        boxcoef[k] = F.coef_off[y];
        boxoff[k + 1] = F.coef_off[y + 1] - F.coef_off[y];
    }
    __syncthreads();
    if (tid == 0) {
        boxoff[0] = 0;
        for (int k = 1; k <= nil; ++k) boxoff[k] += boxoff[k - 1];
    }
    __syncthreads();
    const int S = boxoff[nil], ngroups = (S + BMM_SRC - 1) / BMM_SRC;
    auto coef_of = [&](int s) -> int {
        int lo = 0, hi = nil - 1; // largest e with boxoff[e] <= s
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (boxoff[mid] <= s) lo = mid;
            else hi = mid - 1;
        }
        return boxcoef[lo] + (s - boxoff[lo]);
    };
    // staging of a group of BMM_SRC slots: thread tid < BMM_SRC loads slot tid's coordinates,
    // thread tid loads CPT of slot tid / TPS's 32 columns (prefetching the next group into
    // registers during the products measured no faster and spilled)
    double rx = 0.0, ry = 0.0, rz = 0.0, rw = 0.0, rv[CPT];
    auto load = [&](int gi) {
        // slots past the end of the list (last group only) repeat the group's first source
        // with zero multipoles: every product step reads a full group and adds exact zeros
        const int base = gi * BMM_SRC, take = min(BMM_SRC, S - base);
        if (tid < BMM_SRC) {
            const int c = coef_of(base + (tid < take ? tid : 0));
            rx = F.pvx[c];
            ry = F.pvy[c];
            if constexpr (D == 3) rz = F.pvz[c];
            if constexpr (XW) rw = F.pvw[c];
        }
        const int sl = tid / TPS, part = tid % TPS;
        const int c = coef_of(base + (sl < take ? sl : 0));
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int gc = part * CPT + k, bk = gc / NB;
            rv[k] = sl < take && bk < nblk ? F.vb[bk * bstride + (size_t)c * NB + gc % NB] : 0.0;
        }
    };
    auto store = [&]() {
        if (tid < BMM_SRC) {
            sx[tid] = rx;
            sy[tid] = ry;
            if constexpr (D == 3) sz[tid] = rz;
            if constexpr (XW) sw[tid] = rw;
        }
        const int sl = tid / TPS, part = tid % TPS;
#pragma unroll
        for (int k = 0; k < CPT; ++k) sv[sl * SVS + part * CPT + k] = rv[k];
    };
    const int ks = ntiles >= 3 ? 1 : 4 / ntiles; // waves per tile
    const int per_round = 4 / ks;
    for (int tb = 0; tb < ntiles; tb += per_round) {
        const int tile = tb + wave / ks, part = wave % ks;
        const bool act = tile < ntiles;
        // the round's rows tb * 16 .. through LDS (read once the first group is staged)
        if (tid < 64) {
            const int ia = tb * 16 + tid, ial = ia < r ? ia : 0; // rows past r use pivot 0, not written
            tx[tid] = F.pvx[c0 + ial];
            ty[tid] = F.pvy[c0 + ial];
            if constexpr (D == 3) tz[tid] = F.pvz[c0 + ial];
            if constexpr (XW) tw[tid] = F.pvw[c0 + ial];
        }
        double xa = 0.0, ya = 0.0, za = 0.0, wa = 0.0;
        dbl4 a0 = {0.0, 0.0, 0.0, 0.0}, a1 = a0; // column tiles 0 and 1
        for (int gi = 0; gi < ngroups; ++gi) {
            const int pos = min(BMM_SRC, S - gi * BMM_SRC);
            __syncthreads(); // every wave is done with the previous group
            load(gi);
            store();
            __syncthreads();
            if (gi == 0) {
                const int row = (wave / ks) * 16 + li; // < 64
                xa = tx[row];
                ya = ty[row];
                if constexpr (D == 3) za = tz[row];
                if constexpr (XW) wa = tw[row];
            }
            if (act) {
                // this wave's 4-source steps: part, part + ks, ... (BMM_STEPS per iteration, all inside
                // the staged group since BMM_SRC is a multiple of 4 * BMM_STEPS * ks); one accumulator
                // per column tile (dependent 16x16x4 products issue back to back)
                for (int j0 = 4 * part; j0 < pos; j0 += 4 * BMM_STEPS * ks) {
                    double kv[BMM_STEPS], v0[BMM_STEPS], v1[BMM_STEPS];
#pragma unroll
                    for (int u = 0; u < BMM_STEPS; ++u) {
                        const int j = j0 + 4 * ks * u + lk;
                        v0[u] = sv[j * SVS + li];
                        v1[u] = sv[j * SVS + 16 + li];
                        kv[u] = kval_pos<KIND>(
                            add_extra<KIND>(dist2<false, D>(xa - sx[j], ya - sy[j], za - (D == 3 ? sz[j] : 0.0)), wa,
                                            XW ? sw[j] : 0.0),
                            kp, ktab);
                    }
#pragma unroll
                    for (int u = 0; u < BMM_STEPS; u += 2) {
                        a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(kv[u], v0[u], a0, 0, 0, 0);
                        a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(kv[u + 1], v0[u + 1], a0, 0, 0, 0);
                        if (two) {
                            a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(kv[u], v1[u], a1, 0, 0, 0);
                            a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(kv[u + 1], v1[u + 1], a1, 0, 0, 0);
                        }
                    }
                }
            }
        }
        __syncthreads(); // every wave is done with sv
        const dbl4 t0 = a0, t1 = a1;
        if (ks > 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                sv[(wave * 64 + lane) * 8 + q] = t0[q];
                sv[(wave * 64 + lane) * 8 + 4 + q] = t1[q];
            }
            __syncthreads();
        }
        if (act && part == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double u0 = t0[q], u1 = t1[q];
                for (int w2 = 1; w2 < ks; ++w2) {
                    u0 += sv[((wave + w2) * 64 + lane) * 8 + q];
                    u1 += sv[((wave + w2) * 64 + lane) * 8 + 4 + q];
                }
                const int i = tile * 16 + lk + 4 * q;
                if (i < r) {
                    const int b0 = li / NB, b1 = (16 + li) / NB, c = li % NB;
                    if (b0 < nblk) F.ub[b0 * bstride + (size_t)(c0 + i) * NB + c] = u0;
                    if (two && b1 < nblk) F.ub[b1 * bstride + (size_t)(c0 + i) * NB + c] = u1;
                }
            }
        }
        __syncthreads(); // the partial tiles are read before the next round stages
    }
}

// Near field (as k_p2p), kBatch columns per evaluation; one target per thread.
constexpr int NT_BP = 256;
constexpr int BP_SRC = 512;

template <class P, int KIND, int D>
__global__ __launch_bounds__(NT_BP) void kb_p2p(DevTree<P> t, int32_t leaf_begin)
{
    using PT = typename P::pt_t;
    constexpr bool TAB = sizeof(PT) == 8;
    constexpr bool XW = kExtraCoord<KIND>;
    __shared__ PT sx[BP_SRC], sy[BP_SRC], sz[D == 3 ? BP_SRC : 1], sw[XW ? BP_SRC : 1];
    __shared__ PT sq[BP_SRC * NB];
    __shared__ double red[NT_BP];
    __shared__ __align__(16) double ktab[TAB ? kTabLen<KIND> : 2];
    const int tid = threadIdx.x;
    const int leaf = leaf_begin + xcd_remap(blockIdx.x, gridDim.x), g = t.leaf0 + leaf;
    const int b = t.box_begin[g], n = t.box_end[g] - b;
    const PT diag = (PT)t.diag;
    const KPar<PT> kp = kpar<PT>(t);
    const double *cX = t.box_ctr + 3 * g;
    if constexpr (TAB) stage_table<KIND>(t.ktab, ktab); // first used after a barrier
    for (int i0 = 0; i0 < n; i0 += NT_BP) {
        const int m = min(n - i0, NT_BP), S = NT_BP / m, s = tid / m, i = i0 + tid % m;
        const PT xi = t.px[b + i], yi = t.py[b + i], zi = D == 3 ? t.pz[b + i] : PT(0);
        const PT wi = XW ? t.pw[b + i] : PT(0);
        double acc[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[c] = 0.0;
        int pos = 0, self0 = 0, self1 = 0;
        auto slice_sum = [&](int jb, int je, auto check) {
            constexpr bool CHECK = decltype(check)::value;
            PT part[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) part[c] = 0;
            for (int j = jb + s; j < je; j += S) {
                const PT r2 = add_extra<KIND>(dist2<false, D>(xi - sx[j], yi - sy[j], zi - sz[D == 3 ? j : 0]), wi,
                                              XW ? sw[j] : PT(0));
                PT k;
                if constexpr (sizeof(PT) == 8) k = CHECK ? kval<KIND>(r2, diag, kp, ktab) : kval_pos<KIND>(r2, kp, ktab);
                else k = kval<KIND>(r2, diag, kp);
#pragma unroll
                for (int c = 0; c < NB; ++c) part[c] += k * sq[j * NB + c];
            }
#pragma unroll
            for (int c = 0; c < NB; ++c) acc[c] += (double)part[c];
        };
        auto flush = [&]() {
            __syncthreads();
            if (s < S) {
                slice_sum(0, self0, std::false_type{});
                slice_sum(self0, self1, std::true_type{});
                slice_sum(self1, pos, std::false_type{});
            }
            __syncthreads();
            pos = self0 = self1 = 0;
        };
        for (int e = t.near_off[leaf]; e < t.near_off[leaf + 1]; ++e) {
            const int gs = t.leaf0 + t.near_idx[e];
            const int sb = t.box_begin[gs], sn = t.box_end[gs] - sb;
            double dcx = 0, dcy = 0, dcz = 0;
            if constexpr (P::local) {
                dcx = t.box_ctr[3 * gs] - cX[0];
                dcy = t.box_ctr[3 * gs + 1] - cX[1];
                dcz = t.box_ctr[3 * gs + 2] - cX[2];
            }
            for (int j0 = 0; j0 < sn;) {
                const int take = min(sn - j0, BP_SRC - pos);
                for (int j = tid; j < take; j += NT_BP) {
                    const int src = sb + j0 + j;
                    if constexpr (P::local) {
                        sx[pos + j] = (PT)(dcx + (double)t.px[src]);
                        sy[pos + j] = (PT)(dcy + (double)t.py[src]);
                        if constexpr (D == 3) sz[pos + j] = (PT)(dcz + (double)t.pz[src]);
                    } else {
                        sx[pos + j] = t.px[src];
                        sy[pos + j] = t.py[src];
                        if constexpr (D == 3) sz[pos + j] = t.pz[src];
                    }
                    if constexpr (XW) sw[pos + j] = t.pw[src];
                }
                for (int e2 = tid; e2 < take * NB; e2 += NT_BP)
                    sq[pos * NB + e2] = (PT)t.qb[(size_t)(sb + j0) * NB + e2];
                if (gs == g) {
                    self0 = pos;
                    self1 = pos + take;
                }
                pos += take;
                j0 += take;
                if (pos == BP_SRC) flush();
            }
        }
        if (pos > 0) flush();
        for (int c = 0; c < NB; ++c) {
            red[tid] = s < S ? acc[c] : 0.0;
            __syncthreads();
            if (tid < m) {
                double phi = 0.0;
                for (int q = 0; q < S; ++q) phi += red[q * m + tid];
                t.ynb[(size_t)(b + i) * NB + c] = phi;
            }
            __syncthreads();
        }
    }
}

// yn + shift q + L2P of both families, scattered to user order for the
// block's active columns; threads [0, HALF) far, [HALF, NT) vertex family.
constexpr int NT_BL = 128;

template <class P>
__global__ __launch_bounds__(NT_BL) void kb_down_leaf(DevTree<P> t, double *__restrict__ y, int64_t ldy, int na,
                                                      uint32_t mask)
{
    constexpr bool ORD = P::ordered;
    constexpr int HALF = NT_BL / 2;
    using BT = typename P::basis_t;
    __shared__ double ver_part[HALF * NB];
    const int leaf = xcd_remap(blockIdx.x, gridDim.x), g = t.leaf0 + leaf;
    const int b = t.box_begin[g], n = t.box_end[g] - b;
    const int f = threadIdx.x < HALF ? 0 : 1, il = threadIdx.x - f * HALF;
    const bool on = f == 0 ? (mask & kFar) && t.kappa >= t.far.lmin : (mask & kVer) && t.kappa >= t.ver.lmin;
    const int c0 = f == 0 ? t.far.coef_off[g] : t.ver.coef_off[g];
    const int r = on ? (f == 0 ? t.far.coef_off[g + 1] : t.ver.coef_off[g + 1]) - c0 : 0;
    // kept rows of U column-major (nk x r); a unit row e_a gives the locals of a themselves
    const BT *U = f == 0 ? t.far.U_cm + t.far.uoff[leaf] : t.ver.U_cm + t.ver.uoff[leaf];
    const int16_t *urow = (f == 0 ? t.far.urow : t.ver.urow) + b;
    const int nk = r ? (f == 0 ? t.far.unk[leaf] : t.ver.unk[leaf]) : 0;
    const double *uc = (f == 0 ? t.far.ub : t.ver.ub) + (size_t)c0 * NB;
    for (int i0 = 0; i0 < n; i0 += HALF) {
        const int i = i0 + il;
        double fam[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) fam[c] = 0.0;
        if (i < n && r) {
            const int ki = urow[i];
            if (ki >= 0) ordered_dot_b<ORD>(U + ki, (size_t)nk, r, uc, fam);
            else
#pragma unroll
                for (int c = 0; c < NB; ++c) fam[c] = uc[(size_t)(~ki) * NB + c];
        }
        if (f == 1 && i < n)
#pragma unroll
            for (int c = 0; c < NB; ++c) ver_part[il * NB + c] = fam[c];
        __syncthreads();
        if (f == 0 && i < n) {
            const int dst = t.perm[b + i];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                if (c >= na) continue;
                double phi = 0.0;
                if (mask & kNear)
                    phi = madd<ORD>(t.ynb[(size_t)(b + i) * NB + c], t.shift, t.qb[(size_t)(b + i) * NB + c]);
                if (mask & kFar) phi = phi + fam[c];
                if (mask & kVer) phi = phi + ver_part[il * NB + c];
                y[(size_t)c * ldy + dst] = phi;
            }
        }
        __syncthreads();
    }
}

} // namespace
} // namespace h2s

#include "h2s_kernels_lp.hpp"

namespace h2s {
namespace {

template <class P, int KIND, int D>
hipError_t enqueue_b(const DevTree<P> &t, const LaunchPlan &plan, const double *x, int64_t ldx, double *y,
                     int64_t ldy, int ncols, uint32_t mask, const Streams &st, bool bf16)
{
    hipStream_t s = (hipStream_t)st.main, aux = (hipStream_t)st.aux;
    const int32_t *lev_off = plan.lev_off;
    const bool fam_on = (mask & (kFar | kVer)) && t.kappa >= 1;
    const bool near = (mask & kNear) != 0;
    const int nblk = (ncols + NB - 1) / NB;
    // one description per block of kBatch columns: the same tree, that block's buffers
    DevTree<P> tb[kGroupBlocks];
    for (int k = 0; k < nblk; ++k) {
        tb[k] = t;
        tb[k].qb = t.qb + (size_t)k * t.n * NB;
        tb[k].ynb = t.ynb + (size_t)k * t.n * NB;
        tb[k].far.vb = t.far.vb + (size_t)k * t.far.ncoef * NB;
        tb[k].far.ub = t.far.ub + (size_t)k * t.far.ncoef * NB;
        tb[k].ver.vb = t.ver.vb + (size_t)k * t.ver.ncoef * NB;
        tb[k].ver.ub = t.ver.ub + (size_t)k * t.ver.ncoef * NB;
    }
    auto active = [&](int k) { return min(NB, ncols - k * NB); };
    hipError_t err;
    // up: permutation, near field (second stream) and P2M block by block
    for (int k = 0; k < nblk; ++k) {
        hipLaunchKernelGGL(kb_permute<P>, dim3((t.n + 255) / 256), dim3(256), 0, s, tb[k], x + (size_t)k * NB * ldx, ldx,
                           active(k));
        if ((err = hipGetLastError()) != hipSuccess) return err;
        if (near) {
            if ((err = hipEventRecord((hipEvent_t)st.fork, s)) != hipSuccess) return err;
            if ((err = hipStreamWaitEvent(aux, (hipEvent_t)st.fork, 0)) != hipSuccess) return err;
            hipLaunchKernelGGL((kb_p2p<P, KIND, D>), dim3(t.nleaf), dim3(NT_BP), 0, aux, tb[k], 0);
        }
        if (fam_on) hipLaunchKernelGGL(kb_up_leaf<P>, dim3(t.nleaf), dim3(NT_BG), 0, s, tb[k], mask);
    }
    // M2M of every block per launch, on the matrix cores
    for (int l = t.kappa - 1; l >= 1 && fam_on; --l) {
        const int nb = lev_off[l + 1] - lev_off[l];
        const dim3 grid(nb, (t.max_rank + 15) / 16);
        if (nb && (mask & kFar)) hipLaunchKernelGGL((kb_m2m_mfma<P, true>), grid, dim3(NT_BT), 0, s, t, lev_off[l], nblk);
        if (nb && (mask & kVer)) hipLaunchKernelGGL((kb_m2m_mfma<P, false>), grid, dim3(NT_BT), 0, s, t, lev_off[l], nblk);
    }
    if (near && (err = hipEventRecord((hipEvent_t)st.join, aux)) != hipSuccess) return err;
    if (fam_on) {
        // M2L: one launch per family for every block (matrix cores when two or more blocks share it)
        if ((mask & kFar) && t.far.ntargets) {
            if constexpr (sizeof(typename P::far_t) == 4) {
                // float far field: float or bfloat16 products on the matrix cores, 32 columns a pass
                if (bf16)
                    hipLaunchKernelGGL((kb_m2l_lp<P, KIND, D, true>), dim3(t.far.ntargets), dim3(NT_LP), 0, s, t, nblk);
                else
                    hipLaunchKernelGGL((kb_m2l_lp<P, KIND, D, false>), dim3(t.far.ntargets), dim3(NT_LP), 0, s, t, nblk);
            } else if (nblk > 1) {
                hipLaunchKernelGGL((kb_m2l_mfma<P, true, KIND, D>), dim3(t.far.ntargets), dim3(NT_BMM), 0, s, t, nblk);
            } else {
                for (int k = 0; k < nblk; ++k)
                    hipLaunchKernelGGL((kb_m2l<P, true, KIND, D>), dim3(t.far.ntargets), dim3(NT_BM), 0, s, tb[k]);
            }
        }
        if ((mask & kVer) && t.ver.ntargets) {
            if (nblk > 1)
                hipLaunchKernelGGL((kb_m2l_mfma<P, false, KIND, D>), dim3(t.ver.ntargets), dim3(NT_BMM), 0, s, t, nblk);
            else
                for (int k = 0; k < nblk; ++k)
                    hipLaunchKernelGGL((kb_m2l<P, false, KIND, D>), dim3(t.ver.ntargets), dim3(NT_BM), 0, s, tb[k]);
        }
        // L2L of every block per launch, on the matrix cores
        for (int l = 1; l <= t.kappa - 1; ++l) {
            const int nb = lev_off[l + 1] - lev_off[l];
            const dim3 grid(nb, (t.max_rows + 15) / 16);
            if (nb && (mask & kFar)) hipLaunchKernelGGL((kb_l2l_mfma<P, true>), grid, dim3(NT_BT), 0, s, t, lev_off[l], nblk);
            if (nb && (mask & kVer)) hipLaunchKernelGGL((kb_l2l_mfma<P, false>), grid, dim3(NT_BT), 0, s, t, lev_off[l], nblk);
        }
    }
    if (near && (err = hipStreamWaitEvent(s, (hipEvent_t)st.join, 0)) != hipSuccess) return err;
    for (int k = 0; k < nblk; ++k)
        hipLaunchKernelGGL(kb_down_leaf<P>, dim3(t.nleaf), dim3(NT_BL), 0, s, tb[k], y + (size_t)k * NB * ldy, ldy,
                           active(k), mask);
    return hipGetLastError();
}

} // namespace

// Device address of `scratch` on the current device, looked up on the first call on each device.
hipError_t noalloc_scratch(int device, double **ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = static_cast<double *>(p);
    }
    *ptr = addr[device];
    return hipSuccess;
}

template <class P>
int launch_mvp_batch(const DevTree<P> &t, const LaunchPlan &plan, const double *x, int64_t ldx, double *y,
                     int64_t ldy, int na, uint32_t mask, const Streams &s, bool bf16) // na: columns, <= kGroupCols
{
    const int key = t.kind * 2 + (t.d == 3);
    switch (key) {
    case 0: return (int)enqueue_b<P, H2S_K_LOG_R, 2>(t, plan, x, ldx, y, ldy, na, mask, s, bf16);
    case 1: return (int)enqueue_b<P, H2S_K_LOG_R, 3>(t, plan, x, ldx, y, ldy, na, mask, s, bf16);
    case 2: return (int)enqueue_b<P, H2S_K_INV_R, 2>(t, plan, x, ldx, y, ldy, na, mask, s, bf16);
    case 3: return (int)enqueue_b<P, H2S_K_INV_R, 3>(t, plan, x, ldx, y, ldy, na, mask, s, bf16);
    case 4: return (int)enqueue_b<P, H2S_K_GAUSSIAN, 2>(t, plan, x, ldx, y, ldy, na, mask, s, bf16);
    case 5: return (int)enqueue_b<P, H2S_K_GAUSSIAN, 3>(t, plan, x, ldx, y, ldy, na, mask, s, bf16);
    case 6: return (int)enqueue_b<P, H2S_K_EXP_R, 2>(t, plan, x, ldx, y, ldy, na, mask, s, bf16);
    case 7: return (int)enqueue_b<P, H2S_K_EXP_R, 3>(t, plan, x, ldx, y, ldy, na, mask, s, bf16);
    case 8: return (int)enqueue_b<P, H2S_K_RBF_AR, 2>(t, plan, x, ldx, y, ldy, na, mask, s, bf16);
    case 9: return (int)enqueue_b<P, H2S_K_RBF_AR, 3>(t, plan, x, ldx, y, ldy, na, mask, s, bf16);
    case 10: return (int)enqueue_b<P, H2S_K_RBF_LOG, 2>(t, plan, x, ldx, y, ldy, na, mask, s, bf16);
    case 11: return (int)enqueue_b<P, H2S_K_RBF_LOG, 3>(t, plan, x, ldx, y, ldy, na, mask, s, bf16);
    case 13: // the NTI multiquadric: 3D, not with the float far field
        if constexpr (std::is_same_v<P, P32M>) return (int)hipErrorInvalidValue;
        else return (int)enqueue_b<P, H2S_K_NTI_MQ, 3>(t, plan, x, ldx, y, ldy, na, mask, s, bf16);
    default: return (int)hipErrorInvalidValue;
    }
}

template int launch_mvp_batch<P64>(const DevTree<P64> &, const LaunchPlan &, const double *, int64_t, double *,
                                   int64_t, int, uint32_t, const Streams &, bool);
template int launch_mvp_batch<P32>(const DevTree<P32> &, const LaunchPlan &, const double *, int64_t, double *,
                                   int64_t, int, uint32_t, const Streams &, bool);
template int launch_mvp_batch<P32M>(const DevTree<P32M> &, const LaunchPlan &, const double *, int64_t, double *,
                                    int64_t, int, uint32_t, const Streams &, bool);

} // namespace h2s
