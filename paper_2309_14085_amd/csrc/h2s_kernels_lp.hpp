// h2s_kernels_lp.hpp -- the far-field M2L of the batched product in low
// precision on the matrix cores (included by h2s_kernels_batch.hip).
//
// u_X (r_X x cols) += sum over Y in IL_far(X) of T_XY V_Y with T_XY =
// K(t^{X,i}, t^{Y,i}) (Sec. 3.4.3), for the float far field of the FP32_M2L and
// FP32_BF16M2L policies: pivot coordinates are float offsets from their box's
// centre, so a source is moved into the target box's frame in double once
// when it is staged.  The kernel values are evaluated in float on the vector
// units; the products run on the matrix cores, accumulating in float:
//   FP32: v_mfma_f32_16x16x4f32, A = 16 targets x 4 sources (one value per
//         lane), B = 4 sources x 16 columns;
//   BF16: v_mfma_f32_16x16x32_bf16, A = 16 targets x 32 sources (8 values per
//         lane, rounded to bfloat16), B = 32 sources x 16 columns.
// Two column tiles share every kernel value (32 columns).  For log r the
// value is split as 0.5 log|c|^2 + 0.5 log(r^2 / |c|^2), c the difference of
// the two box centres: the matrix cores take the second term, and the first,
// constant over a source box, is added in double as sum_b 0.5 log|c_b|^2 v_b.
#pragma once

namespace h2s {
namespace {

constexpr int NT_LP = 256;   // 4 waves
constexpr int LP_SRC = 128;  // staged sources per group (a multiple of 32)

typedef float lp_floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 lp_bf16x8 __attribute__((ext_vector_type(8)));

// row of the 16 x 16 product tile held by lane `lane`, item q (both instructions)
__device__ __forceinline__ int lp_row(int lane, int q) { return 4 * (lane >> 4) + q; }

template <class P, int KIND, int D, bool BF16>
__global__ __launch_bounds__(NT_LP) void kb_m2l_lp(DevTree<P> t, int nblk)
{
    constexpr int GC = kGroupCols;
    constexpr bool SPLIT = KIND == H2S_K_LOG_R;
    constexpr int KSTEP = BF16 ? 32 : 4; // sources per product
    static_assert(LP_SRC % 32 == 0 && NT_LP == 2 * LP_SRC, "staging: two threads per source");
    const auto &F = t.far;
    __shared__ float sx[LP_SRC], sy[LP_SRC], sz[D == 3 ? LP_SRC : 1], sic[SPLIT ? LP_SRC : 1];
    __shared__ double slc[SPLIT ? LP_SRC : 1];
    constexpr int SVS = GC + 1; // row stride of the staged multipoles (floats)
    __shared__ float sv[LP_SRC * SVS];
    __shared__ float tx[64], ty[64], tz[D == 3 ? 64 : 1];
    __shared__ double corr[GC];                  // the split's double term, per column
    __shared__ float part[4 * 64 * 8];           // partial tiles of the waves that share one
    __shared__ int32_t boxoff[kMaxList + 1], boxcoef[kMaxList], boxid[kMaxList];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int g = F.targets[xcd_chunk_remap<kM2LChunk>(blockIdx.x, gridDim.x)];
    const int c0 = F.coef_off[g], r = F.coef_off[g + 1] - c0;
    const int e0 = F.il_off[g], nil = F.il_off[g + 1] - e0;
    const KPar<float> kp = kpar<float>(t);
    const float diag = (float)t.diag;
    const double *cX = t.box_ctr + 3 * g;
    const size_t bstride = (size_t)F.ncoef * kBatch;
    const bool two = nblk * kBatch > 16;
    const int ntiles = (r + 15) / 16;
    if (ntiles == 0) return; // uniform over the block
    for (int k = tid; k < nil; k += NT_LP) {
        const int y = F.il_idx[e0 + k];
        boxid[k] = y;
        boxcoef[k] = F.coef_off[y];
        boxoff[k + 1] = F.coef_off[y + 1] - F.coef_off[y];
    }
    if (tid < GC) corr[tid] = 0.0;
    __syncthreads();
    if (tid == 0) {
        boxoff[0] = 0;
        for (int k = 1; k <= nil; ++k) boxoff[k] += boxoff[k - 1];
    }
    __syncthreads();
    const int S = boxoff[nil], ngroups = (S + LP_SRC - 1) / LP_SRC;
    auto box_of = [&](int s) -> int {
        int lo = 0, hi = nil - 1; // largest e with boxoff[e] <= s
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (boxoff[mid] <= s) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    };
    // stage group gi: thread pair (2 s, 2 s + 1) takes source s; the even one its coordinates,
    // both half of its 32 columns.  Slots past the list repeat the group's first source with
    // zero multipoles, so every product step reads a full group and adds exact zeros.
    auto stage = [&](int gi) {
        const int base = gi * LP_SRC, take = min(LP_SRC, S - base);
        const int sl = tid >> 1, half = tid & 1;
        const bool real = sl < take;
        const int e = box_of(base + (real ? sl : 0));
        const int c = boxcoef[e] + (base + (real ? sl : 0) - boxoff[e]);
        if (half == 0) {
            const int y = boxid[e];
            const double dx = t.box_ctr[3 * y] - cX[0], dy = t.box_ctr[3 * y + 1] - cX[1];
            const double dz = D == 3 ? t.box_ctr[3 * y + 2] - cX[2] : 0.0;
            sx[sl] = (float)(dx + (double)F.pvx[c]);
            sy[sl] = (float)(dy + (double)F.pvy[c]);
            if constexpr (D == 3) sz[sl] = (float)(dz + (double)F.pvz[c]);
            if constexpr (SPLIT) {
                const double c2 = dx * dx + dy * dy + dz * dz;
                sic[sl] = (float)(1.0 / c2);
                slc[sl] = real ? 0.5 * log(c2) : 0.0;
            }
        }
#pragma unroll
        for (int k = 0; k < GC / 2; ++k) {
            const int col = half * (GC / 2) + k, bk = col / kBatch;
            sv[sl * SVS + col] =
                real && bk < nblk ? (float)F.vb[bk * bstride + (size_t)c * kBatch + col % kBatch] : 0.0f;
        }
    };
    const int ks = ntiles >= 3 ? 1 : 4 / ntiles; // waves per tile
    const int per_round = 4 / ks;
    for (int tb = 0; tb < ntiles; tb += per_round) {
        const int tile = tb + wave / ks, wpart = wave % ks;
        const bool act = tile < ntiles;
        if (tid < 64) {
            const int ia = tb * 16 + tid, ial = ia < r ? ia : 0;
            tx[tid] = (float)F.pvx[c0 + ial];
            ty[tid] = (float)F.pvy[c0 + ial];
            if constexpr (D == 3) tz[tid] = (float)F.pvz[c0 + ial];
        }
        float xa = 0.f, ya = 0.f, za = 0.f;
        lp_floatx4 a0 = {0.f, 0.f, 0.f, 0.f}, a1 = a0;
        for (int gi = 0; gi < ngroups; ++gi) {
            __syncthreads(); // every wave is done with the previous group
            stage(gi);
            __syncthreads();
            if (gi == 0) {
                const int row = (wave / ks) * 16 + li;
                xa = tx[row];
                ya = ty[row];
                if constexpr (D == 3) za = tz[row];
            }
            if constexpr (SPLIT) {
                // the split's constant term: corr[col] += sum over the group of 0.5 log|c|^2 v, once
                if (tb == 0 && tid < GC) {
                    double sacc = 0.0;
                    for (int j = 0; j < LP_SRC; ++j) sacc += slc[j] * (double)sv[j * SVS + tid];
                    corr[tid] += sacc;
                }
            }
            if (act) {
                auto kv = [&](int j) -> float {
                    const float r2 = dist2<false, D>(xa - sx[j], ya - sy[j], za - (D == 3 ? sz[j] : 0.f));
                    if constexpr (SPLIT) return __log2f(r2 * sic[j]) * 0.34657359027997264f; // ln 2 / 2
                    else return kval<KIND>(r2, diag, kp);
                };
                for (int j0 = KSTEP * wpart; j0 < LP_SRC; j0 += KSTEP * ks) {
                    if constexpr (BF16) {
                        lp_bf16x8 av, b0, b1;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const int j = j0 + 8 * lk + e;
                            av[e] = (__bf16)kv(j);
                            b0[e] = (__bf16)sv[j * SVS + li];
                            b1[e] = (__bf16)sv[j * SVS + 16 + li];
                        }
                        a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b0, a0, 0, 0, 0);
                        if (two) a1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b1, a1, 0, 0, 0);
                    } else {
                        const int j = j0 + lk;
                        const float av = kv(j);
                        a0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, sv[j * SVS + li], a0, 0, 0, 0);
                        if (two) a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, sv[j * SVS + 16 + li], a1, 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads(); // corr and the staged group are complete
        if (ks > 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                part[(wave * 64 + lane) * 8 + q] = a0[q];
                part[(wave * 64 + lane) * 8 + 4 + q] = a1[q];
            }
            __syncthreads();
        }
        if (act && wpart == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double u0 = a0[q], u1 = a1[q];
                for (int w2 = 1; w2 < ks; ++w2) {
                    u0 += part[((wave + w2) * 64 + lane) * 8 + q];
                    u1 += part[((wave + w2) * 64 + lane) * 8 + 4 + q];
                }
                const int i = tile * 16 + lp_row(lane, q);
                if (i < r) {
                    const int b0 = li / kBatch, b1 = (16 + li) / kBatch, cc = li % kBatch;
                    if (b0 < nblk) F.ub[b0 * bstride + (size_t)(c0 + i) * kBatch + cc] = u0 + (SPLIT ? corr[li] : 0.0);
                    if (two && b1 < nblk)
                        F.ub[b1 * bstride + (size_t)(c0 + i) * kBatch + cc] = u1 + (SPLIT ? corr[16 + li] : 0.0);
                }
            }
        }
        __syncthreads(); // the partial tiles are read before the next round stages
    }
}

} // namespace
} // namespace h2s
