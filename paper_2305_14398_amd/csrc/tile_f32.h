// One output tile of the float32 complex product of stage 5 (Section 5.3;
// Algorithm 1, result <- A . result), shared by the single-problem kernel
// (cgemm_f32.hip) and the grouped kernel (grouped.hip).
//
// C = A . B for N x N complex matrices held as float32 planes:
//   A (the step operator) column-major: A[i][k] at A[k*N + i]
//   B (the running product) row-major:  B[k][j] at B[k*N + j]
//   C row-major.
// Both operands are read as rows of length N indexed by k, so every global
// load is a contiguous 16-byte vector and a K-tile lands in LDS as [k][m]
// without a transpose.
//
// MFMA mapping (v_mfma_f32_32x32x2f32, 64 cycles, 4096 flops): lane l holds
// A[m0 + l%32][k] and B[k][n0 + l%32] with k = kbase + 8*(l/32) (the two
// k-slots of the instruction are taken 8 rows apart in the LDS tile, which
// puts the two half-waves on disjoint LDS banks with a 4-float row pad).
//   4M:  Cre += Ar.Br + (-Ai).Bi ;  Cim += Ar.Bi + Ai.Br        (4 MFMAs per k-pair)
//   3M:  T1 += Ar.Br ; T2 += Ai.Bi ; T3 += (Ar+Ai).(Br+Bi)       (3 MFMAs per k-pair)
//        Cre = T1 - T2 ;  Cim = T3 - T1 - T2
// A workgroup of KS x WM x WN waves computes a (32*WM*BMB) x (32*WN*BNB) tile
// of C; each wave owns BMB x BNB blocks of 32x32.  K-tiles of BK rows are
// double buffered in LDS; the next tile's global loads are issued before the
// MFMAs of the current one.  The tile ends with a barrier, so a persistent
// workgroup may start its next tile in the same LDS right away.
//
// KS = 2 splits every K-tile between two groups of WM x WN waves (in each
// 16-row slice, group g takes rows 4g..4g+3 and 8+4g..8+4g+3), so two waves
// share each SIMD and one hides the other's LDS and barrier stalls; each block
// is then finished by one group, which adds the other group's partial sum
// through LDS.  The 3M accumulators (192 registers a wave) leave room for only
// one wave per SIMD otherwise.  The order of the additions into each element
// depends on KS only, not on the tile size or BK.
//
// run_fused() computes the same product without a stored A: each thread
// evaluates its slice of every K-tile of the step operator from the step's
// gates (fused stages 4 and 5), where run() loads it.
#pragma once

#include "common.h"
#include "expand_entry.h"

namespace qsim {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Tile (tm, tn) of local tile id t: ids run in groups of 4 tile-rows so that
// consecutive ids share A and B panels.
__device__ __forceinline__ void grouped_tile_order(int t, int tiles_m, int tiles_n, int& tm, int& tn) {
    constexpr int GROUP_M = 4;
    const int per_group = GROUP_M * tiles_n;
    const int first_m = (t / per_group) * GROUP_M;
    const int gsize = min(tiles_m - first_m, GROUP_M);
    tm = first_m + (t % per_group) % gsize;
    tn = (t % per_group) / gsize;
}

// Blocks are dispatched round-robin over the 8 XCDs: renumber so that each
// XCD receives a contiguous range of tile ids (whose panels then share that
// XCD's L2).
__device__ __forceinline__ int xcd_contiguous_id(int bid, int nblk) {
    return ((nblk & 7) == 0) ? (bid & 7) * (nblk >> 3) + (bid >> 3) : bid;
}

template <int WM, int WN, int BMB, int BNB, bool GAUSS, int KS = 1, int BK = 16>
struct F32Tile {
    static_assert(KS == 1 || KS == 2, "the k range splits over one or two wave groups");
    static_assert(BK % 16 == 0, "K-tiles are whole 16-row slices");
    static constexpr int NT = 64 * WM * WN * KS;
    static constexpr int TM = 32 * WM * BMB;
    static constexpr int TN = 32 * WN * BNB;
    static constexpr int LDA = TM + 4;
    static constexpr int LDB = TN + 4;
    static constexpr int A_V4 = BK * TM / 4 / NT;  // float4 loads per thread per plane
    static constexpr int B_V4 = BK * TN / 4 / NT;
    static_assert(A_V4 * NT * 4 == BK * TM && B_V4 * NT * 4 == BK * TN, "tile/thread mismatch");
    static constexpr int NACC = GAUSS ? 3 : 2;
    static constexpr int STAGE_FLOATS = 2 * 2 * BK * (LDA + LDB);
    static constexpr int XCHG_FLOATS = KS == 2 ? 2 * WM * WN * 2 * 64 * 16 : 0;  // [group][wave][re/im][lane][16]
    static constexpr int SMEM_FLOATS = STAGE_FLOATS > XCHG_FLOATS ? STAGE_FLOATS : XCHG_FLOATS;

    // Entries S[r + c][s], c = 0..3, of a step operator (column s of A).
    __device__ __forceinline__ static void synth_a(const DevStep& st, uint32_t r, uint32_t s, floatx4& re,
                                                   floatx4& im) {
        double vr[4], vi[4];
        step_entries4(st, r, s, vr, vi);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            re[c] = (float)vr[c];
            im[c] = (float)vi[c];
        }
    }

    // PIN: hold the LDS read order below with scheduling barriers (the
    // grouped kernel, whose job lookup keeps more registers live, leaves the
    // order to the compiler to stay within 256 registers).
    template <bool PIN = true>
    __device__ __forceinline__ static void run(int n, const float* __restrict__ A, const float* __restrict__ B,
                                               float* __restrict__ C, int tm, int tn, float* smem) {
        run_impl<false, PIN>(n, A, nullptr, B, C, tm, tn, smem);
    }

    // Stages 4 and 5 fused: the A operand (the step operator) is never
    // stored; each K-tile of it is computed from the step's gates by the same
    // per-entry rule, in float64 rounded once, as the expansion kernel, so the
    // product is bit-identical to expanding S and calling run().
    __device__ __forceinline__ static void run_fused(int n, const DevStep& st, const float* __restrict__ B,
                                                     float* __restrict__ C, int tm, int tn, float* smem) {
        run_impl<true, false>(n, nullptr, &st, B, C, tm, tn, smem);
    }

    template <bool FUSED, bool PIN>
    __device__ __forceinline__ static void run_impl(int n, const float* __restrict__ A, const DevStep* st,
                                                    const float* __restrict__ B, float* __restrict__ C, int tm,
                                                    int tn, float* smem) {
        auto As = reinterpret_cast<float(*)[2][BK][LDA]>(smem);
        auto Bs = reinterpret_cast<float(*)[2][BK][LDB]>(smem + 2 * 2 * BK * LDA);
        const int N = 1 << n;
        const size_t NN = (size_t)N * N;
        const int i0 = tm * TM, j0 = tn * TN;
        const int tid = threadIdx.x;
        const int lane = tid & 63;
        const int wave = (tid >> 6) % (WM * WN);
        const int kgrp = (tid >> 6) / (WM * WN);
        const int wm = wave % WM, wn = wave / WM;
        const int lrow = lane & 31;
        const int khalf = (lane >> 5) * 8;

        floatx16 acc[BMB][BNB][NACC];
#pragma unroll
        for (int x = 0; x < BMB; ++x)
#pragma unroll
            for (int y = 0; y < BNB; ++y)
#pragma unroll
                for (int z = 0; z < NACC; ++z)
#pragma unroll
                    for (int e = 0; e < 16; ++e) acc[x][y][z][e] = 0.f;

        // Per-thread slice of a K-tile: float4 number f = tid + NT*u of a plane
        // covers row f / (T/4) and columns 4*(f % (T/4)) .. +3 of that tile.
        floatx4 ra[2][A_V4], rb[2][B_V4];
#define QSIM_GLOAD(k0)                                                                                   \
    if constexpr (FUSED) {                                                                               \
        _Pragma("unroll") for (int u = 0; u < A_V4; ++u) {                                               \
            const int f = tid + NT * u;                                                                   \
            synth_a(*st, (uint32_t)(i0 + (f % (TM / 4)) * 4), (uint32_t)((k0) + f / (TM / 4)), ra[0][u], \
                    ra[1][u]);                                                                            \
        }                                                                                                 \
    }                                                                                                     \
    _Pragma("unroll") for (int p = 0; p < 2; ++p) {                                                      \
        if constexpr (!FUSED) {                                                                           \
            _Pragma("unroll") for (int u = 0; u < A_V4; ++u) {                                           \
                const int f = tid + NT * u;                                                               \
                ra[p][u] = *reinterpret_cast<const floatx4*>(A + p * NN +                                \
                                                             (size_t)((k0) + f / (TM / 4)) * N + i0 +    \
                                                             (f % (TM / 4)) * 4);                         \
            }                                                                                             \
        }                                                                                                 \
        _Pragma("unroll") for (int u = 0; u < B_V4; ++u) {                                               \
            const int f = tid + NT * u;                                                                   \
            rb[p][u] = *reinterpret_cast<const floatx4*>(B + p * NN + (size_t)((k0) + f / (TN / 4)) * N + \
                                                         j0 + (f % (TN / 4)) * 4);                        \
        }                                                                                                 \
    }
#define QSIM_LSTORE(s)                                                                          \
    _Pragma("unroll") for (int p = 0; p < 2; ++p) {                                             \
        _Pragma("unroll") for (int u = 0; u < A_V4; ++u) {                                      \
            const int f = tid + NT * u;                                                          \
            *reinterpret_cast<floatx4*>(&As[s][p][f / (TM / 4)][(f % (TM / 4)) * 4]) = ra[p][u]; \
        }                                                                                        \
        _Pragma("unroll") for (int u = 0; u < B_V4; ++u) {                                      \
            const int f = tid + NT * u;                                                          \
            *reinterpret_cast<floatx4*>(&Bs[s][p][f / (TN / 4)][(f % (TN / 4)) * 4]) = rb[p][u]; \
        }                                                                                        \
    }

        // Fragments of k-step t+1 are read from LDS before the MFMAs of step t
        // are issued, so their latency hides behind those MFMAs.  The next
        // K-tile is staged before the last k-step of the current one: after
        // the barrier, its first fragments are read while that step's MFMAs
        // run, so no wave waits on LDS at a K-tile boundary.  Scheduling
        // barriers hold that order against the compiler, which otherwise sinks
        // the reads below the MFMAs.  Without PIN (the fused tile, whose entry
        // synthesis shares the K-tile's instruction stream, and the grouped
        // kernel, which would exceed 256 registers) the plain order is kept:
        // each k-step reads its fragments, the next K-tile is stored last.
        constexpr int TS = BK / 2 / KS;
        static_assert(TS % 2 == 0, "step t uses fragment buffer t & 1 in every K-tile");
        float fr[2][4][BMB > BNB ? BMB : BNB];  // [buffer][ar, ai, br, bi][block]
        auto read_frags = [&](int stage, int t, int buf) {
            const int kk = (t / (8 / KS)) * 16 + kgrp * (8 / KS) + t % (8 / KS) + khalf;
#pragma unroll
            for (int x = 0; x < BMB; ++x) {
                const int m = wm * (32 * BMB) + x * 32 + lrow;
                fr[buf][0][x] = As[stage][0][kk][m];
                fr[buf][1][x] = As[stage][1][kk][m];
            }
#pragma unroll
            for (int y = 0; y < BNB; ++y) {
                const int c = wn * (32 * BNB) + y * 32 + lrow;
                fr[buf][2][y] = Bs[stage][0][kk][c];
                fr[buf][3][y] = Bs[stage][1][kk][c];
            }
        };

        // The MFMAs of one k-step on fragments (ar, ai, br, bi) of each block.
        auto mma_step = [&](const float* ar, const float* ai, const float* br, const float* bi) {
#pragma unroll
            for (int x = 0; x < BMB; ++x) {
#pragma unroll
                for (int y = 0; y < BNB; ++y) {
                    if constexpr (!GAUSS) {
                        acc[x][y][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[x], br[y], acc[x][y][0], 0, 0, 0);
                        acc[x][y][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai[x], bi[y], acc[x][y][0], 0, 0, 0);
                        acc[x][y][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[x], bi[y], acc[x][y][1], 0, 0, 0);
                        acc[x][y][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[x], br[y], acc[x][y][1], 0, 0, 0);
                    } else {
                        acc[x][y][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[x], br[y], acc[x][y][0], 0, 0, 0);
                        acc[x][y][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[x], bi[y], acc[x][y][1], 0, 0, 0);
                        acc[x][y][2] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[x] + ai[x], br[y] + bi[y],
                                                                            acc[x][y][2], 0, 0, 0);
                    }
                }
            }
        };

        const int KT = N / BK;
        QSIM_GLOAD(0);
        QSIM_LSTORE(0);
        __syncthreads();
        if constexpr (PIN) {
            read_frags(0, 0, 0);
            for (int kt = 0; kt < KT; ++kt) {
                const int cur = kt & 1;
                const bool more = kt + 1 < KT;
                if (more) { QSIM_GLOAD((kt + 1) * BK); }
#pragma unroll
                for (int t = 0; t < TS; ++t) {
                    __builtin_amdgcn_sched_barrier(0);
                    if (t + 1 < TS) {
                        read_frags(cur, t + 1, (t + 1) & 1);
                    } else {
                        // every read of stage cur ^ 1 (the previous K-tile)
                        // was issued before the previous barrier
                        if (more) { QSIM_LSTORE(cur ^ 1); }
                        __syncthreads();
                        if (more) read_frags(cur ^ 1, 0, 0);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    mma_step(fr[t & 1][0], fr[t & 1][1], fr[t & 1][2], fr[t & 1][3]);
                }
            }
        } else {
            // Each k-step reads its own fragments; the next K-tile is stored
            // after the current one's MFMAs.
            for (int kt = 0; kt < KT; ++kt) {
                const int cur = kt & 1;
                if (kt + 1 < KT) { QSIM_GLOAD((kt + 1) * BK); }
#pragma unroll
                for (int t = 0; t < TS; ++t) {
                    read_frags(cur, t, 0);
                    mma_step(fr[0][0], fr[0][1], fr[0][2], fr[0][3]);
                }
                if (kt + 1 < KT) { QSIM_LSTORE(cur ^ 1); }
                __syncthreads();
            }
        }
#undef QSIM_GLOAD
#undef QSIM_LSTORE

        // Complex value of each 32x32 block (over this wave's k rows) into
        // accumulators 0 (real) and 1 (imaginary).
        if constexpr (GAUSS) {
#pragma unroll
            for (int x = 0; x < BMB; ++x)
#pragma unroll
                for (int y = 0; y < BNB; ++y) {
                    const floatx16 t1 = acc[x][y][0], t2 = acc[x][y][1];
                    acc[x][y][0] = t1 - t2;
                    acc[x][y][1] = acc[x][y][2] - t1 - t2;
                }
        }

        // k split over two groups: block b (= x*BNB + y) is finished by group
        // b & 1.  Blocks go in pairs, one each way per round; an odd last block
        // goes from group 1 to group 0.  Block indices are compile-time after
        // unrolling, so the accumulators stay in registers.
        if constexpr (KS == 2) {
            floatx16* xch = reinterpret_cast<floatx16*>(smem);
            constexpr int NB = BMB * BNB;
            auto slot = [&](int g, int z) { return ((g * (WM * WN) + wave) * 2 + z) * 64 + lane; };
#pragma unroll
            for (int b = 0; b < NB; b += 2) {
                const int x0 = b / BNB, y0 = b % BNB;
                if (b + 1 < NB) {
                    const int x1 = (b + 1) / BNB, y1 = (b + 1) % BNB;
#pragma unroll
                    for (int z = 0; z < 2; ++z) xch[slot(kgrp, z)] = kgrp ? acc[x0][y0][z] : acc[x1][y1][z];
                    __syncthreads();
#pragma unroll
                    for (int z = 0; z < 2; ++z) {
                        const floatx16 r = xch[slot(kgrp ^ 1, z)];
                        if (kgrp)
                            acc[x1][y1][z] += r;
                        else
                            acc[x0][y0][z] += r;
                    }
                } else {
                    if (kgrp) {
#pragma unroll
                        for (int z = 0; z < 2; ++z) xch[slot(1, z)] = acc[x0][y0][z];
                    }
                    __syncthreads();
                    if (!kgrp) {
#pragma unroll
                        for (int z = 0; z < 2; ++z) acc[x0][y0][z] += xch[slot(1, z)];
                    }
                }
                __syncthreads();
            }
        }

        // Accumulator layout of a 32x32 block: register e of lane l is
        // row 8*(e/4) + 4*(l/32) + e%4, column l%32.
#pragma unroll
        for (int x = 0; x < BMB; ++x) {
#pragma unroll
            for (int y = 0; y < BNB; ++y) {
                if (KS == 2 && ((x * BNB + y) & 1) != kgrp) continue;
                const int col = j0 + wn * (32 * BNB) + y * 32 + lrow;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int row = i0 + wm * (32 * BMB) + x * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                    C[(size_t)row * N + col] = acc[x][y][0][e];
                    C[NN + (size_t)row * N + col] = acc[x][y][1][e];
                }
            }
        }
    }
};

// Tile shapes of the single-problem and grouped products: 128 x 128 and
// 64 x 64, with the k range split over two wave groups for 3M.  Both kernels
// use these same shapes, so a product gives the same bits in either.
template <bool GAUSS>
struct F32Shapes {
    using T128 = F32Tile<2, 2, 2, 2, GAUSS, GAUSS ? 2 : 1, 16>;
    using T64 = F32Tile<2, 2, 1, 1, GAUSS, GAUSS ? 2 : 1, GAUSS ? 32 : 16>;
    static constexpr int THREADS = T128::NT;
    static_assert(T64::NT == THREADS, "both shapes run in workgroups of the same size");
    static constexpr int SMEM_FLOATS =
        T128::SMEM_FLOATS > T64::SMEM_FLOATS ? T128::SMEM_FLOATS : T64::SMEM_FLOATS;
};

// Whole product for N <= 32 by a workgroup of `nthreads` threads, one output
// entry per thread and pass, plain float32 FMAs (same 4M / 3M arithmetic).
// With `st` set, A is the step operator computed entry by entry (fused
// stages 4 and 5, the same values the expansion kernel stores).
template <bool GAUSS>
__device__ __forceinline__ void f32_small_product(int n, const float* __restrict__ A, const DevStep* st,
                                                  const float* __restrict__ B, float* __restrict__ C, int first,
                                                  int stride) {
    const int N = 1 << n;
    const int NN = N * N;
    for (int idx = first; idx < NN; idx += stride) {
        const int i = idx / N, j = idx % N;
        float t1 = 0.f, t2 = 0.f, t3 = 0.f;
        for (int k = 0; k < N; ++k) {
            float ar, ai;
            if (st != nullptr) {
                double vr, vi;
                step_entry(*st, (uint32_t)i, (uint32_t)k, vr, vi);
                ar = (float)vr;
                ai = (float)vi;
            } else {
                ar = A[k * N + i];
                ai = A[NN + k * N + i];
            }
            const float br = B[k * N + j], bi = B[NN + k * N + j];
            if constexpr (!GAUSS) {
                t1 = fmaf(ar, br, t1);
                t1 = fmaf(-ai, bi, t1);
                t2 = fmaf(ar, bi, t2);
                t2 = fmaf(ai, br, t2);
            } else {
                t1 = fmaf(ar, br, t1);
                t2 = fmaf(ai, bi, t2);
                t3 = fmaf(ar + ai, br + bi, t3);
            }
        }
        if constexpr (!GAUSS) {
            C[idx] = t1;
            C[NN + idx] = t2;
        } else {
            C[idx] = t1 - t2;
            C[NN + idx] = t3 - t1 - t2;
        }
    }
}

}  // namespace qsim
