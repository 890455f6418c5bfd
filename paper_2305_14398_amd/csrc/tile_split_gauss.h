// One output tile of the stage-5 product (Section 5.3; Algorithm 1) with split
// 16-bit operands, in Gauss's three-product form, shared by the single-problem
// kernel (cgemm_split.hip) and the grouped kernel (grouped.hip).
//
// With X = Xr + i Xi and Y = Yr + i Yi (k-contiguous rows, D = X Y^T):
//   T1 = Xr Yr^T,  T2 = Xi Yi^T,  T3 = (Xr + Xi)(Yr + Yi)^T,
//   Re D = T1 - T2,  Im D = T3 - T1 - T2,
// three real products instead of four.  Each operand component c in {r, i, s}
// (s the float32 sum r + i, rounded once and then split) is carried as
// hi + lo, and each real product in three passes hi hi + hi lo + lo hi (lo lo
// dropped), so a complex product issues 9 MFMAs per 16-deep k-block where the
// four-product form issues 12.  One float32 accumulator per real product:
//   bf16: lo is unscaled, T += hx hy + hx ly + lx hy directly;
//   fp16: lo is stored scaled by 2^12 (clear of fp16 subnormals); the hi x hi
//         pass takes the X hi fragment scaled by 2^12 as well (an exact power
//         of two; entries and sums of unit-norm operands stay far below the
//         fp16 limit once scaled), so the accumulator holds 2^12 T and the
//         epilogue scales back exactly.
//
// Operand buffers hold six 16-bit planes: re_hi, re_lo, im_hi, im_lo, sum_hi,
// sum_lo (12 N^2 bytes).  From n = 6 on they are fragment-blocked: the rows
// (index i) and the contraction index k are cut into 32 x 16 blocks, block
// (i / 32, k / 16) holds its six planes as six contiguous 1 KiB fragments in
// MFMA lane order (lane (i % 32) + 32 ((k / 8) % 2), eight consecutive k per
// lane), and blocks follow in row-block-major, k-block-minor order:
//   element (p, i, k) at ((((i/32) (N/16) + k/16) 6 + p) 512
//                         + ((i % 32) + 32 ((k/8) % 2)) 8 + k % 8.
// A K-tile of 128 rows is then four contiguous 6 KiB runs, every fetched cache
// line is used whole, and a fragment is one 1 KiB read (the planar layout with
// 16-deep K-tiles used a quarter of each 128-byte line per K-tile and re-read
// the rest from HBM later, 14x the operand bytes at 12 qubits).  Below n = 6
// the planes are planar N x N (the one-workgroup path).  Output: float32 planar
// row-major (D_f32) and/or the six split planes, fragment-blocked (D_split),
// written from the float32 results.
//
// The MFMA takes the Y fragment as its A operand and the X fragment as its B
// operand, so an accumulator block is D transposed: lane l holds row
// i = l % 32 and, in registers 4g .. 4g+3, the four consecutive columns
// j = 8 g + 4 (l / 32) + 0..3; every store is a packed 8-byte (16-bit planes)
// or 16-byte (float32) vector.
//
// Tiling: 256 threads, 2 x 2 waves, each wave 2 x 2 blocks of 32 x 32 (a
// 128 x 128 tile; 192 accumulator registers, one wave per SIMD).  K-steps of 16
// go through a ring of three LDS stages (6 planes x 2 operands x 128 rows x
// 32 B = 48 KiB each, 144 KiB), stored in the same fragment order as in HBM,
// so every LDS write and fragment read is 1 KiB contiguous across the wave (no
// bank conflicts).  With one wave per SIMD nothing else hides latency, so the
// tile pipelines it: a stage's global loads are issued two k-steps before it
// is stored to LDS (two register sets), a stage is stored two k-steps before
// it is used (the ring), and each component's fragments are read from LDS
// while the previous component's 12 MFMAs run, across k-steps too (the next
// step's stage was made visible a barrier earlier).  One barrier per k-step
// guards the reuse of the oldest stage.
#pragma once

#include "tile_split.h"

namespace qsim {

// x * 2^12 for the eight fp16 values of a fragment (exact: a power of two; no
// overflow while |x| < 16, which unit-norm operands and their sums satisfy).
// Four v_pk_mul_f16, one per register; written on the whole 8-vector (a
// per-element bit cast of the registers compiled to one multiply whose result
// was copied into all four).
__device__ __forceinline__ u32x4 f16x8_times_4096(u32x4 v) {
    halfx8 h = __builtin_bit_cast(halfx8, v);
    h = h * (_Float16)4096.0f;
    return __builtin_bit_cast(u32x4, h);
}

// Split the four float32 results re[q], im[q] (and their float32 sums) of
// four consecutive entries at o into the six planes (plane stride `ps`
// elements), one 8-byte store per plane.
template <int FMT>
__device__ __forceinline__ void store_split6(uint16_t* __restrict__ D, size_t ps, size_t o, const float (&re)[4],
                                             const float (&im)[4]) {
    uint16_t h[6][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        split_f32<FMT>(re[q], h[0][q], h[1][q]);
        split_f32<FMT>(im[q], h[2][q], h[3][q]);
        split_f32<FMT>(re[q] + im[q], h[4][q], h[5][q]);
    }
#pragma unroll
    for (int p = 0; p < 6; ++p)
        *reinterpret_cast<uint2*>(D + p * ps + o) =
            make_uint2((uint32_t)h[p][0] | ((uint32_t)h[p][1] << 16), (uint32_t)h[p][2] | ((uint32_t)h[p][3] << 16));
}

// N < 32: one thread per output entry, the same three-product arithmetic in float32.
template <int FMT>
__device__ __forceinline__ void split_small_product_gauss(int n, const uint16_t* __restrict__ X,
                                                          const uint16_t* __restrict__ Y, uint16_t* __restrict__ Dsplit,
                                                          float* __restrict__ Df32, int first, int stride) {
    const int N = 1 << n;
    const int NN = N * N;
    const float s = (FMT == FMT_F16) ? 1.0f / (float)(1 << QSIM_LO_SCALE_LOG2) : 1.0f;
    for (int idx = first; idx < NN; idx += stride) {
        const int i = idx / N, j = idx % N;
        float t[3] = {0.f, 0.f, 0.f};
        for (int k = 0; k < N; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float xh = to_f32<FMT>(X[2 * c * NN + i * N + k]), xl = to_f32<FMT>(X[(2 * c + 1) * NN + i * N + k]);
                const float yh = to_f32<FMT>(Y[2 * c * NN + j * N + k]), yl = to_f32<FMT>(Y[(2 * c + 1) * NN + j * N + k]);
                // (hi hi) + (hi lo + lo hi) * s, with lo pre-scaled by 1 / s for fp16
                t[c] = fmaf(xh, yh, fmaf(fmaf(xh, yl, xl * yh), s, t[c]));
            }
        }
        const float re = t[0] - t[1], imv = (t[2] - t[0]) - t[1];
        if (Df32) {
            Df32[idx] = re;
            Df32[NN + idx] = imv;
        }
        if (Dsplit) {
            uint16_t h, l;
            split_f32<FMT>(re, h, l);
            Dsplit[idx] = h;
            Dsplit[NN + idx] = l;
            split_f32<FMT>(imv, h, l);
            Dsplit[2 * NN + idx] = h;
            Dsplit[3 * NN + idx] = l;
            split_f32<FMT>(re + imv, h, l);
            Dsplit[4 * NN + idx] = h;
            Dsplit[5 * NN + idx] = l;
        }
    }
}

template <int WM, int WN, int BMB, int BNB, int FMT>
struct SplitTileG {
    static constexpr int NT = 64 * WM * WN;
    static constexpr int TM = 32 * WM * BMB;
    static constexpr int TN = 32 * WN * BNB;
    static constexpr int GBK = 16;                                    // k values per LDS stage
    static constexpr int FRAG = 64;                                   // 16-byte chunks per fragment (1 KiB)
    static constexpr int XCH = (TM / 32) * 6 * FRAG;                  // chunks per X stage
    static constexpr int YCH = (TN / 32) * 6 * FRAG;
    static constexpr int SMEM_CHUNKS = 3 * (XCH + YCH);

    __device__ __forceinline__ static void run(int n, const uint16_t* __restrict__ X, const uint16_t* __restrict__ Y,
                                               uint16_t* __restrict__ Dsplit, float* __restrict__ Df32, int tm,
                                               int tn, u32x4* smem) {
        constexpr int XV = XCH / NT, YV = YCH / NT;
        static_assert(XV * NT == XCH && YV * NT == YCH, "tile/thread mismatch");
        constexpr bool F16 = (FMT == FMT_F16);

        u32x4* Xs = smem;                // [3][XCH]
        u32x4* Ys = smem + 3 * XCH;      // [3][YCH]

        const int N = 1 << n;
        const size_t NN = (size_t)N * N;
        const int KB = N / GBK;          // k-blocks per row-block
        const int i0 = tm * TM, j0 = tn * TN;
        // 16-byte chunk index of fragment (row-block rb, k-block kb, plane 0)
        auto chunk0 = [&](int rb, int kb) { return ((size_t)rb * KB + kb) * 6 * FRAG; };
        const u32x4* Xc = reinterpret_cast<const u32x4*>(X);
        const u32x4* Yc = reinterpret_cast<const u32x4*>(Y);

        const int tid = threadIdx.x;
        const int lane = tid & 63;
        const int wave = tid >> 6;
        const int wm = wave % WM, wn = wave / WM;
        const int khalf = lane >> 5;
        const int l32 = lane & 31;

        floatx16 acc[BMB][BNB][3];
#pragma unroll
        for (int x = 0; x < BMB; ++x)
#pragma unroll
            for (int y = 0; y < BNB; ++y)
#pragma unroll
                for (int z = 0; z < 3; ++z)
#pragma unroll
                    for (int e = 0; e < 16; ++e) acc[x][y][z][e] = 0.f;

        // A stage is TM / 32 runs of 6 fragments (6 KiB), one per row-block,
        // copied in order: chunk f of the stage is chunk f % 384 of run f / 384.
        // Loads go through buffer resources based at the tile's first row-block
        // (its runs span TM / 32 x N x 384 bytes), so a lane's offsets are fixed
        // for the tile and each k-step only moves the scalar offset.
        constexpr int RUN = 6 * FRAG;
        const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<u32x4*>(Xc + (size_t)(i0 / 32) * KB * RUN), (short)0, (TM / 32) * KB * RUN * 16, 0x00020000);
        const __amdgpu_buffer_rsrc_t yr = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<u32x4*>(Yc + (size_t)(j0 / 32) * KB * RUN), (short)0, (TN / 32) * KB * RUN * 16, 0x00020000);
        int xo[XV], yo[YV];
#pragma unroll
        for (int u = 0; u < XV; ++u) {
            const int f = tid + NT * u;
            xo[u] = ((f / RUN) * KB * RUN + f % RUN) * 16;
        }
#pragma unroll
        for (int u = 0; u < YV; ++u) {
            const int f = tid + NT * u;
            yo[u] = ((f / RUN) * KB * RUN + f % RUN) * 16;
        }
        // part q of 3 of a stage's loads / LDS stores (one part per component phase)
        auto gload = [&](u32x4 (&rx)[XV], u32x4 (&ry)[YV], int kb, int q) {
            const int so = kb * RUN * 16;
#pragma unroll
            for (int u = q * XV / 3; u < (q + 1) * XV / 3; ++u)
                rx[u] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(xr, xo[u], so, 0));
#pragma unroll
            for (int u = q * YV / 3; u < (q + 1) * YV / 3; ++u)
                ry[u] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(yr, yo[u], so, 0));
        };
        auto lstore = [&](const u32x4 (&rx)[XV], const u32x4 (&ry)[YV], int stage, int q) {
            u32x4* xs = Xs + (stage % 3) * XCH;
            u32x4* ys = Ys + (stage % 3) * YCH;
#pragma unroll
            for (int u = q * XV / 3; u < (q + 1) * XV / 3; ++u) xs[tid + NT * u] = rx[u];
#pragma unroll
            for (int u = q * YV / 3; u < (q + 1) * YV / 3; ++u) ys[tid + NT * u] = ry[u];
        };
        // Fragments of component c (planes 2c, 2c + 1) of k-step t.
        struct Frags {
            u32x4 xh[BMB], xl[BMB], yh[BNB], yl[BNB];
        };
        auto fread = [&](Frags& F, int t, int c) {
            const u32x4* xs = Xs + (t % 3) * XCH;
            const u32x4* ys = Ys + (t % 3) * YCH;
#pragma unroll
            for (int x = 0; x < BMB; ++x) {
                const u32x4* fr = xs + ((wm * BMB + x) * 6 + 2 * c) * FRAG + lane;
                F.xh[x] = fr[0];
                F.xl[x] = fr[FRAG];
            }
#pragma unroll
            for (int y = 0; y < BNB; ++y) {
                const u32x4* fr = ys + ((wn * BNB + y) * 6 + 2 * c) * FRAG + lane;
                F.yh[y] = fr[0];
                F.yl[y] = fr[FRAG];
            }
        };
        // The three passes go round the BMB x BNB accumulators in turn, so
        // consecutive MFMAs never feed one another.
        auto fmma = [&](const Frags& F, int c) {
            u32x4 xhh[BMB];
#pragma unroll
            for (int x = 0; x < BMB; ++x) xhh[x] = F16 ? f16x8_times_4096(F.xh[x]) : F.xh[x];
#pragma unroll
            for (int x = 0; x < BMB; ++x)
#pragma unroll
                for (int y = 0; y < BNB; ++y) acc[x][y][c] = mfma16<FMT>(F.yh[y], xhh[x], acc[x][y][c]);
#pragma unroll
            for (int x = 0; x < BMB; ++x)
#pragma unroll
                for (int y = 0; y < BNB; ++y) acc[x][y][c] = mfma16<FMT>(F.yl[y], F.xh[x], acc[x][y][c]);
#pragma unroll
            for (int x = 0; x < BMB; ++x)
#pragma unroll
                for (int y = 0; y < BNB; ++y) acc[x][y][c] = mfma16<FMT>(F.yh[y], F.xl[x], acc[x][y][c]);
        };
        // One component phase: its MFMAs with the next fragments' LDS reads,
        // a third of the next-but-two stage's global loads and a third of the
        // next-but-one stage's LDS stores interleaved between them.
        constexpr int NM = 3 * BMB * BNB, NDR = 2 * (BMB + BNB), NG = (XV + YV) / 3;
        auto interleave = [&]() {
            if constexpr (NDR > NM) __builtin_amdgcn_sched_group_barrier(0x100, NDR - NM, 0);
#pragma unroll
            for (int i = 0; i < NM; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);      // MFMA
                if (i < NDR) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read
                if (i < NG) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // VMEM read
                if (i < NG) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);   // DS write
            }
            __builtin_amdgcn_sched_barrier(0);
        };
        // k-step t: F holds (t, r) on entry; on exit G holds (t + 1, r).
        // R0 holds stage t + 2 (stored to LDS during this step); stage t + 3 is loaded into R1.
        // No branches, so each phase is one scheduling region: past the last
        // stage the loads repeat stage KB - 1 (in range) and the stores and the
        // reads of step KB touch ring slots that hold no live stage any more.
        auto step = [&](int t, Frags& F, Frags& G, u32x4 (&R0x)[XV], u32x4 (&R0y)[YV], u32x4 (&R1x)[XV],
                        u32x4 (&R1y)[YV]) {
            const int ld = t + 3 < KB ? t + 3 : KB - 1;
            fread(G, t, 1);
            gload(R1x, R1y, ld, 0);
            lstore(R0x, R0y, t + 2, 0);
            fmma(F, 0);
            interleave();
            fread(F, t, 2);
            gload(R1x, R1y, ld, 1);
            lstore(R0x, R0y, t + 2, 1);
            fmma(G, 1);
            interleave();
            fread(G, t + 1, 0);
            gload(R1x, R1y, ld, 2);
            lstore(R0x, R0y, t + 2, 2);
            fmma(F, 2);
            interleave();
            __syncthreads();
        };

        u32x4 Ax[XV], Ay[YV], Bx[XV], By[YV];
        Frags F, G;
        for (int q = 0; q < 3; ++q) gload(Ax, Ay, 0, q);
        for (int q = 0; q < 3; ++q) lstore(Ax, Ay, 0, q);
        for (int q = 0; q < 3; ++q) gload(Bx, By, 1, q);
        for (int q = 0; q < 3; ++q) lstore(Bx, By, 1, q);
        for (int q = 0; q < 3; ++q) gload(Ax, Ay, 2, q);  // stored during k-step 0
        __syncthreads();
        fread(F, 0, 0);
        for (int t = 0; t < KB; t += 2) {  // KB = N / 16 is even (n >= 6)
            step(t, F, G, Ax, Ay, Bx, By);
            step(t + 1, G, F, Bx, By, Ax, Ay);
        }

        // Lane l of block (x, y) holds row i = l % 32 and columns 8 g + 4 (l / 32) + q in register 4 g + q.
        // In the fragment-blocked output, columns 8 g .. 8 g + 7 of a row are fragment lane l % 32 + 32 (g % 2)
        // of k-block (block column) / 16 + g / 2, so each (g, plane) store covers 512 contiguous bytes.
        const float scale = F16 ? 1.0f / (float)(1 << QSIM_LO_SCALE_LOG2) : 1.0f;
#pragma unroll
        for (int x = 0; x < BMB; ++x) {
            const int rbase = i0 + wm * (32 * BMB) + x * 32;
            const int row = rbase + l32;
#pragma unroll
            for (int y = 0; y < BNB; ++y) {
                const int cbase = j0 + wn * (32 * BNB) + y * 32;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    float re[4], im[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float t1 = acc[x][y][0][4 * g + q], t2 = acc[x][y][1][4 * g + q];
                        const float t3 = acc[x][y][2][4 * g + q];
                        re[q] = (t1 - t2) * scale;
                        im[q] = ((t3 - t1) - t2) * scale;
                    }
                    if (Df32) {
                        const size_t o = (size_t)row * N + cbase + 8 * g + 4 * khalf;
                        *reinterpret_cast<float4*>(Df32 + o) = make_float4(re[0], re[1], re[2], re[3]);
                        *reinterpret_cast<float4*>(Df32 + NN + o) = make_float4(im[0], im[1], im[2], im[3]);
                    }
                    if (Dsplit) {
                        const size_t o = chunk0(rbase / 32, cbase / 16 + g / 2) * 8 +
                                         (size_t)(l32 + 32 * (g & 1)) * 8 + 4 * khalf;
                        store_split6<FMT>(Dsplit, FRAG * 8, o, re, im);
                    }
                }
            }
        }
    }
};

}  // namespace qsim
