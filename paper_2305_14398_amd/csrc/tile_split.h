// One output tile of the stage-5 product (Section 5.3; Algorithm 1) with split
// 16-bit operands on bf16/fp16 MFMA and float32 accumulation, shared by the
// single-problem kernel (cgemm_split.hip) and the grouped kernel (grouped.hip).
//
// Each float value x is carried as hi + lo * s (hi = round(x), lo = round((x -
// hi) / s); s = 1 for bf16, 2^-12 for fp16 so that lo stays clear of fp16
// subnormals).  A real product is taken in three passes,
//   x * y ~= hi_x hi_y + (hi_x lo_y + lo_x hi_y) * s      (lo_x lo_y dropped),
// and a complex product in four real products (4M), so one complex product
// issues 12 MFMAs per k-block; fp16 keeps the s-scaled cross terms in their own
// accumulators and combines them in the epilogue.
//
// v_mfma_f32_32x32x16_{bf16,f16} wants 8 consecutive k values per lane for both
// operands, so both are stored k-contiguous and the kernel computes
//     D[i][j] = sum_k X[i][k] Y[j][k]      (D = X Y^T, complex, no conjugation)
// with X and Y read as row-major buffers.  Inside a chain the running product U
// is kept COLUMN-major and the step operator S ROW-major:
//   * X = U buffer, Y = S buffer gives D = U^T S^T = (S U)^T, written row-major,
//     i.e. the next product in column-major split form;
//   * X = S buffer, Y = U buffer gives D = S U itself, row-major (the last
//     product, written as float32).
// Operand planes: re_hi, re_lo, im_hi, im_lo (N*N 16-bit each).
//
// Tiling: 256 threads, 2 x 2 waves, each wave 2 x 2 blocks of 32 x 32 (a
// 128 x 128 tile of D), K-tiles of 32 double buffered in LDS; the tile ends
// with a barrier so a persistent workgroup can reuse the LDS for its next tile.  LDS rows are 64
// bytes (32 values) with the four 16-byte chunks of row r stored at chunk index
// c ^ ((r / 4) % 4), which puts any 16 consecutive rows' reads of one chunk on
// 64 distinct banks without padding (4 planes x 2 operands x 128 rows x 64 B
// x 2 stages = 128 KiB of the 160 KiB LDS).
#pragma once

#include "common.h"

namespace qsim {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int SBK = 32;  // k values per LDS tile (two MFMA k-steps of 16)

template <int FMT>
__device__ __forceinline__ floatx16 mfma16(u32x4 a, u32x4 b, floatx16 c) {
    if constexpr (FMT == FMT_BF16)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                       0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(halfx8, a), __builtin_bit_cast(halfx8, b), c,
                                                      0, 0, 0);
}

// float -> (hi, lo) in the operand format; lo is pre-scaled for fp16.
template <int FMT>
__device__ __forceinline__ void split_f32(float x, uint16_t& hi, uint16_t& lo) {
    if constexpr (FMT == FMT_BF16) {
        hi = bf16_rne(x);
        lo = bf16_rne(x - __uint_as_float(((uint32_t)hi) << 16));  // x - hi is exact in float32
    } else {
        const _Float16 h = (_Float16)x;
        const _Float16 l = (_Float16)((x - (float)h) * (float)(1 << QSIM_LO_SCALE_LOG2));
        hi = __builtin_bit_cast(uint16_t, h);
        lo = __builtin_bit_cast(uint16_t, l);
    }
}

template <int WM, int WN, int BMB, int BNB, int FMT>
struct SplitTile {
    static constexpr int NT = 64 * WM * WN;
    static constexpr int TM = 32 * WM * BMB;
    static constexpr int TN = 32 * WN * BNB;
    static constexpr int SMEM_CHUNKS = 2 * 4 * (TM + TN) * 4;  // 16-byte chunks

    __device__ __forceinline__ static void run(int n, const uint16_t* __restrict__ X, const uint16_t* __restrict__ Y,
                               uint16_t* __restrict__ Dsplit, float* __restrict__ Df32, int tm, int tn,
                               u32x4* smem) {
        constexpr int XCH = 4 * TM * 4;  // 16-byte chunks per X stage (4 planes, TM rows, 4 chunks)
        constexpr int YCH = 4 * TN * 4;
        constexpr int XV = XCH / NT, YV = YCH / NT;
        static_assert(XV * NT == XCH && YV * NT == YCH, "tile/thread mismatch");
        constexpr bool F16 = (FMT == FMT_F16);
        constexpr int NACC = F16 ? 4 : 2;  // re, im (+ re_cross, im_cross for fp16)

        auto Xs = reinterpret_cast<u32x4(*)[4][TM][4]>(smem);
        auto Ys = reinterpret_cast<u32x4(*)[4][TN][4]>(smem + 2 * 4 * TM * 4);

        const int N = 1 << n;
        const size_t NN = (size_t)N * N;
        const int i0 = tm * TM, j0 = tn * TN;

        const int tid = threadIdx.x;
        const int lane = tid & 63;
        const int wave = tid >> 6;
        const int wm = wave % WM, wn = wave / WM;
        const int l32 = lane & 31;
        const int khalf = lane >> 5;

        floatx16 acc[BMB][BNB][NACC];
#pragma unroll
        for (int x = 0; x < BMB; ++x)
#pragma unroll
            for (int y = 0; y < BNB; ++y)
#pragma unroll
                for (int z = 0; z < NACC; ++z)
#pragma unroll
                    for (int e = 0; e < 16; ++e) acc[x][y][z][e] = 0.f;

        u32x4 rx[XV], ry[YV];
#define QSIM_SLOAD(k0)                                                                                       \
        _Pragma("unroll") for (int u = 0; u < XV; ++u) {                                                         \
            const int f = tid + NT * u;                                                                          \
            const int p = f / (TM * 4), row = (f % (TM * 4)) >> 2, ch = f & 3;                                   \
            rx[u] = *reinterpret_cast<const u32x4*>(X + p * NN + (size_t)(i0 + row) * N + (k0) + ch * 8);        \
        }                                                                                                        \
        _Pragma("unroll") for (int u = 0; u < YV; ++u) {                                                         \
            const int f = tid + NT * u;                                                                          \
            const int p = f / (TN * 4), row = (f % (TN * 4)) >> 2, ch = f & 3;                                   \
            ry[u] = *reinterpret_cast<const u32x4*>(Y + p * NN + (size_t)(j0 + row) * N + (k0) + ch * 8);        \
        }
#define QSIM_SSTORE(s)                                                                                       \
        _Pragma("unroll") for (int u = 0; u < XV; ++u) {                                                         \
            const int f = tid + NT * u;                                                                          \
            const int p = f / (TM * 4), row = (f % (TM * 4)) >> 2, ch = f & 3;                                   \
            Xs[s][p][row][ch ^ ((row >> 2) & 3)] = rx[u];                                                        \
        }                                                                                                        \
        _Pragma("unroll") for (int u = 0; u < YV; ++u) {                                                         \
            const int f = tid + NT * u;                                                                          \
            const int p = f / (TN * 4), row = (f % (TN * 4)) >> 2, ch = f & 3;                                   \
            Ys[s][p][row][ch ^ ((row >> 2) & 3)] = ry[u];                                                        \
        }

        const int KT = N / SBK;
        QSIM_SLOAD(0);
        QSIM_SSTORE(0);
        __syncthreads();

        const u32x4 signbits = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
        for (int kt = 0; kt < KT; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < KT) { QSIM_SLOAD((kt + 1) * SBK); }
#pragma unroll
            for (int t = 0; t < SBK / 16; ++t) {
                const int c = 2 * t + khalf;
                u32x4 xa[BMB][4], xn[BMB][2], yb[BNB][4];
#pragma unroll
                for (int x = 0; x < BMB; ++x) {
                    const int row = wm * (32 * BMB) + x * 32 + l32;
#pragma unroll
                    for (int p = 0; p < 4; ++p) xa[x][p] = Xs[cur][p][row][c ^ ((row >> 2) & 3)];
                    xn[x][0] = xa[x][2] ^ signbits;  // -Xi_hi
                    xn[x][1] = xa[x][3] ^ signbits;  // -Xi_lo
                }
#pragma unroll
                for (int y = 0; y < BNB; ++y) {
                    const int row = wn * (32 * BNB) + y * 32 + l32;
#pragma unroll
                    for (int p = 0; p < 4; ++p) yb[y][p] = Ys[cur][p][row][c ^ ((row >> 2) & 3)];
                }
#pragma unroll
                for (int x = 0; x < BMB; ++x) {
#pragma unroll
                    for (int y = 0; y < BNB; ++y) {
                        // planes: 0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo
                        constexpr int RC = F16 ? 2 : 0;  // accumulator of the re cross terms
                        constexpr int IC = F16 ? 3 : 1;  // accumulator of the im cross terms
                        floatx16* a = acc[x][y];
                        a[0] = mfma16<FMT>(xa[x][0], yb[y][0], a[0]);   // Xr_h Yr_h
                        a[RC] = mfma16<FMT>(xa[x][0], yb[y][1], a[RC]);  // Xr_h Yr_l
                        a[RC] = mfma16<FMT>(xa[x][1], yb[y][0], a[RC]);  // Xr_l Yr_h
                        a[0] = mfma16<FMT>(xn[x][0], yb[y][2], a[0]);   // -Xi_h Yi_h
                        a[RC] = mfma16<FMT>(xn[x][0], yb[y][3], a[RC]);  // -Xi_h Yi_l
                        a[RC] = mfma16<FMT>(xn[x][1], yb[y][2], a[RC]);  // -Xi_l Yi_h
                        a[1] = mfma16<FMT>(xa[x][0], yb[y][2], a[1]);   // Xr_h Yi_h
                        a[IC] = mfma16<FMT>(xa[x][0], yb[y][3], a[IC]);  // Xr_h Yi_l
                        a[IC] = mfma16<FMT>(xa[x][1], yb[y][2], a[IC]);  // Xr_l Yi_h
                        a[1] = mfma16<FMT>(xa[x][2], yb[y][0], a[1]);   // Xi_h Yr_h
                        a[IC] = mfma16<FMT>(xa[x][2], yb[y][1], a[IC]);  // Xi_h Yr_l
                        a[IC] = mfma16<FMT>(xa[x][3], yb[y][0], a[IC]);  // Xi_l Yr_h
                    }
                }
            }
            if (kt + 1 < KT) { QSIM_SSTORE(cur ^ 1); }
            __syncthreads();
        }
#undef QSIM_SLOAD
#undef QSIM_SSTORE

        // Accumulator layout of a 32x32 block: register e of lane l is row
        // 8*(e/4) + 4*(l/32) + e%4, column l%32.
        const float cross_scale = F16 ? 1.0f / (float)(1 << QSIM_LO_SCALE_LOG2) : 1.0f;
#pragma unroll
        for (int x = 0; x < BMB; ++x) {
#pragma unroll
            for (int y = 0; y < BNB; ++y) {
                const int col = j0 + wn * (32 * BNB) + y * 32 + l32;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int row = i0 + wm * (32 * BMB) + x * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                    float re = acc[x][y][0][e], im = acc[x][y][1][e];
                    if constexpr (F16) {
                        re = fmaf(acc[x][y][2][e], cross_scale, re);
                        im = fmaf(acc[x][y][3][e], cross_scale, im);
                    }
                    const size_t o = (size_t)row * N + col;
                    if (Df32) {
                        Df32[o] = re;
                        Df32[NN + o] = im;
                    }
                    if (Dsplit) {
                        uint16_t h, l;
                        split_f32<FMT>(re, h, l);
                        Dsplit[o] = h;
                        Dsplit[NN + o] = l;
                        split_f32<FMT>(im, h, l);
                        Dsplit[2 * NN + o] = h;
                        Dsplit[3 * NN + o] = l;
                    }
                }
            }
        }
    }
};

// N < 32: one thread per output entry, the same three-pass arithmetic in float32.
template <int FMT>
__device__ __forceinline__ float to_f32(uint16_t v) {
    if constexpr (FMT == FMT_BF16)
        return __uint_as_float(((uint32_t)v) << 16);
    else
        return (float)__builtin_bit_cast(_Float16, v);
}

template <int FMT>
__device__ __forceinline__ void split_small_product(int n, const uint16_t* __restrict__ X,
                                                    const uint16_t* __restrict__ Y, uint16_t* __restrict__ Dsplit,
                                                    float* __restrict__ Df32, int first, int stride) {
    const int N = 1 << n;
    const int NN = N * N;
    for (int idx = first; idx < NN; idx += stride) {
        const int i = idx / N, j = idx % N;
        float rm = 0.f, rc = 0.f, im = 0.f, ic = 0.f;
        for (int k = 0; k < N; ++k) {
            const float xrh = to_f32<FMT>(X[i * N + k]), xrl = to_f32<FMT>(X[NN + i * N + k]);
            const float xih = to_f32<FMT>(X[2 * NN + i * N + k]), xil = to_f32<FMT>(X[3 * NN + i * N + k]);
            const float yrh = to_f32<FMT>(Y[j * N + k]), yrl = to_f32<FMT>(Y[NN + j * N + k]);
            const float yih = to_f32<FMT>(Y[2 * NN + j * N + k]), yil = to_f32<FMT>(Y[3 * NN + j * N + k]);
            rm = fmaf(xrh, yrh, rm);
            rm = fmaf(-xih, yih, rm);
            rc = fmaf(xrh, yrl, fmaf(xrl, yrh, rc));
            rc = fmaf(-xih, yil, fmaf(-xil, yih, rc));
            im = fmaf(xrh, yih, im);
            im = fmaf(xih, yrh, im);
            ic = fmaf(xrh, yil, fmaf(xrl, yih, ic));
            ic = fmaf(xih, yrl, fmaf(xil, yrh, ic));
        }
        const float s = (FMT == FMT_F16) ? 1.0f / (float)(1 << QSIM_LO_SCALE_LOG2) : 1.0f;
        const float re = fmaf(rc, s, rm), imv = fmaf(ic, s, im);
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
        }
    }
}

}  // namespace qsim
