// Single-problem split-operand product of stage 5 (Section 5.3; Algorithm 1).
// The tile bodies, the split arithmetic and the operand layouts are in
// tile_split.h (four real products) and tile_split_gauss.h (three): the kernels
// compute D[i][j] = sum_k X[i][k] Y[j][k].
#include "tile_f32.h"
#include "tile_split.h"
#include "tile_split_gauss.h"

namespace qsim {
namespace {

template <int WM, int WN, int BMB, int BNB, int FMT>
__global__ __launch_bounds__(64 * WM * WN) void cgemm_split_kernel(int n, const uint16_t* __restrict__ X,
                                                                     const uint16_t* __restrict__ Y,
                                                                     uint16_t* __restrict__ Dsplit,
                                                                     float* __restrict__ Df32) {
    using Tile = SplitTile<WM, WN, BMB, BNB, FMT>;
    __shared__ u32x4 smem[Tile::SMEM_CHUNKS];
    const int N = 1 << n;
    int tm, tn;
    grouped_tile_order(xcd_contiguous_id(blockIdx.x, gridDim.x), N / Tile::TM, N / Tile::TN, tm, tn);
    Tile::run(n, X, Y, Dsplit, Df32, tm, tn, smem);
}

template <int FMT>
__global__ void cgemm_split_small(int n, const uint16_t* __restrict__ X, const uint16_t* __restrict__ Y,
                                  uint16_t* __restrict__ Dsplit, float* __restrict__ Df32) {
    split_small_product<FMT>(n, X, Y, Dsplit, Df32, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

template <int WM, int WN, int BMB, int BNB, int FMT>
hipError_t launch_tiled(int n, const uint16_t* X, const uint16_t* Y, uint16_t* Ds, float* Df, hipStream_t stream) {
    const int N = 1 << n;
    const int tiles = (N / (32 * WM * BMB)) * (N / (32 * WN * BNB));
    hipLaunchKernelGGL((cgemm_split_kernel<WM, WN, BMB, BNB, FMT>), dim3(tiles), dim3(64 * WM * WN), 0, stream, n, X, Y,
                       Ds, Df);
    return hipGetLastError();
}

template <int FMT>
hipError_t launch_fmt(int n, int tile, const uint16_t* X, const uint16_t* Y, uint16_t* Ds, float* Df,
                      hipStream_t stream) {
    if (n >= 7 && tile == 128) return launch_tiled<2, 2, 2, 2, FMT>(n, X, Y, Ds, Df, stream);
    if (n >= 6) return launch_tiled<2, 2, 1, 1, FMT>(n, X, Y, Ds, Df, stream);
    if (n == 5) return launch_tiled<1, 1, 1, 1, FMT>(n, X, Y, Ds, Df, stream);
    const int NN = 1 << (2 * n);
    hipLaunchKernelGGL(cgemm_split_small<FMT>, dim3((NN + 255) / 256), dim3(256), 0, stream, n, X, Y, Ds, Df);
    return hipGetLastError();
}

template <int WM, int WN, int BMB, int BNB, int FMT>
__global__ __launch_bounds__(64 * WM * WN) void cgemm_split_gauss_kernel(int n, const uint16_t* __restrict__ X,
                                                                           const uint16_t* __restrict__ Y,
                                                                           uint16_t* __restrict__ Dsplit,
                                                                           float* __restrict__ Df32) {
    using Tile = SplitTileG<WM, WN, BMB, BNB, FMT>;
    __shared__ u32x4 smem[Tile::SMEM_CHUNKS];
    const int N = 1 << n;
    int tm, tn;
    grouped_tile_order(xcd_contiguous_id(blockIdx.x, gridDim.x), N / Tile::TM, N / Tile::TN, tm, tn);
    Tile::run(n, X, Y, Dsplit, Df32, tm, tn, smem);
}

template <int FMT>
__global__ void cgemm_split_gauss_small(int n, const uint16_t* __restrict__ X, const uint16_t* __restrict__ Y,
                                        uint16_t* __restrict__ Dsplit, float* __restrict__ Df32) {
    split_small_product_gauss<FMT>(n, X, Y, Dsplit, Df32, blockIdx.x * blockDim.x + threadIdx.x,
                                   gridDim.x * blockDim.x);
}

template <int WM, int WN, int BMB, int BNB, int FMT>
hipError_t launch_gauss_tiled(int n, const uint16_t* X, const uint16_t* Y, uint16_t* Ds, float* Df,
                              hipStream_t stream) {
    const int N = 1 << n;
    const int tiles = (N / (32 * WM * BMB)) * (N / (32 * WN * BNB));
    hipLaunchKernelGGL((cgemm_split_gauss_kernel<WM, WN, BMB, BNB, FMT>), dim3(tiles), dim3(64 * WM * WN), 0, stream,
                       n, X, Y, Ds, Df);
    return hipGetLastError();
}

template <int FMT>
hipError_t launch_gauss(int n, int tile, const uint16_t* X, const uint16_t* Y, uint16_t* Ds, float* Df,
                        hipStream_t stream) {
    if (n >= 7 && tile == 128) return launch_gauss_tiled<2, 2, 2, 2, FMT>(n, X, Y, Ds, Df, stream);
    if (n >= 6) return launch_gauss_tiled<2, 2, 1, 1, FMT>(n, X, Y, Ds, Df, stream);
    // n <= 5: planar operands, one thread per output entry (as in grouped launches)
    const int NN = 1 << (2 * n);
    hipLaunchKernelGGL(cgemm_split_gauss_small<FMT>, dim3((NN + 255) / 256), dim3(256), 0, stream, n, X, Y, Ds, Df);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cgemm_split(int n, OpFormat fmt, int tile, const void* X, const void* Y, void* D_split,
                              float* D_f32, hipStream_t stream) {
    const uint16_t* x = static_cast<const uint16_t*>(X);
    const uint16_t* y = static_cast<const uint16_t*>(Y);
    uint16_t* ds = static_cast<uint16_t*>(D_split);
    switch (fmt) {
        case FMT_BF16: return launch_fmt<FMT_BF16>(n, tile, x, y, ds, D_f32, stream);
        case FMT_F16: return launch_fmt<FMT_F16>(n, tile, x, y, ds, D_f32, stream);
        case FMT_BF16_G: return launch_gauss<FMT_BF16>(n, tile, x, y, ds, D_f32, stream);
        case FMT_F16_G: return launch_gauss<FMT_F16>(n, tile, x, y, ds, D_f32, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace qsim
