// Single-problem float32 complex product of stage 5 (Section 5.3; Algorithm 1;
// the paper's matrixMultiplication listing of Section 5.5 computes the same
// planar-complex product with one thread per output entry and a serial k
// loop).  The tile body, operand layouts and MFMA mapping are in tile_f32.h.
#include "tile_f32.h"

namespace qsim {
namespace {

template <class Tile>
__global__ __launch_bounds__(Tile::NT) void cgemm_f32_kernel(int n, const float* __restrict__ A,
                                                             const float* __restrict__ B, float* __restrict__ C) {
    __shared__ __attribute__((aligned(16))) float smem[Tile::SMEM_FLOATS];
    const int N = 1 << n;
    int tm, tn;
    grouped_tile_order(xcd_contiguous_id(blockIdx.x, gridDim.x), N / Tile::TM, N / Tile::TN, tm, tn);
    Tile::run(n, A, B, C, tm, tn, smem);
}

template <bool GAUSS>
__global__ void cgemm_f32_small(int n, const float* __restrict__ A, const float* __restrict__ B,
                                float* __restrict__ C) {
    f32_small_product<GAUSS>(n, A, nullptr, B, C, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// Fused stages 4 and 5: C = S . B with S computed from the step's gates inside
// the product.  The descriptor travels as a kernel argument.
template <class Tile>
__global__ __launch_bounds__(Tile::NT) void cgemm_f32_fused_kernel(int n, DevStep st, const float* __restrict__ B,
                                                                   float* __restrict__ C) {
    __shared__ __attribute__((aligned(16))) float smem[Tile::SMEM_FLOATS];
    const int N = 1 << n;
    int tm, tn;
    grouped_tile_order(xcd_contiguous_id(blockIdx.x, gridDim.x), N / Tile::TM, N / Tile::TN, tm, tn);
    Tile::run_fused(n, st, B, C, tm, tn, smem);
}

template <bool GAUSS>
__global__ void cgemm_f32_fused_small(int n, DevStep st, const float* __restrict__ B, float* __restrict__ C) {
    f32_small_product<GAUSS>(n, nullptr, &st, B, C, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

template <class Tile>
hipError_t launch_tiled(int n, const float* A, const float* B, float* C, hipStream_t stream) {
    const int N = 1 << n;
    const int tiles = (N / Tile::TM) * (N / Tile::TN);
    hipLaunchKernelGGL(cgemm_f32_kernel<Tile>, dim3(tiles), dim3(Tile::NT), 0, stream, n, A, B, C);
    return hipGetLastError();
}

template <bool GAUSS>
hipError_t launch_f32(int n, int tile, const float* A, const float* B, float* C, hipStream_t stream) {
    if (n >= 7 && tile == 128) return launch_tiled<typename F32Shapes<GAUSS>::T128>(n, A, B, C, stream);
    if (n >= 6) return launch_tiled<typename F32Shapes<GAUSS>::T64>(n, A, B, C, stream);
    if (n == 5) return launch_tiled<F32Tile<1, 1, 1, 1, GAUSS>>(n, A, B, C, stream);
    const int NN = 1 << (2 * n);
    hipLaunchKernelGGL(cgemm_f32_small<GAUSS>, dim3((NN + 255) / 256), dim3(256), 0, stream, n, A, B, C);
    return hipGetLastError();
}

template <class Tile>
hipError_t launch_fused_tiled(int n, const DevStep& st, const float* B, float* C, hipStream_t stream) {
    const int N = 1 << n;
    const int tiles = (N / Tile::TM) * (N / Tile::TN);
    hipLaunchKernelGGL(cgemm_f32_fused_kernel<Tile>, dim3(tiles), dim3(Tile::NT), 0, stream, n, st, B, C);
    return hipGetLastError();
}

template <bool GAUSS>
hipError_t launch_fused(int n, int tile, const DevStep& st, const float* B, float* C, hipStream_t stream) {
    if (n >= 7 && tile == 128) return launch_fused_tiled<typename F32Shapes<GAUSS>::T128>(n, st, B, C, stream);
    if (n >= 6) return launch_fused_tiled<typename F32Shapes<GAUSS>::T64>(n, st, B, C, stream);
    if (n == 5) return launch_fused_tiled<F32Tile<1, 1, 1, 1, GAUSS>>(n, st, B, C, stream);
    const int NN = 1 << (2 * n);
    hipLaunchKernelGGL(cgemm_f32_fused_small<GAUSS>, dim3((NN + 255) / 256), dim3(256), 0, stream, n, st, B, C);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cgemm_f32_fused(int n, bool gauss, int tile, const DevStep& st, const float* U_row, float* C_row,
                                  hipStream_t stream) {
    return gauss ? launch_fused<true>(n, tile, st, U_row, C_row, stream)
                 : launch_fused<false>(n, tile, st, U_row, C_row, stream);
}

hipError_t launch_cgemm_f32(int n, bool gauss, int tile, const float* S_col, const float* U_row, float* C_row,
                            hipStream_t stream) {
    return gauss ? launch_f32<true>(n, tile, S_col, U_row, C_row, stream)
                 : launch_f32<false>(n, tile, S_col, U_row, C_row, stream);
}

}  // namespace qsim
