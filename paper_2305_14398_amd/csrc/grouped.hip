// Grouped launches for many circuits of mixed size: one launch expands the
// current step of every circuit of a batch (stage 4, Section 5.3) and one
// launch takes the current chain product of every circuit (stage 5,
// Algorithm 1).  Work items come from a device job table; a persistent grid
// walks the concatenated tile (or block) ranges, each workgroup finding its job
// by a binary search over the range starts.  Every job has its own size and
// tile configuration (64 x 64 or 128 x 128 MFMA tiles, or one workgroup for
// the whole product when n <= 5), so small and large circuits share a launch.
#include "expand_entry.h"
#include "tile_f32.h"
#include "tile_split.h"
#include "tile_split_gauss.h"

namespace qsim {
namespace {

// Tile visited by workgroup `bid` in round `r` of a persistent grid of `grid`
// workgroups (a multiple of 8): blocks are dispatched round-robin over the 8
// XCDs, so within each round the XCD of block b takes a contiguous slice of the
// round's tile ids, which keeps its tiles' A and B panels together in its L2.
__device__ __forceinline__ int persistent_tile(int r, int bid, int grid) {
    if (grid & 7) return r * grid + bid;
    return r * grid + (bid & 7) * (grid >> 3) + (bid >> 3);
}

template <class Job>
__device__ __forceinline__ int find_job(const Job* __restrict__ jobs, int njobs, int t, int Job::*begin) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].*begin <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void grouped_expand_kernel(const ExpandJob* __restrict__ jobs, int njobs,
                                                             int total_blocks) {
    for (int b = blockIdx.x; b < total_blocks; b += gridDim.x) {
        const int j = find_job(jobs, njobs, b, &ExpandJob::block_begin);
        const ExpandJob& J = jobs[j];
        const uint64_t items = (1ull << (2 * J.n)) >> 2;
        const uint64_t stride = (uint64_t)J.blocks * 256u;
        for (uint64_t it = (uint64_t)(b - J.block_begin) * 256u + threadIdx.x; it < items; it += stride) {
            if (J.fmt == FMT_F32)
                expand_four<FMT_F32>(J.st, J.n, J.layout_col, J.out, it << 2);
            else if (J.fmt == FMT_BF16)
                expand_four<FMT_BF16>(J.st, J.n, J.layout_col, J.out, it << 2);
            else if (J.fmt == FMT_F16)
                expand_four<FMT_F16>(J.st, J.n, J.layout_col, J.out, it << 2);
            else if (J.fmt == FMT_BF16_G)
                expand_four<FMT_BF16_G>(J.st, J.n, J.layout_col, J.out, it << 2);
            else
                expand_four<FMT_F16_G>(J.st, J.n, J.layout_col, J.out, it << 2);
        }
    }
}

template <bool GAUSS>
__global__ __launch_bounds__(F32Shapes<GAUSS>::THREADS) void grouped_f32_kernel(const GemmJob* __restrict__ jobs,
                                                                               int njobs, int total_tiles) {
    using T128 = typename F32Shapes<GAUSS>::T128;
    using T64 = typename F32Shapes<GAUSS>::T64;
    __shared__ __attribute__((aligned(16))) float smem[F32Shapes<GAUSS>::SMEM_FLOATS];
    const int rounds = (total_tiles + gridDim.x - 1) / gridDim.x;
    for (int r = 0; r < rounds; ++r) {
        const int t = persistent_tile(r, blockIdx.x, gridDim.x);
        if (t >= total_tiles) continue;
        const int j = find_job(jobs, njobs, t, &GemmJob::tile_begin);
        const GemmJob& J = jobs[j];
        const int local = t - J.tile_begin;
        const int N = 1 << J.n;
        const float* A = static_cast<const float*>(J.X);
        const float* B = static_cast<const float*>(J.Y);
        float* C = static_cast<float*>(J.D0);
        int tm, tn;
        if (J.cfg == 128) {
            grouped_tile_order(local, N / 128, N / 128, tm, tn);
            T128::template run<false>(J.n, A, B, C, tm, tn, smem);
        } else if (J.cfg == 64) {
            grouped_tile_order(local, N / 64, N / 64, tm, tn);
            T64::template run<false>(J.n, A, B, C, tm, tn, smem);
        } else {
            f32_small_product<GAUSS>(J.n, A, nullptr, B, C, threadIdx.x, F32Shapes<GAUSS>::THREADS);
        }
    }
}

template <int FMT>
__global__ __launch_bounds__(256) void grouped_split_kernel(const GemmJob* __restrict__ jobs, int njobs,
                                                            int total_tiles) {
    // The fp16 128 x 128 tile needs all 512 registers on its own; inside the
    // grouped loop it would spill, so fp16 jobs always run 64 x 64 tiles.
    constexpr bool BIG = (FMT == FMT_BF16);
    using T128 = SplitTile<2, 2, 2, 2, FMT>;
    using T64 = SplitTile<2, 2, 1, 1, FMT>;
    __shared__ u32x4 smem[BIG ? T128::SMEM_CHUNKS : T64::SMEM_CHUNKS];
    const int rounds = (total_tiles + gridDim.x - 1) / gridDim.x;
    for (int r = 0; r < rounds; ++r) {
        const int t = persistent_tile(r, blockIdx.x, gridDim.x);
        if (t >= total_tiles) continue;
        const int j = find_job(jobs, njobs, t, &GemmJob::tile_begin);
        const GemmJob& J = jobs[j];
        const int local = t - J.tile_begin;
        const int N = 1 << J.n;
        const uint16_t* X = static_cast<const uint16_t*>(J.X);
        const uint16_t* Y = static_cast<const uint16_t*>(J.Y);
        uint16_t* Ds = static_cast<uint16_t*>(J.D0);
        float* Df = static_cast<float*>(J.D1);
        int tm, tn;
        if (BIG && J.cfg == 128) {
            grouped_tile_order(local, N / 128, N / 128, tm, tn);
            T128::run(J.n, X, Y, Ds, Df, tm, tn, smem);
        } else if (J.cfg != 0) {
            grouped_tile_order(local, N / 64, N / 64, tm, tn);
            T64::run(J.n, X, Y, Ds, Df, tm, tn, smem);
        } else {
            split_small_product<FMT>(J.n, X, Y, Ds, Df, threadIdx.x, 256);
        }
    }
}

// Three-product split jobs: 128 x 128 tiles (one wave per SIMD, 96 KiB LDS),
// 64 x 64 tiles, or the whole product by one workgroup.
template <int FMT>
__global__ __launch_bounds__(256) void grouped_split_gauss_kernel(const GemmJob* __restrict__ jobs, int njobs,
                                                                  int total_tiles) {
    using T128 = SplitTileG<2, 2, 2, 2, FMT>;
    using T64 = SplitTileG<2, 2, 1, 1, FMT>;
    __shared__ u32x4 smem[T128::SMEM_CHUNKS];
    const int rounds = (total_tiles + gridDim.x - 1) / gridDim.x;
    for (int r = 0; r < rounds; ++r) {
        const int t = persistent_tile(r, blockIdx.x, gridDim.x);
        if (t >= total_tiles) continue;
        const int j = find_job(jobs, njobs, t, &GemmJob::tile_begin);
        const GemmJob& J = jobs[j];
        const int local = t - J.tile_begin;
        const int N = 1 << J.n;
        const uint16_t* X = static_cast<const uint16_t*>(J.X);
        const uint16_t* Y = static_cast<const uint16_t*>(J.Y);
        uint16_t* Ds = static_cast<uint16_t*>(J.D0);
        float* Df = static_cast<float*>(J.D1);
        int tm, tn;
        if (J.cfg == 128) {
            grouped_tile_order(local, N / 128, N / 128, tm, tn);
            T128::run(J.n, X, Y, Ds, Df, tm, tn, smem);
        } else if (J.cfg != 0) {
            grouped_tile_order(local, N / 64, N / 64, tm, tn);
            T64::run(J.n, X, Y, Ds, Df, tm, tn, smem);
        } else {
            split_small_product_gauss<FMT>(J.n, X, Y, Ds, Df, threadIdx.x, 256);
        }
    }
}

}  // namespace

hipError_t launch_grouped_expand(const ExpandJob* jobs, int njobs, int total_blocks, int grid, hipStream_t stream) {
    if (njobs <= 0 || total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(grouped_expand_kernel, dim3(grid), dim3(256), 0, stream, jobs, njobs, total_blocks);
    return hipGetLastError();
}

hipError_t launch_grouped_gemm(int prec, const GemmJob* jobs, int njobs, int total_tiles, int grid,
                               hipStream_t stream) {
    if (njobs <= 0 || total_tiles <= 0) return hipSuccess;
    switch (prec) {
        case QSIM_FP32_4M:
            hipLaunchKernelGGL(grouped_f32_kernel<false>, dim3(grid), dim3(F32Shapes<false>::THREADS), 0, stream, jobs,
                               njobs, total_tiles);
            break;
        case QSIM_FP32_3M:
            hipLaunchKernelGGL(grouped_f32_kernel<true>, dim3(grid), dim3(F32Shapes<true>::THREADS), 0, stream, jobs,
                               njobs, total_tiles);
            break;
        case QSIM_SPLIT_BF16:
            hipLaunchKernelGGL(grouped_split_kernel<FMT_BF16>, dim3(grid), dim3(256), 0, stream, jobs, njobs,
                               total_tiles);
            break;
        case QSIM_SPLIT_FP16:
            hipLaunchKernelGGL(grouped_split_kernel<FMT_F16>, dim3(grid), dim3(256), 0, stream, jobs, njobs,
                               total_tiles);
            break;
        case QSIM_SPLIT_BF16_3M:
            hipLaunchKernelGGL(grouped_split_gauss_kernel<FMT_BF16>, dim3(grid), dim3(256), 0, stream, jobs, njobs,
                               total_tiles);
            break;
        default:
            hipLaunchKernelGGL(grouped_split_gauss_kernel<FMT_F16>, dim3(grid), dim3(256), 0, stream, jobs, njobs,
                               total_tiles);
            break;
    }
    return hipGetLastError();
}

}  // namespace qsim
