// Stage 4 of the unitary method (Section 5.3; Algorithm 2; Eq. 9s1): write the
// dense 2^n x 2^n operator of one circuit step.  The per-entry rule is in
// expand_entry.h; the kernel is a pure streaming writer (8 bytes of HBM
// traffic per entry, no reads).
#include "expand_entry.h"

namespace qsim {
namespace {

// Each work item writes 4 consecutive storage entries (one row holds fewer
// than 4 only when N = 2); the grid strides over all N*N/4 items.
template <int FMT>
__global__ __launch_bounds__(256) void expand_step_kernel(DevStep st, int n, int layout_col, void* out) {
    const uint64_t items = (1ull << (2 * n)) >> 2;
    for (uint64_t it = (uint64_t)blockIdx.x * 256u + threadIdx.x; it < items; it += (uint64_t)gridDim.x * 256u)
        expand_four<FMT>(st, n, layout_col, out, it << 2);
}

}  // namespace

hipError_t launch_expand_step(const DevStep& st, int n, int layout_col, OpFormat fmt, void* out,
                              hipStream_t stream) {
    const uint64_t N = 1ull << n;
    const uint64_t items = (N * N) >> 2;
    // Enough blocks to cover the chip several times over; larger matrices loop.
    const uint64_t want = (items + 255) / 256;
    const unsigned grid = (unsigned)(want < 8192 ? want : 8192);
    if (fmt == FMT_F32)
        hipLaunchKernelGGL(expand_step_kernel<FMT_F32>, dim3(grid), dim3(256), 0, stream, st, n, layout_col, out);
    else if (fmt == FMT_BF16)
        hipLaunchKernelGGL(expand_step_kernel<FMT_BF16>, dim3(grid), dim3(256), 0, stream, st, n, layout_col, out);
    else if (fmt == FMT_F16)
        hipLaunchKernelGGL(expand_step_kernel<FMT_F16>, dim3(grid), dim3(256), 0, stream, st, n, layout_col, out);
    else if (fmt == FMT_BF16_G)
        hipLaunchKernelGGL(expand_step_kernel<FMT_BF16_G>, dim3(grid), dim3(256), 0, stream, st, n, layout_col, out);
    else
        hipLaunchKernelGGL(expand_step_kernel<FMT_F16_G>, dim3(grid), dim3(256), 0, stream, st, n, layout_col, out);
    return hipGetLastError();
}

}  // namespace qsim
