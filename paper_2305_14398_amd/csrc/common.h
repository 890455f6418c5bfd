// Internal declarations shared by the libqsim host code and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qsim.h"

namespace qsim {

// One gate of a step, as the expansion kernel reads it.  The 2x2 matrix is
// float64, row-major (re, im) pairs, rows indexed by the output bit.
enum : int32_t { GATE_ONE = 1, GATE_CTRL = 2, GATE_SWAP = 3, GATE_CUSTOM = 4 };

struct DevGate {
    int32_t type;  // GATE_ONE: q0 = qubit; GATE_CTRL: q0 = control, q1 = target; GATE_SWAP: q0, q1;
                   // GATE_CUSTOM: qubits q0 .. q0+q1-1, matrix at ext
    int32_t q0;
    int32_t q1;
    int32_t pad;
    const double* ext;  // GATE_CUSTOM: 2^q1 x 2^q1 row-major (re, im) float64 on the launch device
    double m[8];
};

// A step descriptor small enough to travel as a kernel argument (by value).
// Gates are stored in descending order of their span's top qubit, so the
// n_prefix gates whose spans leave out qubits 0 and 1 come first (the others,
// at most two, have the lowest spans).
struct DevStep {
    int32_t n_gates;
    uint32_t idle_mask;  // bit q set: no gate of the step touches qubit q
    int32_t n_prefix;
    int32_t pad;
    DevGate g[QSIM_MAX_GATES_PER_STEP];
};

// One step operator to expand inside a grouped launch.  Job j owns the
// workgroup-iterations [block_begin, block_begin + blocks) of the launch.
struct ExpandJob {
    DevStep st;
    void* out;
    int32_t n;
    int32_t layout_col;
    int32_t fmt;  // OpFormat
    int32_t block_begin;
    int32_t blocks;
    int32_t pad[3];
};

// One chain product inside a grouped launch (all jobs of a launch share the
// arithmetic family).  float32: X = S column-major, Y = U row-major, D0 = C
// row-major.  Split: D = X Y^T with D0 = split output, D1 = float32 output
// (either may be null).  cfg: 0 = whole product by one workgroup (n <= 5),
// 64 or 128 = MFMA tile edge.  Job j owns tiles [tile_begin, tile_begin + tiles).
struct GemmJob {
    const void* X;
    const void* Y;
    void* D0;
    void* D1;
    int32_t n;
    int32_t cfg;
    int32_t tile_begin;
    int32_t tiles;
};

// Output formats of the expansion kernel and operand formats of the GEMMs:
// planar float32; four split 16-bit planes (re_hi, re_lo, im_hi, im_lo); or six
// (the same plus sum_hi, sum_lo of re + im) for the three-product split forms.
enum OpFormat : int { FMT_F32 = 0, FMT_BF16 = 1, FMT_F16 = 2, FMT_BF16_G = 3, FMT_F16_G = 4 };

inline OpFormat format_of(int prec) {
    switch (prec) {
        case QSIM_SPLIT_BF16: return FMT_BF16;
        case QSIM_SPLIT_FP16: return FMT_F16;
        case QSIM_SPLIT_BF16_3M: return FMT_BF16_G;
        case QSIM_SPLIT_FP16_3M: return FMT_F16_G;
        default: return FMT_F32;
    }
}
inline bool is_split(int prec) { return format_of(prec) != FMT_F32; }
// 16-bit element type of a split format (FMT_BF16 or FMT_F16), FMT_F32 otherwise.
__host__ __device__ constexpr int fmt_elem(int fmt) {
    return fmt == FMT_BF16_G ? FMT_BF16 : fmt == FMT_F16_G ? FMT_F16 : fmt;
}
__host__ __device__ constexpr bool fmt_gauss(int fmt) { return fmt == FMT_BF16_G || fmt == FMT_F16_G; }
// Bytes of one N x N operand in a format (8 N^2 for float32 and four planes, 12 N^2 for six).
inline size_t fmt_bytes(int fmt, int n) { return (fmt_gauss(fmt) ? 12u : 8u) * ((size_t)1 << (2 * n)); }

// float32 -> bfloat16, round to nearest even (inputs are finite).
__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ---- kernel launchers (each returns the launch status) ----
hipError_t launch_expand_step(const DevStep& st, int n, int layout_col, OpFormat fmt, void* out,
                              hipStream_t stream);
hipError_t launch_cgemm_f32(int n, bool gauss, int tile, const float* S_col, const float* U_row, float* C_row,
                            hipStream_t stream);
// C = S . U with S (a step operator) computed inside the product, never stored.
hipError_t launch_cgemm_f32_fused(int n, bool gauss, int tile, const DevStep& st, const float* U_row, float* C_row,
                                  hipStream_t stream);
// D = X Y^T over split operands (see cgemm_split.hip); D_split and/or D_f32 row-major.
hipError_t launch_cgemm_split(int n, OpFormat fmt, int tile, const void* X, const void* Y, void* D_split,
                              float* D_f32, hipStream_t stream);
// Grouped launches over device job tables (grouped.hip).  `grid` workgroups
// loop over the `total` tiles / expansion blocks.
hipError_t launch_grouped_expand(const ExpandJob* jobs, int njobs, int total_blocks, int grid, hipStream_t stream);
hipError_t launch_grouped_gemm(int prec, const GemmJob* jobs, int njobs, int total_tiles, int grid,
                               hipStream_t stream);
hipError_t launch_apply_state(int n, const float* U_row, const float* psi0, float* psi, double* prob,
                              double* d_norm2, hipStream_t stream);
hipError_t launch_sample(int n, const double* prob, const double* uniforms, int shots, int64_t* out, double* cdf,
                         hipStream_t stream);
hipError_t launch_drift(int n, const float* U_row, double* partials, int max_partials, double* d_out,
                        hipStream_t stream);

constexpr int kDriftMaxPartials = 2048;
// Probe drift: partial sums of at most this many complex entries (chunks * N).
constexpr int kProbeChunkEntries = 1 << 19;
// Doubles of scratch the probe needs: y (2 N) + partials (2 * kProbeChunkEntries).
constexpr size_t kProbeScratchDoubles = 2 * ((size_t)1 << QSIM_MAX_QUBITS) + 2 * (size_t)kProbeChunkEntries;
hipError_t launch_drift_probe(int n, const float* U_row, double* scratch, double* d_out, hipStream_t stream);
// Device address (on the current device) and size of the drift's static
// partial-sum array, for the allocation-free drift entry point.
hipError_t drift_static_scratch(double** out, size_t* bytes);

}  // namespace qsim
