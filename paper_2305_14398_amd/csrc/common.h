// Internal declarations shared by the libqsim host code and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qsim.h"

namespace qsim {

// One gate of a step, as the expansion kernel reads it.  The 2x2 matrix is
// float64, row-major (re, im) pairs, rows indexed by the output bit.
enum : int32_t { GATE_ONE = 1, GATE_CTRL = 2, GATE_SWAP = 3 };

struct DevGate {
    int32_t type;  // GATE_ONE: q0 = qubit; GATE_CTRL: q0 = control, q1 = target; GATE_SWAP: q0, q1
    int32_t q0;
    int32_t q1;
    int32_t pad;
    double m[8];
};

// A step descriptor small enough to travel as a kernel argument (by value).
struct DevStep {
    int32_t n_gates;
    uint32_t idle_mask;  // bit q set: no gate of the step touches qubit q
    int32_t pad[2];
    DevGate g[QSIM_MAX_GATES_PER_STEP];
};

// Output formats of the expansion kernel and operand formats of the GEMMs.
enum OpFormat : int { FMT_F32 = 0, FMT_BF16 = 1, FMT_F16 = 2 };

inline OpFormat format_of(int prec) {
    return prec == QSIM_SPLIT_BF16 ? FMT_BF16 : prec == QSIM_SPLIT_FP16 ? FMT_F16 : FMT_F32;
}

// ---- kernel launchers (each returns the launch status) ----
hipError_t launch_expand_step(const DevStep& st, int n, int layout_col, OpFormat fmt, void* out,
                              hipStream_t stream);
hipError_t launch_cgemm_f32(int n, bool gauss, const float* S_col, const float* U_row, float* C_row,
                            hipStream_t stream);
// D = X Y^T over split operands (see cgemm_split.hip); D_split and/or D_f32 row-major.
hipError_t launch_cgemm_split(int n, OpFormat fmt, const void* X, const void* Y, void* D_split, float* D_f32,
                              hipStream_t stream);
hipError_t launch_apply_state(int n, const float* U_row, const float* psi0, float* psi, double* prob,
                              double* d_norm2, hipStream_t stream);
hipError_t launch_drift(int n, const float* U_row, double* partials, int max_partials, double* d_out,
                        hipStream_t stream);

constexpr int kDriftMaxPartials = 2048;

}  // namespace qsim
