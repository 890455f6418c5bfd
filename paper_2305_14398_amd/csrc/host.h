// Host-side internals of libqsim shared by the C ABI (api.hip), the batch
// planner (batch.hip) and the serving engine (engine.hip).
#pragma once

#include <string>
#include <vector>

#include "common.h"

namespace qsim {

class Engine;


// --- status and validation (api.hip) ---
qsim_status fail(qsim_status st, const char* fmt, ...);
qsim_status ok();
qsim_status device_fail(const char* what, hipError_t e);
const std::string& last_error_text();
bool aligned(const void* p);
bool valid_n(int n);
bool valid_prec(int p);
qsim_status check_gates(int n, const qsim_gate* gates, int n_gates);
qsim_status check_offsets(const int32_t* off, int n_steps, int n_gates);
// Operation data provider (registry.hip): qubit count of a registered custom
// operation (0 if unknown), its host matrix, and its float64 copy on device `dev`.
int custom_qubits(int32_t id);
const double* custom_host(int32_t id);
qsim_status custom_device(int32_t id, int dev, const double** out);
// 2x2 float64 matrix of a gate (row-major (re, im) pairs, rows = output bit); SWAP has none.
void gate_matrix(const qsim_gate& g, double m[8]);
// Descriptor of one step (gates validated and pairwise span-disjoint).
qsim_status make_step(int n, const qsim_gate* gates, int count, DevStep& st);
// Step formation rule (see qsim_pack_steps).
void pack(const qsim_gate* gates, int n_gates, std::vector<int32_t>& off);
inline size_t mat_bytes(int n) { return (size_t)8 << (2 * n); }
// Bytes of one chain operand (step operator or running product) in the format of `prec`.
inline size_t op_bytes(int n, int prec) { return fmt_bytes(format_of(prec), n); }

// Makes `dev` current for the lifetime of the guard and restores the caller's device.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Optional per-launch timing with HIP events recorded on the launch stream
// around each kernel (qsim_profile_enable / qsim_profile_read).  Used from one
// host thread at a time.
struct Profiler {
    struct Pending {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Pending> pending;
    double total_ms[QSIM_PROFILE_KINDS] = {};
    int64_t count[QSIM_PROFILE_KINDS] = {};

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    hipError_t collect() {
        hipError_t err = hipSuccess;
        for (auto& p : pending) {
            float ms = 0.f;
            hipError_t e = hipEventSynchronize(p.b);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
            if (e == hipSuccess) {
                total_ms[p.kind] += ms;
                count[p.kind] += 1;
            } else {
                err = e;
            }
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
        return err;
    }
    ~Profiler() {
        (void)collect();
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

// Runs `launch` (returning hipError_t) bracketed by events when profiling.
template <class F>
hipError_t timed(Profiler* prof, int kind, hipStream_t s, F&& launch) {
    if (prof == nullptr) return launch();
    hipEvent_t a = prof->get(), b = prof->get();
    (void)hipEventRecord(a, s);
    hipError_t e = launch();
    (void)hipEventRecord(b, s);
    prof->pending.push_back({kind, a, b});
    return e;
}


// MFMA tile edge per qubit count, per precision; filled by the autotuner or by
// the default rule (128 for n >= 7, 64 for n = 6).  The four-product split
// fp16 form always uses 64: its 128-wide tile needs every register and would
// spill inside the grouped kernel.
constexpr int kPrecisions = QSIM_SPLIT_FP16_3M + 1;
struct TuneTable {
    static int family(int prec) { return prec; }
    int tile[kPrecisions][QSIM_MAX_QUBITS + 1];
    bool tuned[kPrecisions];
    // milliseconds per product measured by the autotuner for tile 64 and 128 (-1: not measured)
    double ms[kPrecisions][QSIM_MAX_QUBITS + 1][2];
    TuneTable() {
        for (int f = 0; f < kPrecisions; ++f) {
            tuned[f] = false;
            for (int n = 0; n <= QSIM_MAX_QUBITS; ++n) {
                tile[f][n] = n >= 7 && f != QSIM_SPLIT_FP16 ? 128 : (n >= 6 ? 64 : 0);
                ms[f][n][0] = ms[f][n][1] = -1.0;
            }
        }
    }
    // Never wider than the matrix: n = 6 always uses 64, n <= 5 the whole-product path.
    int get(int prec, int n) const {
        if (n <= 5) return 0;
        if (n == 6) return 64;
        return tile[family(prec)][n];
    }
};

// Shared by the synchronous entry points and the serving engine.
// fused: float32 precisions only; every product after the first step computes
// its step operator inside the product (no scratch operator in d_ws).
qsim_status chain_impl(int n, const qsim_gate* gates, int n_gates, const int32_t* off, int n_steps, int prec, void* d_U,
                       void* d_ws, hipStream_t stream, Profiler* prof, const TuneTable& tune, bool fused = false);

// Workgroups of a persistent grouped product launch on `cus` compute units:
// 4M float32 tiles (256 threads, 67.5 KB LDS) fit two per CU; 3M tiles (512
// threads, 240 registers) and split tiles (128 KB LDS) one.
inline int grouped_gemm_grid(int prec, int cus) { return prec == QSIM_FP32_4M ? 2 * cus : cus; }

// Context scratch layout (doubles): [0] norm2, [2..3] drift, [4..5] probe
// drift, [8, 8 + 2*kDriftMaxPartials) drift partials, then the probe scratch.
constexpr size_t kProbeScratchOffset = 8 + 2 * kDriftMaxPartials;
constexpr size_t kScratchDoubles = kProbeScratchOffset + kProbeScratchDoubles;

}  // namespace qsim

struct qsim_ctx {
    int device = 0;
    double* d_scratch = nullptr;  // [0] norm2, [2..3] drift result, [8..] drift partials
    qsim::Profiler* prof = nullptr;
    qsim::TuneTable tune;
    qsim::Engine* engine = nullptr;
};

namespace qsim {
qsim_status check_ctx(qsim_ctx* ctx);
}  // namespace qsim
