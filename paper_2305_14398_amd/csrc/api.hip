// C ABI of libqsim (declared in include/qsim.h): argument validation, the
// float64 gate table (Section 2.3, Table 1; Section 5.2.2), step formation,
// and the host side of stages 4-6 of the unitary method (Section 5.3).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "engine.h"
#include "host.h"

using namespace qsim;

namespace qsim {

namespace {
thread_local std::string g_last_error = "no error";
}  // namespace

const std::string& last_error_text() { return g_last_error; }

qsim_status fail(qsim_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

qsim_status ok() {
    g_last_error = "no error";
    return QSIM_OK;
}

qsim_status device_fail(const char* what, hipError_t e) {
    return fail(QSIM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

bool valid_n(int n) { return n >= 1 && n <= QSIM_MAX_QUBITS; }

bool valid_prec(int p) { return p >= QSIM_FP32_4M && p <= QSIM_SPLIT_FP16_3M; }

// Precisions with a kernel in this library.
static bool built_prec(int p) { return valid_prec(p); }

static qsim_status check_gate(int n, const qsim_gate& g, int idx) {
    if (g.kind < QSIM_H || g.kind > QSIM_CUSTOM) return fail(QSIM_E_INVALID, "gate %d: unknown kind %d", idx, g.kind);
    if (g.kind != QSIM_CUSTOM && g.op_id != 0) return fail(QSIM_E_INVALID, "gate %d: op_id must be 0 unless CUSTOM", idx);
    if (g.target < 0 || g.target >= n)
        return fail(QSIM_E_INVALID, "gate %d: qubit %d outside 0..%d", idx, g.target, n - 1);
    if (g.kind == QSIM_CUSTOM) {
        const int m = custom_qubits(g.op_id);
        if (m == 0) return fail(QSIM_E_INVALID, "gate %d: custom operation %d is not registered", idx, g.op_id);
        if (g.control != -1) return fail(QSIM_E_INVALID, "gate %d: a custom operation takes no control", idx);
        if (g.target + m > n)
            return fail(QSIM_E_INVALID, "gate %d: custom range %d..%d outside 0..%d", idx, g.target, g.target + m - 1,
                        n - 1);
        return QSIM_OK;
    }
    if (g.kind == QSIM_SWAP && g.control < 0)
        return fail(QSIM_E_INVALID, "gate %d: SWAP needs its second qubit in `control`", idx);
    if (g.control >= n || g.control < -1)
        return fail(QSIM_E_INVALID, "gate %d: qubit %d outside 0..%d", idx, g.control, n - 1);
    if (g.control == g.target) return fail(QSIM_E_INVALID, "gate %d: control equals target (%d)", idx, g.target);
    if ((g.kind == QSIM_R || g.kind == QSIM_RX || g.kind == QSIM_RY || g.kind == QSIM_RZ) && !std::isfinite(g.theta))
        return fail(QSIM_E_INVALID, "gate %d: angle is not finite", idx);
    if (g.kind == QSIM_U2) {
        for (double v : g.u)
            if (!std::isfinite(v)) return fail(QSIM_E_INVALID, "gate %d: custom matrix entry is not finite", idx);
        // The operation data of a custom gate must be a unitary 2x2 (Section 5.2.2).
        const double* u = g.u;
        const double c00r = u[0] * u[0] + u[1] * u[1] + u[4] * u[4] + u[5] * u[5];
        const double c11r = u[2] * u[2] + u[3] * u[3] + u[6] * u[6] + u[7] * u[7];
        const double c01r = u[0] * u[2] + u[1] * u[3] + u[4] * u[6] + u[5] * u[7];
        const double c01i = u[0] * u[3] - u[1] * u[2] + u[4] * u[7] - u[5] * u[6];
        if (std::fabs(c00r - 1) > 1e-9 || std::fabs(c11r - 1) > 1e-9 || std::fabs(c01r) > 1e-9 || std::fabs(c01i) > 1e-9)
            return fail(QSIM_E_INVALID, "gate %d: custom 2x2 matrix is not unitary", idx);
    }
    return QSIM_OK;
}

qsim_status check_gates(int n, const qsim_gate* gates, int n_gates) {
    if (n_gates < 0) return fail(QSIM_E_INVALID, "negative gate count");
    if (n_gates > 0 && gates == nullptr) return fail(QSIM_E_INVALID, "gates is NULL");
    for (int i = 0; i < n_gates; ++i) {
        qsim_status st = check_gate(n, gates[i], i);
        if (st != QSIM_OK) return st;
    }
    return QSIM_OK;
}

static void span_of(const qsim_gate& g, int& lo, int& hi) {
    lo = g.target;
    hi = g.target;
    if (g.kind == QSIM_CUSTOM) {
        hi = g.target + custom_qubits(g.op_id) - 1;
        return;
    }
    if (g.control >= 0) {
        lo = g.control < lo ? g.control : lo;
        hi = g.control > hi ? g.control : hi;
    }
}

static uint32_t span_mask(const qsim_gate& g) {
    int lo, hi;
    span_of(g, lo, hi);
    return (uint32_t)(((1ull << (hi + 1)) - 1) & ~((1ull << lo) - 1));
}

// 2x2 float64 matrix of a gate kind, rows = output bit, (re, im) pairs.
void gate_matrix(const qsim_gate& g, double m[8]) {
    const double r2 = 0.70710678118654752440;
    for (int i = 0; i < 8; ++i) m[i] = 0.0;
    auto set = [&](int idx, double re, double im) {
        m[2 * idx] = re;
        m[2 * idx + 1] = im;
    };
    const double th = g.theta;
    switch (g.kind) {
        case QSIM_H: set(0, r2, 0); set(1, r2, 0); set(2, r2, 0); set(3, -r2, 0); break;
        case QSIM_X: set(1, 1, 0); set(2, 1, 0); break;
        case QSIM_Y: set(1, 0, -1); set(2, 0, 1); break;
        case QSIM_Z: set(0, 1, 0); set(3, -1, 0); break;
        case QSIM_S: set(0, 1, 0); set(3, 0, 1); break;
        case QSIM_T: set(0, 1, 0); set(3, r2, r2); break;
        case QSIM_R: set(0, 1, 0); set(3, std::cos(th), std::sin(th)); break;
        case QSIM_RX: {
            const double c = std::cos(th / 2), s = std::sin(th / 2);
            set(0, c, 0); set(1, 0, -s); set(2, 0, -s); set(3, c, 0);
            break;
        }
        case QSIM_RY: {
            const double c = std::cos(th / 2), s = std::sin(th / 2);
            set(0, c, 0); set(1, -s, 0); set(2, s, 0); set(3, c, 0);
            break;
        }
        case QSIM_RZ: {
            const double c = std::cos(th / 2), s = std::sin(th / 2);
            set(0, c, -s); set(3, c, s);
            break;
        }
        case QSIM_U2: for (int i = 0; i < 8; ++i) m[i] = g.u[i]; break;
        default: break;  // SWAP carries no matrix
    }
}

// Stage 3-4 input: the descriptor of one step (gates must be validated and
// pairwise span-disjoint).  Custom operations point at their matrix on the
// current device, so a descriptor that will be launched is built with the
// launch device current.
qsim_status make_step(int n, const qsim_gate* gates, int count, DevStep& st) {
    if (count > QSIM_MAX_GATES_PER_STEP)
        return fail(QSIM_E_INVALID, "step has %d gates (max %d)", count, QSIM_MAX_GATES_PER_STEP);
    std::memset(&st, 0, sizeof st);
    uint32_t used_span = 0, touched = 0;
    int order[QSIM_MAX_GATES_PER_STEP], top[QSIM_MAX_GATES_PER_STEP], bottom[QSIM_MAX_GATES_PER_STEP];
    for (int i = 0; i < count; ++i) {
        const uint32_t sm = span_mask(gates[i]);
        if (sm & used_span) return fail(QSIM_E_INVALID, "step gate %d overlaps the span of an earlier gate of the step", i);
        used_span |= sm;
        span_of(gates[i], bottom[i], top[i]);
        order[i] = i;
    }
    // Highest span first (spans are disjoint, so the order is total).
    std::sort(order, order + count, [&](int a, int b) { return top[a] > top[b]; });
    for (int slot = 0; slot < count; ++slot) {
        const int i = order[slot];
        const qsim_gate& g = gates[i];
        if (bottom[i] >= 2) st.n_prefix = slot + 1;
        DevGate& d = st.g[slot];
        if (g.kind == QSIM_CUSTOM) {
            d.type = GATE_CUSTOM;
            d.q0 = g.target;
            d.q1 = custom_qubits(g.op_id);
            int dev = 0;
            hipError_t e = hipGetDevice(&dev);
            if (e != hipSuccess) return device_fail("hipGetDevice", e);
            qsim_status cs = custom_device(g.op_id, dev, &d.ext);
            if (cs != QSIM_OK) return cs;
            touched |= span_mask(g);
            continue;
        }
        if (g.kind == QSIM_SWAP) {
            d.type = GATE_SWAP;
            d.q0 = g.target;
            d.q1 = g.control;
        } else if (g.control >= 0) {
            d.type = GATE_CTRL;
            d.q0 = g.control;
            d.q1 = g.target;
        } else {
            d.type = GATE_ONE;
            d.q0 = g.target;
            d.q1 = 0;
        }
        gate_matrix(g, d.m);
        touched |= 1u << g.target;
        if (g.control >= 0) touched |= 1u << g.control;
    }
    st.n_gates = count;
    const uint32_t all = (n >= 32) ? 0xffffffffu : ((1u << n) - 1u);
    st.idle_mask = all & ~touched;
    return QSIM_OK;
}

// Step formation: a gate joins the last step if its span is disjoint from
// every span already in that step, otherwise it opens a new one.
void pack(const qsim_gate* gates, int n_gates, std::vector<int32_t>& off) {
    off.clear();
    off.push_back(0);
    uint32_t last_span = 0;
    int last_count = 0;
    for (int i = 0; i < n_gates; ++i) {
        const uint32_t sm = span_mask(gates[i]);
        if (i > 0 && (sm & last_span) == 0 && last_count < QSIM_MAX_GATES_PER_STEP) {
            last_span |= sm;
            ++last_count;
        } else {
            if (i > 0) off.push_back(i);
            last_span = sm;
            last_count = 1;
        }
    }
    if (n_gates > 0) off.push_back(n_gates);
}

qsim_status check_offsets(const int32_t* off, int n_steps, int n_gates) {
    if (n_steps < 0) return fail(QSIM_E_INVALID, "negative step count");
    if (off[0] != 0 || off[n_steps] != n_gates)
        return fail(QSIM_E_INVALID, "step offsets must start at 0 and end at n_gates");
    for (int j = 0; j < n_steps; ++j) {
        const int c = off[j + 1] - off[j];
        if (c < 1 || c > QSIM_MAX_GATES_PER_STEP)
            return fail(QSIM_E_INVALID, "step %d has %d gates (must be 1..%d)", j, c, QSIM_MAX_GATES_PER_STEP);
    }
    return QSIM_OK;
}




qsim_status check_ctx(qsim_ctx* ctx) {
    if (ctx == nullptr) return fail(QSIM_E_INVALID, "context is NULL");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return device_fail("earlier device error", e);
    return QSIM_OK;
}

}  // namespace qsim

namespace qsim {

// Shared by the synchronous entry points and the serving engine.
qsim_status chain_impl(int n, const qsim_gate* gates, int n_gates, const int32_t* off, int n_steps, int prec, void* d_U,
                       void* d_ws, hipStream_t stream, Profiler* prof, const TuneTable& tune, bool fused) {
    const int tile = tune.get(prec, n);
    const size_t mb = mat_bytes(n);
    const OpFormat fmt = format_of(prec);
    DevStep st;
    qsim_status s;
    hipError_t e;
    if (n_steps == 0) {
        s = make_step(n, nullptr, 0, st);
        if (s != QSIM_OK) return s;
        e = timed(prof, QSIM_PROFILE_EXPAND, stream, [&] { return launch_expand_step(st, n, 0, FMT_F32, d_U, stream); });
        return e == hipSuccess ? QSIM_OK : device_fail("expand", e);
    }
    char* ws = static_cast<char*>(d_ws);
    if (fmt == FMT_F32) {
        // buffers: X0 = d_U, X1 = ws[1]; S = ws[0] (fused: X1 = ws[0], no S).
        // Product j (1..k-1) writes X[(k-1-j) % 2], so the last one lands in d_U.
        void* X[2] = {d_U, fused ? ws : ws + mb};
        void* S = ws;
        const bool gauss = prec == QSIM_FP32_3M;
        const int k = n_steps;
        void* cur = X[(k - 1) & 1];
        s = make_step(n, gates + off[0], off[1] - off[0], st);
        if (s != QSIM_OK) return s;
        e = timed(prof, QSIM_PROFILE_EXPAND, stream, [&] { return launch_expand_step(st, n, 0, FMT_F32, cur, stream); });
        if (e != hipSuccess) return device_fail("expand", e);
        for (int j = 1; j < k; ++j) {
            s = make_step(n, gates + off[j], off[j + 1] - off[j], st);
            if (s != QSIM_OK) return s;
            void* nxt = X[(k - 1 - j) & 1];
            if (fused) {
                e = timed(prof, QSIM_PROFILE_PRODUCT, stream, [&] {
                    return launch_cgemm_f32_fused(n, gauss, tile, st, static_cast<const float*>(cur),
                                                  static_cast<float*>(nxt), stream);
                });
            } else {
                e = timed(prof, QSIM_PROFILE_EXPAND, stream,
                          [&] { return launch_expand_step(st, n, 1, FMT_F32, S, stream); });
                if (e != hipSuccess) return device_fail("expand", e);
                e = timed(prof, QSIM_PROFILE_PRODUCT, stream, [&] {
                    return launch_cgemm_f32(n, gauss, tile, static_cast<const float*>(S),
                                            static_cast<const float*>(cur), static_cast<float*>(nxt), stream);
                });
            }
            if (e != hipSuccess) return device_fail("cgemm", e);
            cur = nxt;
        }
        return QSIM_OK;
    }
    // Split 16-bit operands: the running product is kept column-major in split
    // form (two ping-pong buffers), each step operator row-major in split form;
    // the last product is taken in the direct orientation and written as
    // float32 row-major into d_U.
    const size_t ob = op_bytes(n, prec);
    void* S = ws;
    void* P[2] = {ws + ob, ws + 2 * ob};
    const int k = n_steps;
    s = make_step(n, gates + off[0], off[1] - off[0], st);
    if (s != QSIM_OK) return s;
    if (k == 1) {
        e = timed(prof, QSIM_PROFILE_EXPAND, stream, [&] { return launch_expand_step(st, n, 0, FMT_F32, d_U, stream); });
        return e == hipSuccess ? QSIM_OK : device_fail("expand", e);
    }
    e = timed(prof, QSIM_PROFILE_EXPAND, stream, [&] { return launch_expand_step(st, n, 1, fmt, P[0], stream); });
    if (e != hipSuccess) return device_fail("expand", e);
    int cur = 0;
    for (int j = 1; j < k; ++j) {
        s = make_step(n, gates + off[j], off[j + 1] - off[j], st);
        if (s != QSIM_OK) return s;
        e = timed(prof, QSIM_PROFILE_EXPAND, stream, [&] { return launch_expand_step(st, n, 0, fmt, S, stream); });
        if (e != hipSuccess) return device_fail("expand", e);
        if (j < k - 1) {
            e = timed(prof, QSIM_PROFILE_PRODUCT, stream,
                      [&] { return launch_cgemm_split(n, fmt, tile, P[cur], S, P[cur ^ 1], nullptr, stream); });
            cur ^= 1;
        } else {
            e = timed(prof, QSIM_PROFILE_PRODUCT, stream, [&] {
                return launch_cgemm_split(n, fmt, tile, S, P[cur], nullptr, static_cast<float*>(d_U), stream);
            });
        }
        if (e != hipSuccess) return device_fail("cgemm_split", e);
    }
    return QSIM_OK;
}

}  // namespace qsim

extern "C" {

const char* qsim_last_error(void) { return last_error_text().c_str(); }

const char* qsim_version(void) { return "libqsim 0.1 (gfx950)"; }

qsim_status qsim_ctx_create(int device, qsim_ctx** out) {
    if (out == nullptr) return fail(QSIM_E_INVALID, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return device_fail("hipGetDeviceCount", e);
    if (device < 0 || device >= count) return fail(QSIM_E_RANGE, "device %d outside 0..%d", device, count - 1);
    DeviceGuard g(device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    qsim_ctx* c = new qsim_ctx;
    c->device = device;
    e = hipMalloc(&c->d_scratch, kScratchDoubles * sizeof(double));
    if (e != hipSuccess) {
        delete c;
        return device_fail("hipMalloc(scratch)", e);
    }
    *out = c;
    return ok();
}

qsim_status qsim_ctx_destroy(qsim_ctx* ctx) {
    if (ctx == nullptr) return ok();
    delete ctx->engine;  // serves admitted requests to completion first
    ctx->engine = nullptr;
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    delete ctx->prof;
    (void)hipFree(ctx->d_scratch);
    delete ctx;
    return ok();
}

qsim_status qsim_pack_steps(int n_qubits, const qsim_gate* gates, int n_gates, int32_t* step_offsets,
                            int* n_steps_out) {
    if (!valid_n(n_qubits)) return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", n_qubits, QSIM_MAX_QUBITS);
    if (step_offsets == nullptr || n_steps_out == nullptr) return fail(QSIM_E_INVALID, "output pointer is NULL");
    qsim_status s = check_gates(n_qubits, gates, n_gates);
    if (s != QSIM_OK) return s;
    std::vector<int32_t> off;
    pack(gates, n_gates, off);
    std::memcpy(step_offsets, off.data(), off.size() * sizeof(int32_t));
    *n_steps_out = (int)off.size() - 1;
    return ok();
}

size_t qsim_chain_workspace_bytes(int n_qubits, int prec) {
    if (!valid_n(n_qubits) || !valid_prec(prec)) return 0;
    return format_of(prec) == FMT_F32 ? 2 * mat_bytes(n_qubits) : 3 * op_bytes(n_qubits, prec);
}

size_t qsim_op_bytes(int n_qubits, int prec) {
    if (!valid_n(n_qubits) || !valid_prec(prec)) return 0;
    return op_bytes(n_qubits, prec);
}

size_t qsim_chain_fused_workspace_bytes(int n_qubits, int prec) {
    if (!valid_n(n_qubits) || !valid_prec(prec) || format_of(prec) != FMT_F32) return 0;
    return mat_bytes(n_qubits);
}

qsim_status qsim_build_step(qsim_ctx* ctx, int n_qubits, const qsim_gate* gates, int n_gates, int prec, int layout,
                            void* d_op, void* stream) {
    qsim_status s = QSIM_OK;
    if (!valid_n(n_qubits)) return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", n_qubits, QSIM_MAX_QUBITS);
    if (!valid_prec(prec)) return fail(QSIM_E_INVALID, "unknown precision %d", prec);
    if (layout != QSIM_LAYOUT_ROW && layout != QSIM_LAYOUT_COL) return fail(QSIM_E_INVALID, "unknown layout %d", layout);
    if (d_op == nullptr || !aligned(d_op)) return fail(QSIM_E_INVALID, "d_op is NULL or not 256-byte aligned");
    s = check_gates(n_qubits, gates, n_gates);
    if (s != QSIM_OK) return s;
    DevStep st;
    s = make_step(n_qubits, gates, n_gates, st);  // validation (the device pointers are rebuilt below)
    if (s != QSIM_OK) return s;
    s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    s = make_step(n_qubits, gates, n_gates, st);
    if (s != QSIM_OK) return s;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipError_t e = timed(ctx->prof, QSIM_PROFILE_EXPAND, hs,
                         [&] { return launch_expand_step(st, n_qubits, layout, format_of(prec), d_op, hs); });
    return e == hipSuccess ? ok() : device_fail("expand_step launch", e);
}

qsim_status qsim_step_multiply(qsim_ctx* ctx, int n_qubits, int prec, const void* d_S, const void* d_Uin, void* d_Uout,
                               void* d_Uout_split, void* stream) {
    qsim_status s = QSIM_OK;
    if (!valid_n(n_qubits)) return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", n_qubits, QSIM_MAX_QUBITS);
    if (!valid_prec(prec)) return fail(QSIM_E_INVALID, "unknown precision %d", prec);
    if (!built_prec(prec)) return fail(QSIM_E_INVALID, "precision %d is not available in this library", prec);
    const OpFormat fmt = format_of(prec);
    if (!d_S || !d_Uin || !aligned(d_S) || !aligned(d_Uin))
        return fail(QSIM_E_INVALID, "d_S / d_Uin is NULL or not 256-byte aligned");
    if (fmt == FMT_F32 && (d_Uout == nullptr || d_Uout_split != nullptr))
        return fail(QSIM_E_INVALID, "float32 precisions write d_Uout only (d_Uout_split must be NULL)");
    if (fmt != FMT_F32 && d_Uout == nullptr && d_Uout_split == nullptr)
        return fail(QSIM_E_INVALID, "split precisions need d_Uout and/or d_Uout_split");
    for (const void* o : {static_cast<const void*>(d_Uout), static_cast<const void*>(d_Uout_split)}) {
        if (o == nullptr) continue;
        if (!aligned(o)) return fail(QSIM_E_INVALID, "output not 256-byte aligned");
        if (o == d_S || o == d_Uin) return fail(QSIM_E_INVALID, "an output aliases an input");
    }
    if (d_Uout && d_Uout == d_Uout_split) return fail(QSIM_E_INVALID, "the two outputs alias");
    s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const int tile = ctx->tune.get(prec, n_qubits);
    hipError_t e = hipSuccess;
    if (fmt == FMT_F32) {
        e = timed(ctx->prof, QSIM_PROFILE_PRODUCT, hs, [&] {
            return launch_cgemm_f32(n_qubits, prec == QSIM_FP32_3M, tile, static_cast<const float*>(d_S),
                                    static_cast<const float*>(d_Uin), static_cast<float*>(d_Uout), hs);
        });
    } else {
        if (d_Uout_split)
            e = timed(ctx->prof, QSIM_PROFILE_PRODUCT, hs,
                      [&] { return launch_cgemm_split(n_qubits, fmt, tile, d_Uin, d_S, d_Uout_split, nullptr, hs); });
        if (e == hipSuccess && d_Uout)
            e = timed(ctx->prof, QSIM_PROFILE_PRODUCT, hs, [&] {
                return launch_cgemm_split(n_qubits, fmt, tile, d_S, d_Uin, nullptr, static_cast<float*>(d_Uout), hs);
            });
    }
    return e == hipSuccess ? ok() : device_fail("cgemm launch", e);
}

qsim_status qsim_step_multiply_fused(qsim_ctx* ctx, int n_qubits, int prec, const qsim_gate* gates, int n_gates,
                                     const void* d_Uin, void* d_Uout, void* stream) {
    qsim_status s = QSIM_OK;
    if (!valid_n(n_qubits)) return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", n_qubits, QSIM_MAX_QUBITS);
    if (!valid_prec(prec)) return fail(QSIM_E_INVALID, "unknown precision %d", prec);
    if (format_of(prec) != FMT_F32) return fail(QSIM_E_INVALID, "fused products are float32 (4M or 3M) only");
    if (!built_prec(prec)) return fail(QSIM_E_INVALID, "precision %d is not available in this library", prec);
    if (!d_Uin || !d_Uout || !aligned(d_Uin) || !aligned(d_Uout))
        return fail(QSIM_E_INVALID, "d_Uin / d_Uout is NULL or not 256-byte aligned");
    if (d_Uin == d_Uout) return fail(QSIM_E_INVALID, "d_Uout aliases d_Uin");
    s = check_gates(n_qubits, gates, n_gates);
    if (s != QSIM_OK) return s;
    DevStep st;
    s = make_step(n_qubits, gates, n_gates, st);  // validation (the device pointers are rebuilt below)
    if (s != QSIM_OK) return s;
    s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    s = make_step(n_qubits, gates, n_gates, st);
    if (s != QSIM_OK) return s;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const int tile = ctx->tune.get(prec, n_qubits);
    hipError_t e = timed(ctx->prof, QSIM_PROFILE_PRODUCT, hs, [&] {
        return launch_cgemm_f32_fused(n_qubits, prec == QSIM_FP32_3M, tile, st, static_cast<const float*>(d_Uin),
                                      static_cast<float*>(d_Uout), hs);
    });
    return e == hipSuccess ? ok() : device_fail("fused cgemm launch", e);
}

static qsim_status unitary_chain_entry(qsim_ctx* ctx, int n_qubits, const qsim_gate* gates, int n_gates,
                                       const int32_t* step_offsets, int n_steps, int prec, void* d_U, void* d_ws,
                                       size_t ws_bytes, void* stream, bool fused) {
    qsim_status s = QSIM_OK;
    if (!valid_n(n_qubits)) return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", n_qubits, QSIM_MAX_QUBITS);
    if (!valid_prec(prec)) return fail(QSIM_E_INVALID, "unknown precision %d", prec);
    if (!built_prec(prec)) return fail(QSIM_E_INVALID, "precision %d is not available in this library", prec);
    if (d_U == nullptr || !aligned(d_U)) return fail(QSIM_E_INVALID, "d_U is NULL or not 256-byte aligned");
    s = check_gates(n_qubits, gates, n_gates);
    if (s != QSIM_OK) return s;
    std::vector<int32_t> off;
    if (step_offsets == nullptr) {
        pack(gates, n_gates, off);
    } else {
        if (n_steps < 0) return fail(QSIM_E_INVALID, "negative step count");
        off.assign(step_offsets, step_offsets + n_steps + 1);
        s = check_offsets(off.data(), n_steps, n_gates);
        if (s != QSIM_OK) return s;
    }
    const int k = (int)off.size() - 1;
    if (k > 0) {
        if (d_ws == nullptr || !aligned(d_ws)) return fail(QSIM_E_INVALID, "d_ws is NULL or not 256-byte aligned");
        const size_t need =
            fused ? qsim_chain_fused_workspace_bytes(n_qubits, prec) : qsim_chain_workspace_bytes(n_qubits, prec);
        if (ws_bytes < need) return fail(QSIM_E_RANGE, "workspace %zu bytes, need %zu", ws_bytes, need);
        const char* w = static_cast<const char*>(d_ws);
        const char* u = static_cast<const char*>(d_U);
        if (u < w + need && w < u + mat_bytes(n_qubits)) return fail(QSIM_E_INVALID, "d_U overlaps the workspace");
    }
    // validate every step before the first launch
    DevStep st;
    for (int j = 0; j < k; ++j) {
        s = make_step(n_qubits, gates + off[j], off[j + 1] - off[j], st);
        if (s != QSIM_OK) return fail(s, "step %d: %s", j, last_error_text().c_str());
    }
    s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    s = chain_impl(n_qubits, gates, n_gates, off.data(), k, prec, d_U, d_ws, static_cast<hipStream_t>(stream), ctx->prof,
                   ctx->tune, fused);
    return s == QSIM_OK ? ok() : s;
}

qsim_status qsim_unitary_chain(qsim_ctx* ctx, int n_qubits, const qsim_gate* gates, int n_gates,
                               const int32_t* step_offsets, int n_steps, int prec, void* d_U, void* d_ws, size_t ws_bytes,
                               void* stream) {
    return unitary_chain_entry(ctx, n_qubits, gates, n_gates, step_offsets, n_steps, prec, d_U, d_ws, ws_bytes, stream,
                               false);
}

qsim_status qsim_unitary_chain_fused(qsim_ctx* ctx, int n_qubits, const qsim_gate* gates, int n_gates,
                                     const int32_t* step_offsets, int n_steps, int prec, void* d_U, void* d_ws,
                                     size_t ws_bytes, void* stream) {
    if (valid_prec(prec) && format_of(prec) != FMT_F32)
        return fail(QSIM_E_INVALID, "fused chains are float32 (4M or 3M) only");
    return unitary_chain_entry(ctx, n_qubits, gates, n_gates, step_offsets, n_steps, prec, d_U, d_ws, ws_bytes, stream,
                               true);
}

qsim_status qsim_apply_state(qsim_ctx* ctx, int n_qubits, const void* d_U, const void* d_psi0, void* d_psi,
                             double* d_prob, double* h_norm2, void* stream) {
    qsim_status s = QSIM_OK;
    if (!valid_n(n_qubits)) return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", n_qubits, QSIM_MAX_QUBITS);
    if (!d_U || !aligned(d_U) || !d_psi || !aligned(d_psi))
        return fail(QSIM_E_INVALID, "d_U / d_psi is NULL or not 256-byte aligned");
    if ((d_psi0 && !aligned(d_psi0)) || (d_prob && !aligned(d_prob)))
        return fail(QSIM_E_INVALID, "d_psi0 / d_prob not 256-byte aligned");
    if (d_psi == d_psi0) return fail(QSIM_E_INVALID, "d_psi aliases d_psi0");
    s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipError_t e = timed(ctx->prof, QSIM_PROFILE_APPLY, hs, [&] {
        return launch_apply_state(n_qubits, static_cast<const float*>(d_U), static_cast<const float*>(d_psi0),
                                  static_cast<float*>(d_psi), d_prob, ctx->d_scratch, hs);
    });
    if (e != hipSuccess) return device_fail("apply_state launch", e);
    if (h_norm2) {
        e = hipMemcpyAsync(h_norm2, ctx->d_scratch, sizeof(double), hipMemcpyDeviceToHost, hs);
        if (e == hipSuccess) e = hipStreamSynchronize(hs);
        if (e != hipSuccess) return device_fail("norm readback", e);
    }
    return ok();
}

qsim_status qsim_unitarity_drift(qsim_ctx* ctx, int n_qubits, const void* d_U, double* h_out, void* stream) {
    qsim_status s = QSIM_OK;
    if (!valid_n(n_qubits)) return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", n_qubits, QSIM_MAX_QUBITS);
    if (!d_U || !aligned(d_U) || !h_out) return fail(QSIM_E_INVALID, "d_U is NULL/unaligned or h_out is NULL");
    s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipError_t e = timed(ctx->prof, QSIM_PROFILE_DRIFT, hs, [&] {
        return launch_drift(n_qubits, static_cast<const float*>(d_U), ctx->d_scratch + 8, kDriftMaxPartials,
                            ctx->d_scratch + 2, hs);
    });
    if (e != hipSuccess) return device_fail("drift launch", e);
    e = hipMemcpyAsync(h_out, ctx->d_scratch + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return device_fail("drift readback", e);
    return ok();
}

qsim_status qsim_unitarity_drift_async(qsim_ctx* ctx, int n_qubits, const void* d_U, double* d_out, void* stream) {
    qsim_status s = QSIM_OK;
    if (!valid_n(n_qubits)) return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", n_qubits, QSIM_MAX_QUBITS);
    if (!d_U || !aligned(d_U)) return fail(QSIM_E_INVALID, "d_U is NULL or not 256-byte aligned");
    if (!d_out || (reinterpret_cast<uintptr_t>(d_out) & 7u)) return fail(QSIM_E_INVALID, "d_out is NULL or unaligned");
    s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipError_t e = timed(ctx->prof, QSIM_PROFILE_DRIFT, hs, [&] {
        return launch_drift(n_qubits, static_cast<const float*>(d_U), ctx->d_scratch + 8, kDriftMaxPartials, d_out,
                            hs);
    });
    return e == hipSuccess ? ok() : device_fail("drift launch", e);
}

qsim_status qsim_unitarity_drift_noalloc(int n_qubits, const void* d_U, double* d_out, void* stream) {
    if (!valid_n(n_qubits)) return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", n_qubits, QSIM_MAX_QUBITS);
    if (!d_U || !aligned(d_U)) return fail(QSIM_E_INVALID, "d_U is NULL or not 256-byte aligned");
    if (!d_out || (reinterpret_cast<uintptr_t>(d_out) & 7u)) return fail(QSIM_E_INVALID, "d_out is NULL or unaligned");
    double* partials = nullptr;
    size_t bytes = 0;
    hipError_t e = drift_static_scratch(&partials, &bytes);
    if (e != hipSuccess) return device_fail("drift scratch address", e);
    // launch_drift never runs more workgroups than kDriftMaxPartials, one pair each.
    if (bytes < 2 * (size_t)kDriftMaxPartials * sizeof(double))
        return fail(QSIM_E_RANGE, "static drift scratch holds %zu bytes, %zu needed", bytes,
                    2 * (size_t)kDriftMaxPartials * sizeof(double));
    e = launch_drift(n_qubits, static_cast<const float*>(d_U), partials, kDriftMaxPartials, d_out,
                     static_cast<hipStream_t>(stream));
    return e == hipSuccess ? ok() : device_fail("drift launch", e);
}

qsim_status qsim_profile_enable(qsim_ctx* ctx, int enable) {
    if (ctx == nullptr) return fail(QSIM_E_INVALID, "context is NULL");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    delete ctx->prof;
    ctx->prof = enable ? new Profiler : nullptr;
    return ok();
}

qsim_status qsim_profile_read(qsim_ctx* ctx, qsim_kernel_stats* out) {
    if (ctx == nullptr || out == nullptr) return fail(QSIM_E_INVALID, "context or out is NULL");
    if (ctx->prof == nullptr) return fail(QSIM_E_INVALID, "profiling is not enabled on this context");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    hipError_t e = ctx->prof->collect();
    if (e != hipSuccess) return device_fail("event timing", e);
    for (int k = 0; k < QSIM_PROFILE_KINDS; ++k) {
        out->count[k] = ctx->prof->count[k];
        out->total_ms[k] = ctx->prof->total_ms[k];
    }
    return ok();
}

qsim_status qsim_unitarity_drift_probe(qsim_ctx* ctx, int n_qubits, const void* d_U, double* h_out, void* stream) {
    qsim_status s = QSIM_OK;
    if (!valid_n(n_qubits)) return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", n_qubits, QSIM_MAX_QUBITS);
    if (!d_U || !aligned(d_U) || !h_out) return fail(QSIM_E_INVALID, "d_U is NULL/unaligned or h_out is NULL");
    s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipError_t e = timed(ctx->prof, QSIM_PROFILE_DRIFT, hs, [&] {
        return launch_drift_probe(n_qubits, static_cast<const float*>(d_U), ctx->d_scratch + kProbeScratchOffset,
                                  ctx->d_scratch + 4, hs);
    });
    if (e != hipSuccess) return device_fail("probe drift launch", e);
    e = hipMemcpyAsync(h_out, ctx->d_scratch + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return device_fail("probe drift readback", e);
    return ok();
}

qsim_status qsim_sample(qsim_ctx* ctx, int n_qubits, const double* d_prob, const double* d_uniform, int shots,
                        int64_t* d_out, void* stream) {
    qsim_status s = QSIM_OK;
    if (!valid_n(n_qubits)) return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", n_qubits, QSIM_MAX_QUBITS);
    if (shots < 0) return fail(QSIM_E_INVALID, "negative shot count");
    if (!d_prob || !aligned(d_prob)) return fail(QSIM_E_INVALID, "d_prob is NULL or not 256-byte aligned");
    if (shots > 0 && (!d_uniform || !d_out || !aligned(d_uniform) || !aligned(d_out)))
        return fail(QSIM_E_INVALID, "d_uniform / d_out is NULL or not 256-byte aligned");
    s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipError_t e = launch_sample(n_qubits, d_prob, d_uniform, shots, d_out, ctx->d_scratch + kProbeScratchOffset, hs);
    return e == hipSuccess ? ok() : device_fail("sample launch", e);
}

}  // extern "C"
