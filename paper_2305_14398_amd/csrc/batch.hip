// Batches of circuits of mixed size (stages 4-5 of Section 5.3 for many
// circuits at once) and the tile autotuner.
//
// A plan turns a batch into "iterations": iteration j expands step j of every
// circuit that has one (one grouped launch) and, for j >= 1, takes the j-th
// chain product of each of those circuits (one grouped launch).  The job tables
// of all iterations are built and uploaded once when the plan is created; a
// launch only enqueues 2 kernels per iteration, and with QSIM_BATCH_GRAPH the
// whole sequence is captured once into a hipGraph and replayed.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>

#ifndef QSIM_BUILD_ID
#define QSIM_BUILD_ID "unknown"
#endif

#include "chain_jobs.h"

using namespace qsim;

struct qsim_batch_plan {
    qsim_ctx* ctx = nullptr;
    int prec = 0;
    int count = 0;
    int grid_expand = 0, grid_gemm = 0;
    struct Iter {
        int e_off, e_cnt, e_total;  // expand jobs [e_off, e_off+e_cnt), total workgroup-iterations
        int g_off, g_cnt, g_total;  // product jobs, total tiles
    };
    std::vector<Iter> iters;
    ExpandJob* d_expand = nullptr;
    GemmJob* d_gemm = nullptr;
    double flops = 0.0;  // 8 N^3 per product
    int products = 0;
    bool use_graph = false;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Operand words for the autotuner's timing runs: seeded pseudo-random
// mantissas under a fixed small exponent, so the timed products switch their
// multiplier inputs as dense chain operands do (all-zero operands run faster
// than any real chain, and the tile chosen on them need not be the fastest).
__global__ __launch_bounds__(256) void tune_fill_kernel(uint32_t* __restrict__ p, size_t words, uint32_t seed,
                                                        uint32_t one, uint32_t mant) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (size_t)gridDim.x * 256) {
        uint32_t x = (uint32_t)i * 0x9e3779b9u ^ seed;
        x ^= x >> 16;
        x *= 0x7feb352du;
        x ^= x >> 15;
        x *= 0x846ca68bu;
        x ^= x >> 16;
        p[i] = one | (x & mant);
    }
}

size_t per_circuit_ws(int n, int prec) {
    return is_split(prec) ? 3 * align256(op_bytes(n, prec)) : 2 * align256(mat_bytes(n));
}

qsim_status check_desc(const qsim_circuit_desc& c, int idx, std::vector<int32_t>& off) {
    if (!valid_n(c.n_qubits)) return fail(QSIM_E_RANGE, "circuit %d: n_qubits %d outside 1..%d", idx, c.n_qubits, QSIM_MAX_QUBITS);
    if (c.reserved != 0) return fail(QSIM_E_INVALID, "circuit %d: reserved field must be 0", idx);
    qsim_status s = check_gates(c.n_qubits, c.gates, c.n_gates);
    if (s != QSIM_OK) return fail(s, "circuit %d: %s", idx, last_error_text().c_str());
    if (c.step_offsets == nullptr) {
        pack(c.gates, c.n_gates, off);
    } else {
        if (c.n_steps < 0) return fail(QSIM_E_INVALID, "circuit %d: negative step count", idx);
        off.assign(c.step_offsets, c.step_offsets + c.n_steps + 1);
        s = check_offsets(off.data(), c.n_steps, c.n_gates);
        if (s != QSIM_OK) return fail(s, "circuit %d: %s", idx, last_error_text().c_str());
    }
    if (c.d_U == nullptr || !aligned(c.d_U)) return fail(QSIM_E_INVALID, "circuit %d: d_U is NULL or not 256-byte aligned", idx);
    return QSIM_OK;
}

int device_cus(int device) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0) cus = 256;
    return cus;
}

int tiles_of(int n, int cfg) { return ChainCursor::tiles_of(n, cfg); }

hipError_t enqueue(qsim_batch_plan* p, hipStream_t s) {
    for (const auto& it : p->iters) {
        hipError_t e = launch_grouped_expand(p->d_expand + it.e_off, it.e_cnt, it.e_total,
                                             std::min(it.e_total, p->grid_expand), s);
        if (e != hipSuccess) return e;
        e = launch_grouped_gemm(p->prec, p->d_gemm + it.g_off, it.g_cnt, it.g_total, std::min(it.g_total, p->grid_gemm), s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

qsim_status qsim_batch_workspace_bytes(const qsim_circuit_desc* circuits, int count, int prec, size_t* out) {
    if (out == nullptr) return fail(QSIM_E_INVALID, "out is NULL");
    *out = 0;
    if (count < 0 || (count > 0 && circuits == nullptr)) return fail(QSIM_E_INVALID, "bad circuit list");
    if (!valid_prec(prec)) return fail(QSIM_E_INVALID, "unknown precision %d", prec);
    size_t total = 0;
    for (int i = 0; i < count; ++i) {
        if (!valid_n(circuits[i].n_qubits)) return fail(QSIM_E_RANGE, "circuit %d: n_qubits out of range", i);
        total += per_circuit_ws(circuits[i].n_qubits, prec);
    }
    *out = total;
    return ok();
}

qsim_status qsim_batch_plan_create(qsim_ctx* ctx, const qsim_circuit_desc* circuits, int count, int prec, void* d_ws,
                                   size_t ws_bytes, int flags, qsim_batch_plan** out) {
    if (out == nullptr) return fail(QSIM_E_INVALID, "out is NULL");
    *out = nullptr;
    if (count <= 0 || circuits == nullptr) return fail(QSIM_E_INVALID, "empty circuit list");
    if (!valid_prec(prec)) return fail(QSIM_E_INVALID, "unknown precision %d", prec);
    if (flags & ~QSIM_BATCH_GRAPH) return fail(QSIM_E_INVALID, "unknown flags 0x%x", flags);
    std::vector<std::vector<int32_t>> offs(count);
    size_t need = 0;
    for (int i = 0; i < count; ++i) {
        qsim_status s = check_desc(circuits[i], i, offs[i]);
        if (s != QSIM_OK) return s;
        need += per_circuit_ws(circuits[i].n_qubits, prec);
    }
    if (ws_bytes < need) return fail(QSIM_E_RANGE, "workspace %zu bytes, need %zu", ws_bytes, need);
    if (need > 0 && (d_ws == nullptr || !aligned(d_ws))) return fail(QSIM_E_INVALID, "d_ws is NULL or not 256-byte aligned");
    // outputs must be distinct and outside the workspace
    {
        std::vector<std::pair<const char*, const char*>> ranges;
        for (int i = 0; i < count; ++i) {
            const char* u = static_cast<const char*>(circuits[i].d_U);
            ranges.push_back({u, u + mat_bytes(circuits[i].n_qubits)});
        }
        std::sort(ranges.begin(), ranges.end());
        for (size_t i = 1; i < ranges.size(); ++i)
            if (ranges[i].first < ranges[i - 1].second) return fail(QSIM_E_INVALID, "two circuits' d_U overlap");
        const char* w = static_cast<const char*>(d_ws);
        for (auto& r : ranges)
            if (need > 0 && r.first < w + need && w < r.second) return fail(QSIM_E_INVALID, "a d_U overlaps the workspace");
    }
    qsim_status s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    // Step descriptors hold device pointers of custom operations: build them on the context's device.
    DeviceGuard dg(ctx->device);
    if (dg.err != hipSuccess) return device_fail("hipSetDevice", dg.err);

    // Host job tables, per iteration.
    int maxk = 1;
    for (int i = 0; i < count; ++i) maxk = std::max<int>(maxk, (int)offs[i].size() - 1);
    std::vector<std::vector<ExpandJob>> ej(maxk);
    std::vector<std::vector<GemmJob>> gj(maxk);
    char* ws = static_cast<char*>(d_ws);
    size_t base = 0;
    double flops = 0.0;
    int products = 0;
    for (int i = 0; i < count; ++i) {
        const qsim_circuit_desc& c = circuits[i];
        const int n = c.n_qubits;
        const int k = (int)offs[i].size() - 1;
        const size_t mb = is_split(prec) ? align256(op_bytes(n, prec)) : align256(mat_bytes(n));
        char* S = ws + base;
        char* W1 = ws + base + mb;
        char* W2 = ws + base + 2 * mb;
        base += per_circuit_ws(n, prec);
        ChainCursor cc;
        cc.n = n;
        cc.k = k;
        cc.prec = prec;
        cc.cfg = n <= 5 ? 0 : ctx->tune.get(prec, n);
        cc.gates = c.gates;
        cc.off = offs[i];
        cc.U = c.d_U;
        cc.S = S;
        cc.W1 = W1;
        cc.W2 = W2;
        for (int j = 0; j < std::max(k, 1); ++j) {
            ExpandJob E;
            GemmJob Gj;
            bool has_gemm = false;
            s = cc.emit(j, E, Gj, has_gemm);
            if (s != QSIM_OK) return fail(s, "circuit %d step %d: %s", i, j, last_error_text().c_str());
            ej[j].push_back(E);
            if (has_gemm) {
                gj[j].push_back(Gj);
                flops += 8.0 * (double)(1ll << (3 * n));
                ++products;
            }
        }
    }

    qsim_batch_plan* p = new qsim_batch_plan;
    p->ctx = ctx;
    p->prec = prec;
    p->count = count;
    p->flops = flops;
    p->products = products;
    p->use_graph = (flags & QSIM_BATCH_GRAPH) != 0;
    const int cus = device_cus(ctx->device);
    p->grid_expand = cus * 8;
    p->grid_gemm = grouped_gemm_grid(prec, cus);
    std::vector<ExpandJob> all_e;
    std::vector<GemmJob> all_g;
    for (int j = 0; j < maxk; ++j) {
        // Largest jobs first so the persistent grid ends with the small ones.
        std::stable_sort(ej[j].begin(), ej[j].end(), [](const ExpandJob& a, const ExpandJob& b) { return a.n > b.n; });
        std::stable_sort(gj[j].begin(), gj[j].end(), [](const GemmJob& a, const GemmJob& b) { return a.n > b.n; });
        qsim_batch_plan::Iter it;
        it.e_off = (int)all_e.size();
        it.e_cnt = (int)ej[j].size();
        int tot = 0;
        for (auto& J : ej[j]) {
            J.block_begin = tot;
            tot += J.blocks;
            all_e.push_back(J);
        }
        it.e_total = tot;
        it.g_off = (int)all_g.size();
        it.g_cnt = (int)gj[j].size();
        tot = 0;
        for (auto& G : gj[j]) {
            G.tile_begin = tot;
            tot += G.tiles;
            all_g.push_back(G);
        }
        it.g_total = tot;
        p->iters.push_back(it);
    }
    DeviceGuard g(ctx->device);
    hipError_t e = g.err;
    if (e == hipSuccess) e = hipMalloc(&p->d_expand, std::max<size_t>(1, all_e.size()) * sizeof(ExpandJob));
    if (e == hipSuccess) e = hipMalloc(&p->d_gemm, std::max<size_t>(1, all_g.size()) * sizeof(GemmJob));
    if (e == hipSuccess && !all_e.empty())
        e = hipMemcpy(p->d_expand, all_e.data(), all_e.size() * sizeof(ExpandJob), hipMemcpyHostToDevice);
    if (e == hipSuccess && !all_g.empty())
        e = hipMemcpy(p->d_gemm, all_g.data(), all_g.size() * sizeof(GemmJob), hipMemcpyHostToDevice);
    if (e == hipSuccess && p->use_graph) e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        qsim_batch_plan_destroy(p);
        return device_fail("batch plan setup", e);
    }
    *out = p;
    return ok();
}

qsim_status qsim_batch_plan_launch(qsim_batch_plan* p, void* stream) {
    if (p == nullptr) return fail(QSIM_E_INVALID, "plan is NULL");
    qsim_status s = check_ctx(p->ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(p->ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (!p->use_graph) {
        hipError_t e = enqueue(p, hs);
        return e == hipSuccess ? ok() : device_fail("grouped launch", e);
    }
    if (p->exec == nullptr) {
        // Capture on the plan's own stream (capturing the null stream is not allowed).
        hipError_t e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return device_fail("hipStreamBeginCapture", e);
        hipError_t le = enqueue(p, p->capture_stream);
        e = hipStreamEndCapture(p->capture_stream, &p->graph);
        if (le != hipSuccess) return device_fail("grouped launch under capture", le);
        if (e != hipSuccess) return device_fail("hipStreamEndCapture", e);
        e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            p->exec = nullptr;
            return device_fail("hipGraphInstantiate", e);
        }
    }
    hipError_t e = hipGraphLaunch(p->exec, hs);
    return e == hipSuccess ? ok() : device_fail("hipGraphLaunch", e);
}

qsim_status qsim_batch_plan_info(const qsim_batch_plan* p, int* iterations, int* products, double* flops) {
    if (p == nullptr) return fail(QSIM_E_INVALID, "plan is NULL");
    if (iterations) *iterations = (int)p->iters.size();
    if (products) *products = p->products;
    if (flops) *flops = p->flops;
    return ok();
}

qsim_status qsim_batch_plan_destroy(qsim_batch_plan* p) {
    if (p == nullptr) return ok();
    DeviceGuard g(p->ctx->device);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    (void)hipDeviceSynchronize();
    (void)hipFree(p->d_expand);
    (void)hipFree(p->d_gemm);
    delete p;
    return ok();
}

qsim_status qsim_unitary_chain_batched(qsim_ctx* ctx, const qsim_circuit_desc* circuits, int count, int prec,
                                       void* d_ws, size_t ws_bytes, void* stream) {
    qsim_batch_plan* p = nullptr;
    qsim_status s = qsim_batch_plan_create(ctx, circuits, count, prec, d_ws, ws_bytes, 0, &p);
    if (s != QSIM_OK) return s;
    s = qsim_batch_plan_launch(p, stream);
    // the job tables must outlive the kernels that read them
    if (s == QSIM_OK) {
        hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
        if (e != hipSuccess) s = device_fail("hipStreamSynchronize", e);
    }
    qsim_status d = qsim_batch_plan_destroy(p);
    return s != QSIM_OK ? s : d;
}

// Tile autotuner: for each qubit count, time grouped launches of identical
// products with 64 x 64 and 128 x 128 tiles (enough copies to give every CU
// work) and keep the faster per unit of work.
qsim_status qsim_autotune(qsim_ctx* ctx, int prec, int n_lo, int n_hi, double* ms_out) {
    if (!valid_prec(prec)) return fail(QSIM_E_INVALID, "unknown precision %d", prec);
    if (n_lo < 7) n_lo = 7;  // below 7 qubits a 128-wide tile does not fit: nothing to choose
    if (n_hi > 13) return fail(QSIM_E_RANGE, "autotuning goes up to 13 qubits");
    if (n_lo > n_hi) return fail(QSIM_E_RANGE, "empty qubit range");
    qsim_status s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    const bool split = is_split(prec);
    const int cus = device_cus(ctx->device);
    const int grid = grouped_gemm_grid(prec, cus);
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int n = n_lo; n <= n_hi && e == hipSuccess; ++n) {
        const int copies = std::max(1, (2 * grid) / tiles_of(n, 128));
        const size_t mb = align256(split ? op_bytes(n, prec) : mat_bytes(n));
        void* buf = nullptr;
        GemmJob* dj = nullptr;
        e = hipMalloc(&buf, 3 * mb * copies);
        if (e == hipSuccess) {
            // float32: values in [2^-7, 2^-6); bf16 / fp16 halves: the same range in their own format
            const int elem = fmt_elem(format_of(prec));
            const uint32_t one = elem == FMT_F32 ? 0x3c000000u : elem == FMT_BF16 ? 0x3c003c00u : 0x20002000u;
            const uint32_t mant = elem == FMT_F32 ? 0x007fffffu : elem == FMT_BF16 ? 0x007f007fu : 0x03ff03ffu;
            const size_t words = 3 * mb * copies / 4;
            hipLaunchKernelGGL(tune_fill_kernel, dim3(std::min<size_t>((words + 255) / 256, 8192)), dim3(256), 0, st,
                               static_cast<uint32_t*>(buf), words, 0x5eedu + (uint32_t)n, one, mant);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMalloc(&dj, copies * sizeof(GemmJob));
        double best = 1e30;
        int best_cfg = 128;
        const int cfgs[2] = {64, 128};
        for (int ci = 0; ci < 2 && e == hipSuccess; ++ci) {
            const int cfg = cfgs[ci];
            if (split && prec == QSIM_SPLIT_FP16 && cfg == 128) {
                if (ms_out) ms_out[(n - 7) * 2 + ci] = -1.0;  // fp16 grouped tiles are always 64 x 64
                ctx->tune.ms[TuneTable::family(prec)][n][ci] = -1.0;
                continue;
            }
            std::vector<GemmJob> jobs(copies);
            int tot = 0;
            for (int c = 0; c < copies; ++c) {
                char* b = static_cast<char*>(buf) + 3 * mb * c;
                GemmJob& J = jobs[c];
                J.X = b;
                J.Y = b + mb;
                J.D0 = b + 2 * mb;
                J.D1 = nullptr;
                J.n = n;
                J.cfg = cfg;
                J.tiles = tiles_of(n, cfg);
                J.tile_begin = tot;
                tot += J.tiles;
            }
            e = hipMemcpyAsync(dj, jobs.data(), copies * sizeof(GemmJob), hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = launch_grouped_gemm(prec, dj, copies, tot, std::min(tot, grid), st);  // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            const int reps = 3;
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_grouped_gemm(prec, dj, copies, tot, std::min(tot, grid), st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            const double per = ms / reps / copies;  // per product
            if (ms_out) ms_out[(n - 7) * 2 + ci] = per;
            if (e == hipSuccess) ctx->tune.ms[TuneTable::family(prec)][n][ci] = per;
            if (e == hipSuccess && per < best) {
                best = per;
                best_cfg = cfg;
            }
        }
        if (e == hipSuccess) ctx->tune.tile[TuneTable::family(prec)][n] = best_cfg;
        if (buf) (void)hipFree(buf);
        if (dj) (void)hipFree(dj);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (e != hipSuccess) return device_fail("autotune", e);
    ctx->tune.tuned[TuneTable::family(prec)] = true;
    return ok();
}

const char* qsim_build_id(void) { return QSIM_BUILD_ID; }

}  // extern "C"

namespace {
std::string device_key(int device) {
    hipDeviceProp_t p{};
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
    char buf[512];
    snprintf(buf, sizeof buf, "%s|%s|%d", p.name, p.gcnArchName, p.multiProcessorCount);
    for (char* c = buf; *c; ++c)
        if (*c == '"' || *c == '\\') *c = '_';
    return buf;
}

// The string value of `"key": "..."` in text, or "" if absent.
std::string json_string(const std::string& text, const char* key) {
    const std::string k = std::string("\"") + key + "\":";
    size_t at = text.find(k);
    if (at == std::string::npos) return "";
    at = text.find('"', at + k.size());
    if (at == std::string::npos) return "";
    const size_t end = text.find('"', at + 1);
    return end == std::string::npos ? "" : text.substr(at + 1, end - at - 1);
}
}  // namespace

extern "C" {

qsim_status qsim_tune_save(qsim_ctx* ctx, const char* path) {
    if (ctx == nullptr || path == nullptr) return fail(QSIM_E_INVALID, "context or path is NULL");
    FILE* f = fopen(path, "w");
    if (!f) return fail(QSIM_E_INVALID, "cannot write %s", path);
    fprintf(f, "{\n \"library\": \"libqsim\",\n \"build\": \"%s\",\n \"device\": \"%s\",\n \"tiles\": [",
            QSIM_BUILD_ID, device_key(ctx->device).c_str());
    for (int p = 0; p < kPrecisions; ++p) {
        fprintf(f, "%s\n  [", p ? "," : "");
        for (int n = 0; n <= QSIM_MAX_QUBITS; ++n) fprintf(f, "%s%d", n ? ", " : "", ctx->tune.tile[p][n]);
        fprintf(f, "]");
    }
    fprintf(f, "\n ],\n \"tuned\": [");
    for (int p = 0; p < kPrecisions; ++p) fprintf(f, "%s%d", p ? ", " : "", ctx->tune.tuned[p] ? 1 : 0);
    fprintf(f, "],\n \"ms_per_product_tile64_tile128\": [");
    for (int p = 0; p < kPrecisions; ++p) {
        fprintf(f, "%s\n  [", p ? "," : "");
        for (int n = 0; n <= QSIM_MAX_QUBITS; ++n)
            fprintf(f, "%s[%.17g, %.17g]", n ? ", " : "", ctx->tune.ms[p][n][0], ctx->tune.ms[p][n][1]);
        fprintf(f, "]");
    }
    fprintf(f, "\n ]\n}\n");
    const bool bad = ferror(f) != 0;
    fclose(f);
    return bad ? fail(QSIM_E_INVALID, "write error on %s", path) : ok();
}

qsim_status qsim_tune_load(qsim_ctx* ctx, const char* path) {
    if (ctx == nullptr || path == nullptr) return fail(QSIM_E_INVALID, "context or path is NULL");
    FILE* f = fopen(path, "r");
    if (!f) return fail(QSIM_E_INVALID, "cannot read %s", path);
    std::string text;
    char chunk[4096];
    size_t got;
    while ((got = fread(chunk, 1, sizeof chunk, f)) > 0) text.append(chunk, got);
    fclose(f);
    if (json_string(text, "library") != "libqsim") return fail(QSIM_E_INVALID, "%s is not a libqsim tile cache", path);
    if (json_string(text, "build") != QSIM_BUILD_ID)
        return fail(QSIM_E_INVALID, "%s was written by another library build", path);
    if (json_string(text, "device") != device_key(ctx->device))
        return fail(QSIM_E_INVALID, "%s was written for another device", path);
    TuneTable t = ctx->tune;
    auto numbers = [&](const char* key, std::vector<double>& out, size_t count) {
        size_t at = text.find(std::string("\"") + key + "\":");
        if (at == std::string::npos) return false;
        at = text.find('[', at);
        const char* c = text.c_str() + at;
        while (out.size() < count && *c) {
            if ((*c >= '0' && *c <= '9') || *c == '-') {
                char* end = nullptr;
                out.push_back(strtod(c, &end));
                c = end;
            } else {
                ++c;
            }
        }
        return out.size() == count;
    };
    std::vector<double> tiles, tuned, ms;
    if (!numbers("tiles", tiles, (size_t)kPrecisions * (QSIM_MAX_QUBITS + 1)) ||
        !numbers("tuned", tuned, kPrecisions) ||
        !numbers("ms_per_product_tile64_tile128", ms, (size_t)kPrecisions * (QSIM_MAX_QUBITS + 1) * 2))
        return fail(QSIM_E_INVALID, "%s: malformed tile cache", path);
    for (int p = 0; p < kPrecisions; ++p) {
        for (int n = 0; n <= QSIM_MAX_QUBITS; ++n) {
            const int tile = (int)tiles[p * (QSIM_MAX_QUBITS + 1) + n];
            const bool okv = (n <= 5 && tile == 0) || (n == 6 && tile == 64) ||
                             (n >= 7 && (tile == 64 || (tile == 128 && p != QSIM_SPLIT_FP16)));
            if (!okv) return fail(QSIM_E_INVALID, "%s: tile %d for precision %d, n = %d is not valid", path, tile, p, n);
            t.tile[p][n] = tile;
            t.ms[p][n][0] = ms[(p * (QSIM_MAX_QUBITS + 1) + n) * 2];
            t.ms[p][n][1] = ms[(p * (QSIM_MAX_QUBITS + 1) + n) * 2 + 1];
        }
        t.tuned[p] = tuned[p] != 0.0;
    }
    ctx->tune = t;
    return ok();
}

qsim_status qsim_tune_ms(qsim_ctx* ctx, int prec, double* ms_out) {
    if (ctx == nullptr || ms_out == nullptr) return fail(QSIM_E_INVALID, "context or output is NULL");
    if (!valid_prec(prec)) return fail(QSIM_E_INVALID, "unknown precision %d", prec);
    for (int n = 0; n <= QSIM_MAX_QUBITS; ++n) {
        ms_out[2 * n] = ctx->tune.ms[prec][n][0];
        ms_out[2 * n + 1] = ctx->tune.ms[prec][n][1];
    }
    return ok();
}

qsim_status qsim_tune_get(qsim_ctx* ctx, int prec, int* tiles_out) {
    if (ctx == nullptr || tiles_out == nullptr) return fail(QSIM_E_INVALID, "context or output is NULL");
    if (!valid_prec(prec)) return fail(QSIM_E_INVALID, "unknown precision %d", prec);
    for (int n = 0; n <= QSIM_MAX_QUBITS; ++n) tiles_out[n] = ctx->tune.get(prec, n);
    return ok();
}

qsim_status qsim_tune_set(qsim_ctx* ctx, int prec, int n_qubits, int tile) {
    if (ctx == nullptr) return fail(QSIM_E_INVALID, "context is NULL");
    if (!valid_prec(prec)) return fail(QSIM_E_INVALID, "unknown precision %d", prec);
    if (n_qubits < 7 || n_qubits > QSIM_MAX_QUBITS) return fail(QSIM_E_RANGE, "tile choice exists for n in 7..16");
    if (tile != 64 && tile != 128) return fail(QSIM_E_INVALID, "tile must be 64 or 128");
    if (prec == QSIM_SPLIT_FP16 && tile != 64) return fail(QSIM_E_INVALID, "split fp16 products use 64-wide tiles");
    ctx->tune.tile[TuneTable::family(prec)][n_qubits] = tile;
    return ok();
}

}  // extern "C"
