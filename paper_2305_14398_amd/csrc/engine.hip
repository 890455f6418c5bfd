// Serving engine: requests (circuits) arrive with qsim_submit and are served
// by a host thread per context on its own HIP stream.
//
// Continuous mode: a request is admitted (strict arrival order) once the
// caller's device arena has room for its footprint (chain workspace, plus U if
// the caller does not want it back) and a slot is free.  Every engine
// iteration advances every admitted request by one step of the unitary method
// (Section 5.3, stages 4-5: expand step j, take product j) in one grouped
// expansion launch and one grouped product launch; a request whose chain is
// complete also gets stage 6 (the state product with the float64 norm) and the
// float64 probe drift check, and its results are copied back.  New requests
// join at the next iteration boundary, so requests of every size overlap on
// the device.  Two iterations are kept in flight: the host builds iteration
// i+1 while the device runs iteration i.
//
// FIFO mode is the plain baseline: one request at a time through the
// single-circuit path (qsim_unitary_chain's kernels), no grouping.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "chain_jobs.h"
#include "engine.h"

namespace qsim {

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// First-fit allocator over [0, size) with coalescing frees (offsets only).
class Arena {
  public:
    explicit Arena(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t& off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                const size_t base = it->first + bytes;
                free_.erase(it);
                if (rest) free_[base] = rest;
                used_ += bytes;
                if (used_ > high_) high_ = used_;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t high_water() const { return high_; }

  private:
    size_t size_;
    size_t used_ = 0, high_ = 0;
    std::map<size_t, size_t> free_;
};

struct Engine::Req {
    uint64_t id = 0;
    int n = 0;
    std::vector<qsim_gate> gates;
    std::vector<int32_t> off;
    void* d_psi = nullptr;
    const void* d_psi0 = nullptr;
    void* d_U = nullptr;
    uint32_t flags = 0;
    size_t foot = 0, arena_off = 0;
    int slot = -1;
    int next_j = 0;
    double step_work = 0.0;  // 8 N^3: one chain product
    ChainCursor cc;
    double remaining() const { return step_work * (double)(std::max<int>((int)off.size() - 1, 1) - next_j); }
    qsim_result res{};
};

struct Engine::Inflight {
    hipEvent_t ev = nullptr;
    int table = 0;
    std::vector<Req*> finishing;
};

Engine::Engine(qsim_ctx* ctx, const qsim_serve_config& cfg) : ctx_(ctx), cfg_(cfg) {}

size_t Engine::footprint(int n, const qsim_request& r) const {
    const size_t mb = a256(mat_bytes(n));
    const size_t ws = is_split(cfg_.prec) ? 3 * a256(op_bytes(n, cfg_.prec)) : 2 * mb;
    return ws + (r.d_U ? 0 : mb);
}

qsim_status Engine::init() {
    DeviceGuard g(ctx_->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    const int cap = cfg_.max_active;
    nslots_ = 3 * cap;
    hipError_t e = hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking);
    for (int t = 0; t < 2 && e == hipSuccess; ++t) {
        e = hipHostMalloc(&h_expand_[t], cap * sizeof(ExpandJob), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(&h_gemm_[t], cap * sizeof(GemmJob), hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(&d_expand_[t], cap * sizeof(ExpandJob));
        if (e == hipSuccess) e = hipMalloc(&d_gemm_[t], cap * sizeof(GemmJob));
    }
    if (e == hipSuccess) e = hipMalloc(&d_results_, nslots_ * 4 * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc(&h_results_, nslots_ * 4 * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(&d_probe_, kProbeScratchDoubles * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&d_drift_part_, 2 * kDriftMaxPartials * sizeof(double));
    if (e != hipSuccess) return device_fail("serving engine setup", e);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx_->device) != hipSuccess || cus <= 0)
        cus = 256;
    grid_expand_ = 8 * cus;
    grid_gemm_ = grouped_gemm_grid(cfg_.prec, cus);
    arena_.reset(new Arena(cfg_.arena_bytes));
    for (int s = nslots_ - 1; s >= 0; --s) free_slots_.push_back(s);
    thread_ = std::thread([this] { loop(); });
    return ok();
}

Engine::~Engine() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_.notify_all();
    if (thread_.joinable()) thread_.join();
    DeviceGuard g(ctx_->device);
    if (stream_) (void)hipStreamSynchronize(stream_);
    for (int t = 0; t < 2; ++t) {
        if (h_expand_[t]) (void)hipHostFree(h_expand_[t]);
        if (h_gemm_[t]) (void)hipHostFree(h_gemm_[t]);
        if (d_expand_[t]) (void)hipFree(d_expand_[t]);
        if (d_gemm_[t]) (void)hipFree(d_gemm_[t]);
    }
    if (d_results_) (void)hipFree(d_results_);
    if (h_results_) (void)hipHostFree(h_results_);
    if (d_probe_) (void)hipFree(d_probe_);
    if (d_drift_part_) (void)hipFree(d_drift_part_);
    for (hipEvent_t ev : event_pool_) (void)hipEventDestroy(ev);
    if (stream_) (void)hipStreamDestroy(stream_);
    for (auto& kv : reqs_) delete kv.second;
}

qsim_status Engine::submit(const qsim_request& r, uint64_t* id_out) {
    if (!valid_n(r.n_qubits)) return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", r.n_qubits, QSIM_MAX_QUBITS);
    if (r.reserved != 0 || (r.flags & ~(QSIM_REQ_DRIFT_PROBE | QSIM_REQ_DRIFT_FULL)))
        return fail(QSIM_E_INVALID, "unknown request flags");
    if ((r.flags & QSIM_REQ_DRIFT_PROBE) && (r.flags & QSIM_REQ_DRIFT_FULL))
        return fail(QSIM_E_INVALID, "request flags: the probe and the full drift check are exclusive");
    if (r.d_psi == nullptr || !aligned(r.d_psi)) return fail(QSIM_E_INVALID, "d_psi is NULL or not 256-byte aligned");
    if ((r.d_psi0 && !aligned(r.d_psi0)) || (r.d_U && !aligned(r.d_U)))
        return fail(QSIM_E_INVALID, "d_psi0 / d_U not 256-byte aligned");
    qsim_status s = check_gates(r.n_qubits, r.gates, r.n_gates);
    if (s != QSIM_OK) return s;
    std::unique_ptr<Req> q(new Req);
    q->n = r.n_qubits;
    q->gates.assign(r.gates, r.gates + r.n_gates);
    pack(q->gates.data(), r.n_gates, q->off);
    DevStep st;
    for (size_t j = 0; j + 1 < q->off.size(); ++j) {
        s = make_step(q->n, q->gates.data() + q->off[j], q->off[j + 1] - q->off[j], st);
        if (s != QSIM_OK) return s;
    }
    q->d_psi = r.d_psi;
    q->d_psi0 = r.d_psi0;
    q->d_U = r.d_U;
    q->flags = r.flags;
    q->foot = footprint(q->n, r);
    q->step_work = 8.0 * (double)(1ll << (3 * q->n));
    if (q->foot > cfg_.arena_bytes)
        return fail(QSIM_E_OOM, "request needs %zu arena bytes, the arena has %zu", q->foot, cfg_.arena_bytes);
    q->res.status = QSIM_PENDING;
    q->res.n_steps = (int)q->off.size() - 1;
    q->res.norm2 = q->res.drift_max = q->res.drift_l2 = -1.0;
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (dead_ != hipSuccess) return device_fail("serving engine stopped after a device error", dead_);
        if (stop_) return fail(QSIM_E_INVALID, "serving engine is stopping");
        if ((int)queue_.size() >= cfg_.queue_capacity) return fail(QSIM_E_FULL, "submit queue full (%d)", cfg_.queue_capacity);
        q->id = ++next_id_;
        q->res.t_submit_ns = now_ns();
        *id_out = q->id;
        reqs_[q->id] = q.get();
        queue_.push_back(q.release());
    }
    cv_.notify_all();
    return ok();
}

qsim_status Engine::poll(uint64_t id, qsim_result* out) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(id);
    if (it == reqs_.end()) return fail(QSIM_E_UNKNOWN_ID, "no request %llu", (unsigned long long)id);
    Req* q = it->second;
    *out = q->res;
    if (q->res.status == QSIM_PENDING) return QSIM_PENDING;
    reqs_.erase(it);
    delete q;
    return ok();
}

void Engine::stats(qsim_serve_stats* out) {
    std::lock_guard<std::mutex> lk(mu_);
    *out = stats_;
    out->arena_high_water = arena_ ? arena_->high_water() : 0;
}

hipEvent_t Engine::event() {
    if (!event_pool_.empty()) {
        hipEvent_t e = event_pool_.back();
        event_pool_.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
    return e;
}

double Engine::priority(const Req* q, uint64_t now) const {
    double k = q->remaining();
    if (cfg_.policy == QSIM_POLICY_AGED && now > q->res.t_submit_ns)
        k -= cfg_.aging_tflop_per_s * 1e12 * (double)(now - q->res.t_submit_ns) * 1e-9;
    return k;
}

// Caller holds mu_.  Moves queued requests to the active set while they fit:
// queue heads in arrival order, or the least estimated work first.
void Engine::admit_locked() {
    const bool shortest =
        (cfg_.policy == QSIM_POLICY_SHORTEST || cfg_.policy == QSIM_POLICY_AGED) && cfg_.mode == QSIM_SERVE_CONTINUOUS;
    const uint64_t now = now_ns();
    auto key = [&](const Req* q) { return priority(q, now); };
    while (!queue_.empty() && (int)active_.size() < cfg_.max_active && !free_slots_.empty()) {
        auto pick = queue_.begin();
        size_t off = 0;
        if (shortest) {
            // the smallest request that fits; ties keep arrival order
            auto best = queue_.end();
            for (auto it = queue_.begin(); it != queue_.end(); ++it)
                if (best == queue_.end() || key(*it) < key(*best)) best = it;
            pick = best;
            if (!arena_->alloc((*pick)->foot, off)) {
                // try others in increasing work order until one fits
                std::vector<std::deque<Req*>::iterator> order;
                for (auto it = queue_.begin(); it != queue_.end(); ++it) order.push_back(it);
                std::stable_sort(order.begin(), order.end(), [&](auto a, auto b) { return key(*a) < key(*b); });
                pick = queue_.end();
                for (auto it : order)
                    if (arena_->alloc((*it)->foot, off)) {
                        pick = it;
                        break;
                    }
                if (pick == queue_.end()) break;
            }
        } else if (!arena_->alloc((*pick)->foot, off)) {
            break;  // strict arrival order: wait for room
        }
        Req* q = *pick;
        queue_.erase(pick);
        q->arena_off = off;
        q->slot = free_slots_.back();
        free_slots_.pop_back();
        q->res.t_start_ns = now_ns();
        char* base = static_cast<char*>(cfg_.d_arena) + off;
        const size_t mb = is_split(cfg_.prec) ? a256(op_bytes(q->n, cfg_.prec)) : a256(mat_bytes(q->n));
        ChainCursor& cc = q->cc;
        cc.n = q->n;
        cc.k = (int)q->off.size() - 1;
        cc.prec = cfg_.prec;
        cc.cfg = q->n <= 5 ? 0 : ctx_->tune.get(cfg_.prec, q->n);
        cc.gates = q->gates.data();
        cc.off = q->off;
        cc.S = base;
        cc.W1 = base + mb;
        cc.W2 = base + 2 * mb;
        cc.U = q->d_U ? q->d_U : base + (is_split(cfg_.prec) ? 3 : 2) * mb;
        active_.push_back(q);
        stats_.admitted += 1;
        if ((int64_t)active_.size() > stats_.peak_active) stats_.peak_active = (int64_t)active_.size();
    }
}

// Stage 6 and the drift check (probe or full) for a finished chain, then the copy of its results.
hipError_t Engine::finish_launches(Req* q) {
    double* dres = d_results_ + 4 * q->slot;
    hipError_t e = launch_apply_state(q->n, static_cast<const float*>(q->cc.U), static_cast<const float*>(q->d_psi0),
                                      static_cast<float*>(q->d_psi), nullptr, dres, stream_);
    if (e == hipSuccess && (q->flags & QSIM_REQ_DRIFT_PROBE))
        e = launch_drift_probe(q->n, static_cast<const float*>(q->cc.U), d_probe_, dres + 1, stream_);
    if (e == hipSuccess && (q->flags & QSIM_REQ_DRIFT_FULL))
        e = launch_drift(q->n, static_cast<const float*>(q->cc.U), d_drift_part_, kDriftMaxPartials, dres + 1, stream_);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h_results_ + 4 * q->slot, dres, 4 * sizeof(double), hipMemcpyDeviceToHost, stream_);
    return e;
}

void Engine::complete(Inflight& f, hipError_t err) {
    const uint64_t t = now_ns();
    std::lock_guard<std::mutex> lk(mu_);
    for (Req* q : f.finishing) {
        if (err == hipSuccess) {
            const double* r = h_results_ + 4 * q->slot;
            q->res.norm2 = r[0];
            if (q->flags & (QSIM_REQ_DRIFT_PROBE | QSIM_REQ_DRIFT_FULL)) {
                q->res.drift_max = r[1];
                q->res.drift_l2 = r[2];
            }
            q->res.status = QSIM_OK;
        } else {
            q->res.status = QSIM_E_DEVICE;
        }
        q->res.t_done_ns = t;
        arena_->release(q->arena_off, q->foot);
        free_slots_.push_back(q->slot);
        stats_.completed += 1;
    }
    event_pool_.push_back(f.ev);
}

void Engine::fail_all_locked(hipError_t err) {
    dead_ = err;
    const uint64_t t = now_ns();
    for (Req* q : active_) {
        q->res.status = QSIM_E_DEVICE;
        q->res.t_done_ns = t;
    }
    active_.clear();
    for (Req* q : queue_) {
        q->res.status = QSIM_E_DEVICE;
        q->res.t_done_ns = t;
    }
    queue_.clear();
}

hipError_t Engine::iterate(std::deque<Inflight>& inflight) {
    // Reuse of a job-table slot requires the iteration that used it to be done.
    if (inflight.size() >= 2) {
        Inflight f = std::move(inflight.front());
        inflight.pop_front();
        hipError_t e = hipEventSynchronize(f.ev);
        complete(f, e);
        if (e != hipSuccess) return e;
    }
    const int t = table_++ & 1;
    std::vector<Req*> work;
    {
        std::lock_guard<std::mutex> lk(mu_);
        work = active_;
    }
    if (cfg_.policy == QSIM_POLICY_SHORTEST || cfg_.policy == QSIM_POLICY_AGED) {
        // least remaining (aged) work first, up to the iteration budget (at least one request)
        const uint64_t now = now_ns();
        std::stable_sort(work.begin(), work.end(),
                         [&](const Req* a, const Req* b) { return priority(a, now) < priority(b, now); });
        const double budget = cfg_.iter_budget_tflop * 1e12;
        double used = 0.0;
        size_t keep = 0;
        while (keep < work.size() && (keep == 0 || used + work[keep]->step_work <= budget)) used += work[keep++]->step_work;
        work.resize(keep);
    }
    // largest circuits first: the persistent grid then ends on small tiles
    std::stable_sort(work.begin(), work.end(), [](const Req* a, const Req* b) { return a->n > b->n; });
    int ne = 0, ng = 0, te = 0, tg = 0;
    Inflight f;
    f.table = t;
    for (Req* q : work) {
        ExpandJob& E = h_expand_[t][ne];
        GemmJob G;
        bool has_gemm = false;
        (void)q->cc.emit(q->next_j, E, G, has_gemm);  // every step was validated at submit
        E.block_begin = te;
        te += E.blocks;
        ++ne;
        if (has_gemm) {
            G.tile_begin = tg;
            tg += G.tiles;
            h_gemm_[t][ng++] = G;
        }
        q->next_j += 1;
        if (q->next_j >= std::max(q->cc.k, 1)) f.finishing.push_back(q);
    }
    hipError_t e = hipMemcpyAsync(d_expand_[t], h_expand_[t], ne * sizeof(ExpandJob), hipMemcpyHostToDevice, stream_);
    if (e == hipSuccess && ng)
        e = hipMemcpyAsync(d_gemm_[t], h_gemm_[t], ng * sizeof(GemmJob), hipMemcpyHostToDevice, stream_);
    if (e == hipSuccess) e = launch_grouped_expand(d_expand_[t], ne, te, std::min(te, grid_expand_), stream_);
    if (e == hipSuccess && ng) e = launch_grouped_gemm(cfg_.prec, d_gemm_[t], ng, tg, std::min(tg, grid_gemm_), stream_);
    for (Req* q : f.finishing)
        if (e == hipSuccess) e = finish_launches(q);
    f.ev = event();
    if (e == hipSuccess) e = hipEventRecord(f.ev, stream_);
    {
        std::lock_guard<std::mutex> lk(mu_);
        for (Req* q : f.finishing) active_.erase(std::find(active_.begin(), active_.end(), q));
        stats_.iterations += 1;
        stats_.grouped_launches += 1 + (ng ? 1 : 0);
    }
    inflight.push_back(std::move(f));
    return e;
}

hipError_t Engine::serve_fifo_one(Req* q) {
    // the plain path: qsim_unitary_chain's kernels on the request's workspace
    char* base = static_cast<char*>(cfg_.d_arena) + q->arena_off;
    qsim_status s = chain_impl(q->n, q->gates.data(), (int)q->gates.size(), q->off.data(), (int)q->off.size() - 1,
                               cfg_.prec, q->cc.U, base, stream_, nullptr, ctx_->tune);
    if (s != QSIM_OK) return hipErrorLaunchFailure;
    hipError_t e = finish_launches(q);
    if (e == hipSuccess) e = hipStreamSynchronize(stream_);
    Inflight f;
    f.ev = event();
    f.finishing.push_back(q);
    {
        std::lock_guard<std::mutex> lk(mu_);
        active_.erase(std::find(active_.begin(), active_.end(), q));
        stats_.iterations += 1;
    }
    complete(f, e);
    return e;
}

void Engine::loop() {
    (void)hipSetDevice(ctx_->device);
    std::deque<Inflight> inflight;
    for (;;) {
        std::unique_lock<std::mutex> lk(mu_);
        if (dead_ == hipSuccess) admit_locked();
        const bool idle = active_.empty();
        if (idle && inflight.empty()) {
            if (stop_ || dead_ != hipSuccess) {
                const uint64_t t = now_ns();
                for (Req* q : queue_) {  // requests never admitted
                    q->res.status = QSIM_E_CANCELLED;
                    q->res.t_done_ns = t;
                }
                queue_.clear();
                break;
            }
            cv_.wait_for(lk, std::chrono::milliseconds(20));
            continue;
        }
        lk.unlock();
        hipError_t e = hipSuccess;
        if (idle) {  // drain the oldest in-flight iteration
            Inflight f = std::move(inflight.front());
            inflight.pop_front();
            e = hipEventSynchronize(f.ev);
            complete(f, e);
        } else if (cfg_.mode == QSIM_SERVE_FIFO) {
            Req* q;
            {
                std::lock_guard<std::mutex> g(mu_);
                q = active_.front();
            }
            e = serve_fifo_one(q);
        } else {
            e = iterate(inflight);
        }
        if (e != hipSuccess) {
            while (!inflight.empty()) {
                Inflight f = std::move(inflight.front());
                inflight.pop_front();
                (void)hipEventSynchronize(f.ev);
                complete(f, e);
            }
            std::lock_guard<std::mutex> g(mu_);
            fail_all_locked(e);
        }
    }
}

}  // namespace qsim

using namespace qsim;

extern "C" {

qsim_status qsim_serve_start(qsim_ctx* ctx, const qsim_serve_config* cfg) {
    if (cfg == nullptr) return fail(QSIM_E_INVALID, "config is NULL");
    if (!valid_prec(cfg->prec)) return fail(QSIM_E_INVALID, "unknown precision %d", cfg->prec);
    if (cfg->mode != QSIM_SERVE_CONTINUOUS && cfg->mode != QSIM_SERVE_FIFO) return fail(QSIM_E_INVALID, "unknown mode");
    if (cfg->max_active < 1 || cfg->max_active > 4096) return fail(QSIM_E_RANGE, "max_active must be 1..4096");
    if (cfg->queue_capacity < 1) return fail(QSIM_E_RANGE, "queue_capacity must be >= 1");
    if (cfg->d_arena == nullptr || !aligned(cfg->d_arena) || cfg->arena_bytes < 256)
        return fail(QSIM_E_INVALID, "arena is NULL, unaligned or empty");
    if (cfg->policy != QSIM_POLICY_ARRIVAL && cfg->policy != QSIM_POLICY_SHORTEST && cfg->policy != QSIM_POLICY_AGED)
        return fail(QSIM_E_INVALID, "unknown policy %d", cfg->policy);
    if (cfg->reserved != 0) return fail(QSIM_E_INVALID, "reserved field must be 0");
    if (cfg->policy != QSIM_POLICY_ARRIVAL && !(cfg->iter_budget_tflop > 0.0))
        return fail(QSIM_E_INVALID, "iter_budget_tflop must be positive");
    if (cfg->policy == QSIM_POLICY_AGED && !(cfg->aging_tflop_per_s > 0.0))
        return fail(QSIM_E_INVALID, "aging_tflop_per_s must be positive");
    qsim_status s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    if (ctx->engine) return fail(QSIM_E_INVALID, "a serving engine is already running on this context");
    qsim_serve_config c = *cfg;
    if (c.mode == QSIM_SERVE_FIFO) c.max_active = 1;
    Engine* e = new Engine(ctx, c);
    s = e->init();
    if (s != QSIM_OK) {
        delete e;
        return s;
    }
    ctx->engine = e;
    return ok();
}

qsim_status qsim_serve_stop(qsim_ctx* ctx) {
    if (ctx == nullptr) return fail(QSIM_E_INVALID, "context is NULL");
    delete ctx->engine;  // finishes admitted work, cancels the rest
    ctx->engine = nullptr;
    return ok();
}

qsim_status qsim_submit(qsim_ctx* ctx, const qsim_request* req, uint64_t* id_out) {
    if (ctx == nullptr || req == nullptr || id_out == nullptr) return fail(QSIM_E_INVALID, "NULL argument");
    if (ctx->engine == nullptr) return fail(QSIM_E_INVALID, "no serving engine on this context (qsim_serve_start)");
    return ctx->engine->submit(*req, id_out);
}

qsim_status qsim_poll(qsim_ctx* ctx, uint64_t id, qsim_result* out) {
    if (ctx == nullptr || out == nullptr) return fail(QSIM_E_INVALID, "NULL argument");
    if (ctx->engine == nullptr) return fail(QSIM_E_INVALID, "no serving engine on this context");
    return ctx->engine->poll(id, out);
}

qsim_status qsim_serve_get_stats(qsim_ctx* ctx, qsim_serve_stats* out) {
    if (ctx == nullptr || out == nullptr) return fail(QSIM_E_INVALID, "NULL argument");
    if (ctx->engine == nullptr) return fail(QSIM_E_INVALID, "no serving engine on this context");
    ctx->engine->stats(out);
    return ok();
}

}  // extern "C"
