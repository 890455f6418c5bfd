// Serving engine of libqsim (engine.hip): continuous batching of submitted
// circuits over the grouped kernels, admission by device-arena footprint.
#pragma once

#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host.h"

namespace qsim {

class Arena;

class Engine {
  public:
    Engine(qsim_ctx* ctx, const qsim_serve_config& cfg);
    ~Engine();  // serves every admitted request to completion, cancels the rest
    qsim_status init();
    qsim_status submit(const qsim_request& r, uint64_t* id_out);
    qsim_status poll(uint64_t id, qsim_result* out);
    void stats(qsim_serve_stats* out);

  private:
    struct Req;
    struct Inflight;
    size_t footprint(int n, const qsim_request& r) const;
    void admit_locked();
    void fail_all_locked(hipError_t err);
    hipError_t iterate(std::deque<Inflight>& inflight);
    hipError_t serve_fifo_one(Req* q);
    // Scheduling key (smaller runs first): remaining work, less the aging credit
    // under QSIM_POLICY_AGED.
    double priority(const Req* q, uint64_t now) const;
    hipError_t finish_launches(Req* q);
    void complete(Inflight& f, hipError_t err);
    hipEvent_t event();
    void loop();

    qsim_ctx* ctx_;
    qsim_serve_config cfg_;
    hipStream_t stream_ = nullptr;
    ExpandJob* h_expand_[2] = {nullptr, nullptr};
    GemmJob* h_gemm_[2] = {nullptr, nullptr};
    ExpandJob* d_expand_[2] = {nullptr, nullptr};
    GemmJob* d_gemm_[2] = {nullptr, nullptr};
    double* d_results_ = nullptr;  // 4 doubles per slot: norm2, probe max, probe l2, pad
    double* h_results_ = nullptr;
    double* d_probe_ = nullptr;
    double* d_drift_part_ = nullptr;  // partial sums of the full drift check (its own: the context's are the caller's)
    int nslots_ = 0;
    int grid_expand_ = 0, grid_gemm_ = 0;
    int table_ = 0;
    std::vector<hipEvent_t> event_pool_;

    std::mutex mu_;
    std::condition_variable cv_;
    std::thread thread_;
    bool stop_ = false;
    hipError_t dead_ = hipSuccess;
    uint64_t next_id_ = 0;
    std::deque<Req*> queue_;
    std::vector<Req*> active_;
    std::vector<int> free_slots_;
    std::unordered_map<uint64_t, Req*> reqs_;
    std::unique_ptr<Arena> arena_;
    qsim_serve_stats stats_{};
};

}  // namespace qsim
