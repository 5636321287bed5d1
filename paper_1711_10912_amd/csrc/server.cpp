// Native request server: continuous batching of TTV / TTM / TTT requests on
// one GPU (the ABI is declared in include/tlib.h, tlib_server_*).
//
// A scheduler thread owns S HIP streams ("slots").  Requests are admitted in
// arrival order while a slot is free and their output fits in the output
// arena (the HBM budget for results), so requests that arrive while others
// run start as soon as memory and slots free up.  Consecutive small TTV/TTM/TTT
// requests are fused into one grouped launch: the batch is planned into a
// pinned host table, copied to the slot's device table and run by a graph
// captured once per slot.  Every other request runs through the regular entry
// points on its slot's stream.  A request's kernel depends only on the request,
// never on the mix, so its result is the same alone and batched.  Completion
// times come from events referenced to the host clock.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace {

using clk = std::chrono::steady_clock;

double now_s() { return std::chrono::duration<double>(clk::now().time_since_epoch()).count(); }

struct Desc {
    tlib_tensor t{};
    int64_t n[TLIB_MAX_ORDER] = {};
    int64_t w[TLIB_MAX_ORDER] = {};
    void set(const tlib_tensor* src) {
        t = *src;
        for (int r = 0; r < src->order; ++r) {
            n[r] = src->extents[r];
            if (src->strides) w[r] = src->strides[r];
        }
        if (!src->strides) tlib_strides_from_layout(src->order, src->extents, src->layout, w);
        t.extents = n;
        t.strides = w;
        t.layout = nullptr;
    }
};

struct Job {
    int64_t rid = 0;
    int op = 0;  // 0 ttv, 1 ttm, 2 ttt
    int mode = 0, q = 0;
    int32_t phi[TLIB_MAX_ORDER] = {}, psi[TLIB_MAX_ORDER] = {};
    Desc a, b, c;
    size_t out_bytes = 0, out_off = 0;
    bool own_out = true;  // output lives in the arena
    bool grouped = false;
    double t_arrival = 0, t_done = 0;
    int err = 0;
    tlib_request request() {
        return tlib_request{op, mode, &a.t, &b.t, &c.t, q, 0, op == 2 ? phi : nullptr, op == 2 ? psi : nullptr};
    }
};

// First-fit allocator over [0, size) with 256-byte granularity.
class Arena {
  public:
    void init(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
        size_ = size;
    }
    bool alloc(size_t bytes, size_t& off) {
        bytes = (bytes + 255) & ~size_t(255);
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        if (bytes == 0) bytes = 256;
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

  private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void* tab_host = nullptr;  // pinned
    void* tab_dev = nullptr;
    hipGraphExec_t graph = nullptr;
    std::vector<Job*> jobs;  // in flight
};

}  // namespace

struct tlib_server {
    int device = 0;
    size_t budget = 0;
    int group_max = 64;
    int64_t group_macs = 1 << 21;
    int grid = 1024;
    bool keep = false;
    void* arena_ptr = nullptr;
    Arena arena;
    size_t in_flight = 0;
    std::vector<Slot> slots;
    size_t table_bytes = 0;
    hipEvent_t ref = nullptr;
    double t_ref = 0;
    std::deque<Job*> pending;
    std::vector<Job*> completed;
    std::map<int64_t, Job*> results;  // kept outputs by request id
    int64_t next_id = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::thread th;
    bool stop = false;
    std::atomic<int> busy_slots{0};
    bool dev_err = false;  // the server thread could not select its device: every job fails

    // device-clock time of a recorded event on the host timeline; a failed
    // query (an event that was never recorded) reads as the reference time
    double ev_time(hipEvent_t ev) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ref, ev) != hipSuccess) ms = 0.f;
        return t_ref + double(ms) * 1e-3;
    }

    void retire() {
        for (auto& s : slots) {
            if (s.jobs.empty()) continue;
            if (hipEventQuery(s.done) != hipSuccess) continue;
            const double t = ev_time(s.done);
            for (Job* j : s.jobs) {
                j->t_done = t;
                in_flight -= j->out_bytes;
                if (!keep) {
                    if (j->own_out) arena.release(j->out_off, j->out_bytes);
                } else {
                    results[j->rid] = j;
                }
                completed.push_back(j);
            }
            s.jobs.clear();
            --busy_slots;
        }
    }

    void place_output(Job* j) {
        if (!j->own_out) return;
        j->c.t.data = (char*)arena_ptr + j->out_off;
    }

    void launch_single(Slot& s, Job* j) {
        place_output(j);
        if (dev_err) {
            j->err = TLIB_EHIP;
            return;
        }
        void* st = (void*)s.stream;
        if (j->op == 0) j->err = tlib_ttv(&j->a.t, &j->b.t, j->mode, &j->c.t, st);
        else if (j->op == 1) j->err = tlib_ttm(&j->a.t, &j->b.t, j->mode, &j->c.t, st);
        else j->err = tlib_ttt(&j->a.t, &j->b.t, j->q, j->phi, j->psi, &j->c.t, st);
    }

    void launch_group(Slot& s, std::vector<Job*>& jobs) {
        std::vector<tlib_request> req(jobs.size());
        for (size_t i = 0; i < jobs.size(); ++i) {
            place_output(jobs[i]);
            req[i] = jobs[i]->request();
        }
        int64_t units = 0;
        int32_t bad = -1;
        int rc = tlib_batch_plan(req.data(), int32_t(req.size()), s.tab_host, table_bytes, &units, &bad);
        if (rc != TLIB_OK) {
            // run everything singly (a request the grouped kernel cannot take)
            for (Job* j : jobs) launch_single(s, j);
            return;
        }
        int err = dev_err ? TLIB_EHIP : TLIB_OK;
        if (!err && hipMemcpyAsync(s.tab_dev, s.tab_host, tlib_batch_table_bytes(int32_t(req.size())),
                                   hipMemcpyHostToDevice, s.stream) != hipSuccess)
            err = TLIB_EHIP;
        if (!err) {
            if (s.graph) err = hipGraphLaunch(s.graph, s.stream) == hipSuccess ? TLIB_OK : TLIB_EHIP;
            else err = tlib_batch_run(s.tab_dev, grid, (void*)s.stream);
        }
        if (err)
            for (Job* j : jobs) j->err = err;
    }

    bool admit() {
        Slot* slot = nullptr;
        for (auto& s : slots)
            if (s.jobs.empty()) {
                slot = &s;
                break;
            }
        if (!slot || pending.empty()) return false;
        Job* head = pending.front();
        if (head->own_out) {
            if (!arena.alloc(head->out_bytes, head->out_off)) return false;  // wait for memory
        }
        pending.pop_front();
        std::vector<Job*> jobs{head};
        in_flight += head->out_bytes;
        if (head->grouped) {
            while (!pending.empty() && int(jobs.size()) < group_max && pending.front()->grouped) {
                Job* j = pending.front();
                if (j->own_out && !arena.alloc(j->out_bytes, j->out_off)) break;
                pending.pop_front();
                in_flight += j->out_bytes;
                jobs.push_back(j);
            }
            launch_group(*slot, jobs);
        } else {
            launch_single(*slot, head);
        }
        // an event that cannot be recorded reads as complete: the slot's
        // jobs are then reported failed instead of waiting forever
        if (hipEventRecord(slot->done, slot->stream) != hipSuccess)
            for (Job* j : jobs)
                if (!j->err) j->err = TLIB_EHIP;
        slot->jobs = jobs;
        ++busy_slots;
        return true;
    }

    void loop() {
        if (hipSetDevice(device) != hipSuccess) dev_err = true;
        std::unique_lock<std::mutex> lk(mu);
        while (!stop) {
            retire();
            bool started = false;
            while (admit()) started = true;
            if (!started) {
                if (pending.empty() && busy_slots.load() == 0) {
                    cv.wait_for(lk, std::chrono::milliseconds(5));
                } else {
                    lk.unlock();
                    std::this_thread::sleep_for(std::chrono::microseconds(20));
                    lk.lock();
                }
            }
        }
    }
};

extern "C" {

tlib_server* tlib_server_create(int32_t device, size_t output_budget, int32_t slots, int32_t group_max,
                                int64_t group_macs, int32_t keep_results) {
    if (slots < 1 || slots > 32 || group_max < 1) return nullptr;
    if (hipSetDevice(device) != hipSuccess) return nullptr;
    auto* S = new tlib_server();
    S->device = device;
    S->budget = output_budget;
    S->group_max = group_max;
    S->group_macs = group_macs;
    S->keep = keep_results != 0;
    if (output_budget && hipMalloc(&S->arena_ptr, output_budget) != hipSuccess) {
        (void)hipGetLastError();
        delete S;
        return nullptr;
    }
    S->arena.init(output_budget);
    S->table_bytes = tlib_batch_table_bytes(group_max);
    S->slots.resize(slots);
    for (auto& s : S->slots) {
        // each slot's stream gets its workspace now, so that requests never
        // allocate (or fail for want of scratch) once the server runs
        bool ok = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) == hipSuccess &&
                  tlib_workspace_reserve((void*)s.stream, TLIB_WORKSPACE_DEFAULT_BYTES) == TLIB_OK &&
                  hipEventCreate(&s.done) == hipSuccess &&
                  hipHostMalloc(&s.tab_host, S->table_bytes, hipHostMallocDefault) == hipSuccess &&
                  hipMalloc(&s.tab_dev, S->table_bytes) == hipSuccess &&
                  hipMemsetAsync(s.tab_dev, 0, S->table_bytes, s.stream) == hipSuccess &&
                  hipStreamSynchronize(s.stream) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            tlib_server_destroy(S);
            return nullptr;
        }
        // capture the grouped launch once; replays read the table's current contents
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            const int rc = tlib_batch_run(s.tab_dev, S->grid, (void*)s.stream);
            if (hipStreamEndCapture(s.stream, &g) == hipSuccess && rc == TLIB_OK && g) {
                if (hipGraphInstantiate(&s.graph, g, nullptr, nullptr, 0) != hipSuccess) s.graph = nullptr;
            }
            if (g) (void)hipGraphDestroy(g);
        }
        (void)hipGetLastError();
    }
    // reference event: device time zero on the host clock
    if (hipEventCreate(&S->ref) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
        hipEventRecord(S->ref, S->slots[0].stream) != hipSuccess || hipEventSynchronize(S->ref) != hipSuccess) {
        (void)hipGetLastError();
        tlib_server_destroy(S);
        return nullptr;
    }
    S->t_ref = now_s();
    S->th = std::thread([S] { S->loop(); });
    return S;
}

int tlib_server_submit(tlib_server* S, int32_t op, const tlib_tensor* A, const tlib_tensor* B, int32_t mode,
                       int32_t q, const int32_t* phi, const int32_t* psi, const tlib_tensor* C, int64_t* rid) {
    if (!S) return TLIB_EINVAL;
    const double t = now_s();
    // every argument is checked before anything is copied from it
    const int vrc = tlib_request_check(op, A, B, mode, q, phi, psi, C);
    if (vrc != TLIB_OK) return vrc;
    Job* j = new Job();
    j->op = op;
    j->mode = mode;
    j->q = q;
    j->a.set(A);
    j->b.set(B);
    j->c.set(C);
    j->own_out = C->data == nullptr;
    if (op == 2) {
        for (int r = 0; r < A->order; ++r) j->phi[r] = phi[r];
        for (int r = 0; r < B->order; ++r) j->psi[r] = psi[r];
    }
    int64_t outs = 1, span = 0;
    for (int r = 0; r < C->order; ++r) {
        outs *= j->c.n[r];
        span += (j->c.n[r] - 1) * j->c.w[r];
    }
    const int esz = C->dtype == TLIB_F64 ? 8 : C->dtype == TLIB_F32 ? 4 : 2;
    j->out_bytes = size_t(span + 1) * size_t(esz);
    int64_t macs = outs;
    if (op == 0 || op == 1) {
        macs = outs * j->a.n[mode - 1];
    } else {
        for (int k = A->order - q; k < A->order; ++k) macs *= j->a.n[phi[k] - 1];
    }
    // grouping depends on the request alone, so it runs the same way in any mix
    if (macs <= S->group_macs) {
        const tlib_request rq = j->request();
        j->grouped = tlib_request_groupable(&rq) == 1;
    }
    j->t_arrival = t;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (j->own_out && j->out_bytes > S->budget) {
            delete j;
            return TLIB_ENOMEM;
        }
        j->rid = S->next_id++;
        S->pending.push_back(j);
    }
    S->cv.notify_one();
    if (rid) *rid = j->rid;
    return TLIB_OK;
}

int tlib_server_drain(tlib_server* S, double timeout_s) {
    if (!S) return TLIB_EINVAL;
    const double t0 = now_s();
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->pending.empty() && S->busy_slots.load() == 0) return TLIB_OK;
        }
        if (now_s() - t0 > timeout_s) return TLIB_EHIP;
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
}

int tlib_server_stats(tlib_server* S, tlib_server_stats_t* out) {
    if (!S || !out) return TLIB_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    std::vector<double> lat;
    double first = 1e300, last = -1e300;
    int64_t grouped = 0, errors = 0;
    for (Job* j : S->completed) {
        if (j->err) {
            ++errors;
            continue;
        }
        lat.push_back(j->t_done - j->t_arrival);
        first = std::min(first, j->t_arrival);
        last = std::max(last, j->t_done);
        grouped += j->grouped;
    }
    std::memset(out, 0, sizeof(*out));
    out->completed = int64_t(S->completed.size());
    out->grouped = grouped;
    out->errors = errors;
    if (lat.empty()) return TLIB_OK;
    std::sort(lat.begin(), lat.end());
    auto pick = [&](double f) { return lat[std::min(lat.size() - 1, size_t(f * double(lat.size())))]; };
    out->p50_s = pick(0.50);
    out->p99_s = pick(0.99);
    double sum = 0;
    for (double v : lat) sum += v;
    out->mean_s = sum / double(lat.size());
    out->req_per_s = last > first ? double(lat.size()) / (last - first) : 0.0;
    return TLIB_OK;
}

int tlib_server_result(tlib_server* S, int64_t rid, tlib_tensor* out, int32_t* err) {
    if (!S || !out) return TLIB_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->results.find(rid);
    if (it == S->results.end()) return TLIB_EINVAL;
    Job* j = it->second;
    *out = j->c.t;
    if (err) *err = j->err;
    return TLIB_OK;
}

void tlib_server_reset_stats(tlib_server* S) {
    if (!S) return;
    std::lock_guard<std::mutex> lk(S->mu);
    for (Job* j : S->completed)
        if (!S->keep) delete j;
    S->completed.clear();
}

void tlib_server_destroy(tlib_server* S) {
    if (!S) return;
    if (S->th.joinable()) {
        tlib_server_drain(S, 600.0);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
        }
        S->cv.notify_one();
        S->th.join();
    }
    // best-effort release: a failure here leaves nothing to recover
    for (auto& s : S->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        if (s.graph) (void)hipGraphExecDestroy(s.graph);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.tab_host) (void)hipHostFree(s.tab_host);
        if (s.tab_dev) (void)hipFree(s.tab_dev);
        if (s.stream) (void)hipStreamDestroy(s.stream);
    }
    if (S->ref) (void)hipEventDestroy(S->ref);
    if (S->arena_ptr) (void)hipFree(S->arena_ptr);
    (void)hipGetLastError();
    for (Job* j : S->completed) delete j;
    for (Job* j : S->pending) delete j;
    delete S;
}

}  // extern "C"
