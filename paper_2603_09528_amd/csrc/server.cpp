// Serving loop: continuous batching of solve requests on one GPU.
//
// A worker thread admits queued requests into free slots (one HIP stream
// each, default priority) when their workspace fits in the HBM budget (a
// first-fit arena carved from one allocation), groups the requests admitted
// together into one multi-problem work list (one launch per stage for the
// whole group), and detects completion with an event per slot.  Slots run
// concurrently, so work of requests that arrive while others are on the GPU
// overlaps with them.  Eigenbases stay device-resident in the plan cache.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>

#include "multi.h"

namespace tpt {

double now_seconds() {
    using namespace std::chrono;
    static const steady_clock::time_point t0 = steady_clock::now();
    return duration<double>(steady_clock::now() - t0).count();
}

// First-fit allocator over one device allocation.
class Arena {
   public:
    int init(size_t bytes) {
        size_ = bytes;
        if (hipMalloc(&base_, bytes) != hipSuccess) {
            (void)hipGetLastError();
            base_ = nullptr;
            return fail(TPT_ERR_OOM, "server arena of " + std::to_string(bytes) + " bytes");
        }
        free_.clear();
        free_[0] = bytes;
        return TPT_OK;
    }
    // offset or -1
    long long alloc(size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used_[off] = bytes;
                return (long long)off;
            }
        }
        return -1;
    }
    void release(long long off) {
        auto u = used_.find((size_t)off);
        if (u == used_.end()) return;
        size_t o = u->first, len = u->second;
        used_.erase(u);
        auto nx = free_.lower_bound(o);
        if (nx != free_.end() && o + len == nx->first) {
            len += nx->second;
            free_.erase(nx);
        }
        auto pv = free_.lower_bound(o);
        if (pv != free_.begin()) {
            --pv;
            if (pv->first + pv->second == o) {
                o = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[o] = len;
    }
    char* ptr(long long off) const { return (char*)base_ + off; }
    size_t size() const { return size_; }
    ~Arena() {
        if (base_) (void)hipFree(base_);
    }

   private:
    void* base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_, used_;
};

struct Request {
    unsigned long long ticket = 0;
    tpt_plan_s* plan = nullptr;
    const double* rhs = nullptr;
    double* out = nullptr;
    double t_submit = 0, t_start = 0, t_done = 0;
    int state = 0;  // 0 queued, 1 running, 2 done, < 0 error code
    size_t ws = 0;
    std::string error;
    tpt_info info{};
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    double* h_stats = nullptr;  // pinned copy of the group's per-request sums
    MultiExec exec;
    void* d_desc = nullptr;
    size_t d_desc_bytes = 0;
    std::vector<Request*> reqs;
    long long arena_off = -1;
    bool busy = false;
};

}  // namespace tpt

struct tpt_server_s {
    int device = 0;
    tpt::Arena arena;
    std::vector<std::unique_ptr<tpt::Slot>> slots;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<tpt::Request*> queue;
    std::map<unsigned long long, std::unique_ptr<tpt::Request>> reqs;
    std::thread worker;
    bool stop = false;
    unsigned long long next_ticket = 1;
    int max_group = 16;
    int running = 0;

    void loop();
    bool complete_locked();
    bool admit_locked();
};

using namespace tpt;

bool tpt_server_s::complete_locked() {
    bool any = false;
    for (auto& sp : slots) {
        Slot& s = *sp;
        if (!s.busy) continue;
        hipError_t q = hipEventQuery(s.done);
        if (q == hipErrorNotReady) continue;
        const double t = now_seconds();
        for (size_t i = 0; i < s.reqs.size(); ++i) {
            Request* r = s.reqs[i];
            r->t_done = t;
            if (q == hipSuccess) {
                r->state = 2;
                stats_to_info(r->plan, s.h_stats + i * (MultiExec::STATS_BYTES / sizeof(double)),
                              r->info.iters > 0, &r->info);
            } else {
                r->state = TPT_ERR_HIP;
                r->error = hipGetErrorString(q);
            }
        }
        s.reqs.clear();
        arena.release(s.arena_off);
        s.arena_off = -1;
        s.busy = false;
        --running;
        any = true;
    }
    return any;
}

bool tpt_server_s::admit_locked() {
    bool any = false;
    for (auto& sp : slots) {
        if (queue.empty()) break;
        Slot& s = *sp;
        if (s.busy) continue;
        // group compatible requests from the head of the queue (FIFO)
        Request* head = queue.front();
        std::vector<Request*> grp;
        size_t need = 0;
        for (Request* r : queue) {
            if ((int)grp.size() >= max_group) break;
            if (r->plan->desc.precision != head->plan->desc.precision ||
                r->plan->desc.fixed_refine != head->plan->desc.fixed_refine)
                break;
            grp.push_back(r);
        }
        // shrink the group until its workspace fits the arena right now
        long long off = -1;
        while (!grp.empty()) {
            std::vector<tpt_plan_s*> plans;
            for (Request* r : grp) plans.push_back(r->plan);
            if (s.exec.init(plans) != TPT_OK) {
                // the head itself is not servable: fail it
                if (grp.size() == 1) {
                    head->state = TPT_ERR_UNSUPPORTED;
                    head->error = tpt_last_error();
                    head->t_done = now_seconds();
                    queue.pop_front();
                    any = true;
                }
                grp.pop_back();
                continue;
            }
            need = s.exec.workspace_bytes();
            off = arena.alloc(need);
            if (off >= 0) break;
            grp.pop_back();
        }
        if (grp.empty() || off < 0) {
            if (!queue.empty() && running == 0) {
                Request* h = queue.front();
                std::vector<tpt_plan_s*> one{h->plan};
                if (s.exec.init(one) == TPT_OK && s.exec.workspace_bytes() > arena.size()) {
                    h->state = TPT_ERR_OOM;
                    h->error = "request workspace exceeds the server's HBM budget";
                    h->t_done = now_seconds();
                    queue.pop_front();
                    any = true;
                }
            }
            break;  // wait for memory to free up
        }
        for (size_t i = 0; i < grp.size(); ++i) queue.pop_front();
        std::vector<const double*> rhs;
        std::vector<double*> out;
        for (Request* r : grp) {
            rhs.push_back(r->rhs);
            out.push_back(r->out);
        }
        int rc = s.exec.build(rhs.data(), out.data(), arena.ptr(off));
        if (rc == TPT_OK && s.d_desc_bytes < s.exec.desc_bytes()) {
            if (s.d_desc) (void)hipFree(s.d_desc);
            s.d_desc = nullptr;
            s.d_desc_bytes = 0;
            if (hipMalloc(&s.d_desc, s.exec.desc_bytes()) != hipSuccess) {
                (void)hipGetLastError();
                rc = TPT_ERR_OOM;
            } else {
                s.d_desc_bytes = s.exec.desc_bytes();
            }
        }
        if (rc == TPT_OK) rc = s.exec.upload(s.d_desc, s.stream);
        const double t = now_seconds();
        if (rc == TPT_OK) rc = s.exec.enqueue(s.stream);
        if (rc == TPT_OK && hipMemcpyAsync(s.h_stats, s.exec.norms(0), grp.size() * MultiExec::STATS_BYTES,
                                           hipMemcpyDeviceToHost, s.stream) != hipSuccess)
            rc = fail(TPT_ERR_HIP, "copy of request sums");
        if (rc == TPT_OK && hipEventRecord(s.done, s.stream) != hipSuccess) rc = TPT_ERR_HIP;
        if (rc != TPT_OK) {
            const std::string msg = tpt_last_error();
            for (Request* r : grp) {
                r->state = rc;
                r->error = msg;
                r->t_start = t;
                r->t_done = now_seconds();
            }
            arena.release(off);
            any = true;
            continue;
        }
        for (Request* r : grp) {
            r->state = 1;
            r->t_start = t;
            r->info.iters = s.exec.iterations();
            r->info.null_line = r->plan->null_line;
            r->info.rel_correction = 0.0;
            r->info.rel_residual = -1.0;
            r->info.compat_defect = -1.0;
            r->info.nonfinite = -1;
        }
        s.reqs = grp;
        s.arena_off = off;
        s.busy = true;
        ++running;
        any = true;
    }
    return any;
}

void tpt_server_s::loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lock(mu);
    for (;;) {
        const bool c = complete_locked();
        const bool a = admit_locked();
        if (c || a) cv.notify_all();
        if (stop && queue.empty() && running == 0) break;
        if (!c && !a) {
            if (running > 0) {
                lock.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lock.lock();
            } else {
                cv.wait_for(lock, std::chrono::milliseconds(5));
            }
        }
    }
}

extern "C" {

int tpt_server_create(size_t budget, int max_slots, tpt_server* out) {
    if (!out || max_slots < 1 || max_slots > 64) return fail(TPT_ERR_INVALID, "bad server arguments");
    *out = nullptr;
    std::unique_ptr<tpt_server_s> s(new tpt_server_s());
    TPT_HIP(hipGetDevice(&s->device));
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        TPT_HIP(hipMemGetInfo(&fr, &tot));
        budget = fr / 4 * 3;
    }
    int rc = s->arena.init(budget);
    if (rc) return rc;
    for (int i = 0; i < max_slots; ++i) {
        auto sl = std::make_unique<Slot>();
        TPT_HIP(hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking));
        TPT_HIP(hipEventCreateWithFlags(&sl->done, hipEventDisableTiming));
        TPT_HIP(hipHostMalloc((void**)&sl->h_stats, s->max_group * MultiExec::STATS_BYTES, hipHostMallocDefault));
        s->slots.push_back(std::move(sl));
    }
    tpt_server_s* raw = s.get();
    s->worker = std::thread([raw] { raw->loop(); });
    *out = s.release();
    return TPT_OK;
}

int tpt_server_submit(tpt_server s, tpt_plan plan, const double* rhs, double* out, unsigned long long* ticket) {
    if (!s || !plan || !rhs || !out || !ticket) return fail(TPT_ERR_INVALID, "NULL argument");
    if (plan->host_only) return fail(TPT_ERR_INVALID, "host-only plan");
    if (plan->desc.nrhs != 1) return fail(TPT_ERR_UNSUPPORTED, "server requests need nrhs = 1");
    if (plan->desc.precision != TPT_FP64 && plan->desc.fixed_refine < 0)
        return fail(TPT_ERR_UNSUPPORTED, "server requests with mixed precision need fixed_refine >= 0");
    auto r = std::make_unique<Request>();
    r->plan = plan;
    r->rhs = rhs;
    r->out = out;
    r->t_submit = now_seconds();
    {
        std::lock_guard<std::mutex> lock(s->mu);
        if (s->stop) return fail(TPT_ERR_INVALID, "server is stopping");
        r->ticket = s->next_ticket++;
        *ticket = r->ticket;
        s->queue.push_back(r.get());
        s->reqs[r->ticket] = std::move(r);
    }
    s->cv.notify_all();
    return TPT_OK;
}

int tpt_server_poll(tpt_server s, unsigned long long ticket, tpt_info* info, double* t_submit, double* t_start,
                    double* t_done) {
    if (!s) return fail(TPT_ERR_INVALID, "NULL server");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(TPT_ERR_INVALID, "unknown ticket");
    Request* r = it->second.get();
    if (r->state == 0 || r->state == 1) return TPT_PENDING;
    if (info) *info = r->info;
    if (t_submit) *t_submit = r->t_submit;
    if (t_start) *t_start = r->t_start;
    if (t_done) *t_done = r->t_done;
    const int st = r->state;
    const std::string err = r->error;
    s->reqs.erase(it);
    if (st < 0) return fail(st, "request failed: " + err);
    return TPT_OK;
}

int tpt_server_drain(tpt_server s) {
    if (!s) return fail(TPT_ERR_INVALID, "NULL server");
    std::unique_lock<std::mutex> lock(s->mu);
    s->cv.wait(lock, [s] { return s->queue.empty() && s->running == 0; });
    return TPT_OK;
}

int tpt_server_destroy(tpt_server s) {
    if (!s) return TPT_OK;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto& sl : s->slots) {
        if (sl->stream) (void)hipStreamSynchronize(sl->stream);
        if (sl->d_desc) (void)hipFree(sl->d_desc);
        if (sl->done) (void)hipEventDestroy(sl->done);
        if (sl->h_stats) (void)hipHostFree(sl->h_stats);
        if (sl->stream) (void)hipStreamDestroy(sl->stream);
    }
    delete s;
    return TPT_OK;
}

}  // extern "C"
