// Registration serving engine of libnrr.so (C ABI in include/nrr.h).
//
// Requests (a volume pair plus selection and search parameters) arrive at any
// time.  A scheduler thread admits them in arrival order whenever a slot (a
// HIP stream) and room in the device memory arena are free -- an admitted
// request does not wait for others to finish, so requests of different sizes
// overlap on the GPU (continuous batching rather than a queue served one at
// a time).  An admitted request runs upload, selection, window statistics,
// exhaustive search and download on its slot's stream; its arena blocks are
// returned when its completion event fires.  A request that arrives while
// the head of the queue waits for memory may pass it if it fits, at most
// kMaxBypass times per waiting request (no starvation).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "nrr.h"
#include "nrr_internal.h"

namespace {

constexpr int kMaxBypass = 8;
constexpr size_t kAlign = 256;

size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over one device region; offsets in bytes.  Used by the
// scheduler thread only.
class Arena {
  public:
    void reset(size_t size) {
        free_.clear();
        free_[0] = size;
        size_ = size;
        used_ = peak_ = 0;
    }
    bool alloc(size_t n, size_t *off) {
        n = up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += n;
                peak_ = std::max(peak_, used_);
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n) {
        n = up(n);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {  // merge right
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {  // merge left
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t peak() const { return peak_; }
    size_t used() const { return used_; }

  private:
    std::map<size_t, size_t> free_;  // offset -> length
    size_t size_ = 0, used_ = 0, peak_ = 0;
};

// Device bytes of one request and the offsets of its buffers inside them.
struct Footprint {
    size_t ref, flt, sel, stats, centers, disp, ncc, conf, total;
    int64_t k;
    int32_t grid[3];
};

bool footprint(const nrr_request &r, Footprint *f) {
    int64_t k = 0;
    size_t selb = 0, statsb = 0;
    if (nrr_grid_shape(r.dims, r.block, r.stride, f->grid) != NRR_OK) return false;
    if ((int64_t)f->grid[0] * f->grid[1] * f->grid[2] >= (1ll << 31)) return false;
    if (nrr_select_count(r.dims, r.block, r.stride, r.fraction, &k) != NRR_OK) return false;
    if (nrr_select_workspace_bytes(r.dims, r.block, r.stride, &selb) != NRR_OK) return false;
    if (nrr_match_workspace_bytes(r.dtype, r.dims, r.block, &statsb) != NRR_OK) return false;
    const size_t vox = (size_t)r.dims[0] * r.dims[1] * r.dims[2];
    const size_t vb = vox * (r.dtype == NRR_U16 ? 2 : 4);
    size_t at = 0;
    f->ref = at, at += up(vb);
    f->flt = at, at += up(vb);
    f->sel = at, at += up(selb);
    f->stats = at, at += up(statsb);
    f->centers = at, at += up((size_t)std::max<int64_t>(k, 1) * 12);
    f->disp = at, at += up((size_t)std::max<int64_t>(k, 1) * 12);
    f->ncc = at, at += up((size_t)std::max<int64_t>(k, 1) * 4);
    f->conf = at, at += up((size_t)std::max<int64_t>(k, 1) * 4);
    f->total = at;
    f->k = k;
    return true;
}

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Request {
    nrr_request r;
    Footprint f;
    int64_t ticket = 0;
    int32_t state = 0;  // 0 queued, 1 running, 2 done, 3 failed
    int32_t status = NRR_OK;
    int bypassed = 0, slot = -1;
    size_t off = 0;
    hipEvent_t done = nullptr;
    Clock::time_point t_submit, t_admit, t_done;
};

}  // namespace

struct nrr_server {
    int device = 0;
    size_t budget = 0;
    char *base = nullptr;
    Arena arena;
    std::vector<hipStream_t> streams;
    std::vector<bool> slot_busy;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<std::shared_ptr<Request>> pending;
    std::vector<std::shared_ptr<Request>> running;
    std::map<int64_t, std::shared_ptr<Request>> all;
    int64_t next_ticket = 1;
    int64_t admitted = 0, completed = 0;
    int32_t max_running = 0;
    bool stop = false;
    std::thread worker;
};

namespace {

// Enqueue one request on its slot stream.
hipError_t enqueue(nrr_server *S, Request &q) {
    hipStream_t st = S->streams[q.slot];
    char *b = S->base + q.off;
    const nrr_request &r = q.r;
    const Footprint &f = q.f;
    const size_t vb = (size_t)r.dims[0] * r.dims[1] * r.dims[2] * (r.dtype == NRR_U16 ? 2 : 4);
    hipError_t e = hipMemcpyAsync(b + f.ref, r.ref, vb, hipMemcpyDefault, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b + f.flt, r.flt, vb, hipMemcpyDefault, st);
    if (e != hipSuccess) return e;
    if (f.k > 0) {
        int32_t *centers = reinterpret_cast<int32_t *>(b + f.centers);
        e = nrr::launch_select(b + f.ref, r.dtype, r.dims, r.block, r.stride, f.grid, f.k, centers,
                               b + f.sel, st);
        if (e == hipSuccess) e = nrr::launch_stats(b + f.flt, r.dtype, r.dims, r.block, b + f.stats, st);
        if (e != hipSuccess) return e;
        const nrr::StatsLayout L = nrr::stats_layout(r.dtype, r.dims, r.block);
        nrr::MatchArgs a;
        a.ref = b + f.ref;
        a.flt = b + f.flt;
        a.nx = r.dims[0];
        a.ny = r.dims[1];
        a.nz = r.dims[2];
        a.centers = centers;
        a.n = f.k;
        a.block = r.block;
        a.window = r.window;
        a.stats = b + f.stats;
        a.pairs = L.pair_off ? reinterpret_cast<const uint32_t *>(b + f.stats + L.pair_off) : nullptr;
        a.ox = L.ox;
        a.oy = L.oy;
        a.disp = reinterpret_cast<int32_t *>(b + f.disp);
        a.ncc = reinterpret_cast<float *>(b + f.ncc);
        a.conf = reinterpret_cast<float *>(b + f.conf);
        if ((e = nrr::launch_match(r.dtype, a, st)) != hipSuccess) return e;
        const size_t k = (size_t)f.k;
        if (r.centers) e = hipMemcpyAsync(r.centers, centers, k * 12, hipMemcpyDefault, st);
        if (e == hipSuccess && r.disp) e = hipMemcpyAsync(r.disp, a.disp, k * 12, hipMemcpyDefault, st);
        if (e == hipSuccess && r.ncc) e = hipMemcpyAsync(r.ncc, a.ncc, k * 4, hipMemcpyDefault, st);
        if (e == hipSuccess && r.conf) e = hipMemcpyAsync(r.conf, a.conf, k * 4, hipMemcpyDefault, st);
        if (e != hipSuccess) return e;
    }
    return hipEventRecord(q.done, st);
}

void finish(nrr_server *S, Request &q, int32_t state, int32_t status) {
    S->arena.release(q.off, q.f.total);
    S->slot_busy[q.slot] = false;
    q.state = state;
    q.status = status;
    q.t_done = Clock::now();
    ++S->completed;
}

void scheduler(nrr_server *S) {
    hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        // retire finished requests
        for (size_t i = 0; i < S->running.size();) {
            Request &q = *S->running[i];
            const hipError_t e = hipEventQuery(q.done);
            if (e == hipErrorNotReady) {
                ++i;
                continue;
            }
            finish(S, q, e == hipSuccess ? 2 : 3, e == hipSuccess ? NRR_OK : NRR_ERR_HIP);
            S->running.erase(S->running.begin() + i);
            S->cv_done.notify_all();
        }
        // admit: the oldest request that fits a free slot and the arena; a
        // request may pass an older one only while that one has been passed
        // fewer than kMaxBypass times
        int slot = -1;
        for (size_t i = 0; i < S->slot_busy.size(); ++i)
            if (!S->slot_busy[i]) {
                slot = (int)i;
                break;
            }
        bool admitted_one = false;
        if (slot >= 0) {
            for (size_t i = 0; i < S->pending.size(); ++i) {
                Request &q = *S->pending[i];
                size_t off = 0;
                if (S->arena.alloc(q.f.total, &off)) {
                    for (size_t j = 0; j < i; ++j) ++S->pending[j]->bypassed;
                    q.off = off;
                    q.slot = slot;
                    q.state = 1;
                    q.t_admit = Clock::now();
                    S->slot_busy[slot] = true;
                    ++S->admitted;
                    const hipError_t e = enqueue(S, q);
                    if (e != hipSuccess) {
                        hipGetLastError();
                        finish(S, q, 3, NRR_ERR_HIP);
                        S->cv_done.notify_all();
                    } else {
                        S->running.push_back(S->pending[i]);
                        S->max_running = std::max<int32_t>(S->max_running, (int32_t)S->running.size());
                    }
                    S->pending.erase(S->pending.begin() + i);
                    admitted_one = true;
                    break;
                }
                if (q.bypassed >= kMaxBypass) break;  // it waits; nobody passes it
            }
        }
        if (admitted_one) continue;
        if (S->stop && S->pending.empty() && S->running.empty()) break;
        // nothing to admit now: wait for a submission or poll the running work
        if (S->running.empty())
            S->cv.wait(lk, [&] { return S->stop || !S->pending.empty(); });
        else
            S->cv.wait_for(lk, std::chrono::microseconds(50));
    }
}

nrr_status check_request(const nrr_request *r, Footprint *f) {
    if (!r) return NRR_ERR_INVALID_ARG;
    if (r->dtype != NRR_U16 && r->dtype != NRR_F32) return NRR_ERR_INVALID_ARG;
    if (!r->ref || !r->flt) return NRR_ERR_INVALID_ARG;
    if (!(r->fraction > 0.0 && r->fraction <= 1.0) || r->window < 0) return NRR_ERR_INVALID_ARG;
    if (!footprint(*r, f)) return NRR_ERR_INVALID_ARG;
    if (f->k > 0 && r->capacity < f->k) return NRR_ERR_BUFFER_TOO_SMALL;
    return NRR_OK;
}

void fill_info(const Request &q, nrr_request_info *info) {
    info->state = q.state;
    info->status = q.status;
    info->k = q.f.k;
    info->device_bytes = (int64_t)q.f.total;
    const auto now = Clock::now();
    info->queued_ms = ms_between(q.t_submit, q.state >= 1 ? q.t_admit : now);
    info->run_ms = q.state >= 2 ? ms_between(q.t_admit, q.t_done)
                                : (q.state == 1 ? ms_between(q.t_admit, now) : 0.0);
    info->total_ms = ms_between(q.t_submit, q.state >= 2 ? q.t_done : now);
}

}  // namespace

extern "C" {

nrr_status nrr_request_footprint(const nrr_request *r, size_t *bytes) {
    Footprint f;
    const nrr_status s = check_request(r, &f);
    if (s != NRR_OK && s != NRR_ERR_BUFFER_TOO_SMALL) return s;
    if (bytes) *bytes = f.total;
    return NRR_OK;
}

nrr_status nrr_server_create(size_t device_bytes, int32_t slots, nrr_server **out) {
    if (!out || slots < 1 || slots > 64 || device_bytes < kAlign) return NRR_ERR_INVALID_ARG;
    *out = nullptr;
    auto S = std::make_unique<nrr_server>();
    if (hipGetDevice(&S->device) != hipSuccess) return NRR_ERR_HIP;
    S->budget = device_bytes / kAlign * kAlign;
    if (hipMalloc(reinterpret_cast<void **>(&S->base), S->budget) != hipSuccess) {
        hipGetLastError();
        return NRR_ERR_HIP;
    }
    S->arena.reset(S->budget);
    for (int i = 0; i < slots; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : S->streams) hipStreamDestroy(x);
            hipFree(S->base);
            return NRR_ERR_HIP;
        }
        S->streams.push_back(st);
    }
    S->slot_busy.assign(slots, false);
    nrr_server *raw = S.release();
    raw->worker = std::thread(scheduler, raw);
    *out = raw;
    return NRR_OK;
}

nrr_status nrr_server_submit(nrr_server *S, const nrr_request *r, int64_t *ticket) {
    if (!S || !ticket) return NRR_ERR_INVALID_ARG;
    auto q = std::make_shared<Request>();
    const nrr_status s = check_request(r, &q->f);
    if (s != NRR_OK) return s;
    if (q->f.total > S->budget) return NRR_ERR_UNSUPPORTED;  // could never be admitted
    if (q->f.k > 0 && nrr_match_supported(r->dtype, r->block, r->window) != NRR_OK)
        return NRR_ERR_UNSUPPORTED;
    q->r = *r;
    if (hipEventCreateWithFlags(&q->done, hipEventDisableTiming) != hipSuccess) return NRR_ERR_HIP;
    q->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) {
            hipEventDestroy(q->done);
            return NRR_ERR_INVALID_ARG;
        }
        q->ticket = S->next_ticket++;
        S->all[q->ticket] = q;
        S->pending.push_back(q);
    }
    S->cv.notify_all();
    *ticket = q->ticket;
    return NRR_OK;
}

nrr_status nrr_server_poll(nrr_server *S, int64_t ticket, nrr_request_info *info) {
    if (!S || !info) return NRR_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return NRR_ERR_INVALID_ARG;
    fill_info(*it->second, info);
    return NRR_OK;
}

nrr_status nrr_server_wait(nrr_server *S, int64_t ticket, nrr_request_info *info) {
    if (!S) return NRR_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return NRR_ERR_INVALID_ARG;
    std::shared_ptr<Request> q = it->second;
    S->cv_done.wait(lk, [&] { return q->state >= 2; });
    if (info) fill_info(*q, info);
    return q->status == NRR_OK ? NRR_OK : (nrr_status)q->status;
}

nrr_status nrr_server_stats(nrr_server *S, nrr_server_info *info) {
    if (!S || !info) return NRR_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    info->device_bytes = (int64_t)S->budget;
    info->peak_bytes = (int64_t)S->arena.peak();
    info->used_bytes = (int64_t)S->arena.used();
    info->slots = (int32_t)S->streams.size();
    info->max_running = S->max_running;
    info->submitted = S->next_ticket - 1;
    info->admitted = S->admitted;
    info->completed = S->completed;
    info->pending = (int64_t)S->pending.size();
    return NRR_OK;
}

nrr_status nrr_server_destroy(nrr_server *S) {
    if (!S) return NRR_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();  // drains pending and running work
    for (auto &kv : S->all)
        if (kv.second->done) hipEventDestroy(kv.second->done);
    for (hipStream_t st : S->streams) hipStreamDestroy(st);
    hipFree(S->base);
    delete S;
    return NRR_OK;
}

}  // extern "C"
