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
//
// Resident volumes: a volume added to the server is copied once into memory
// the server holds until it is removed; requests name it by id instead of
// uploading it.  The block selection of a resident pre-operative volume is
// computed by the first request that needs it (per block, stride, fraction)
// and kept with the volume: later requests wait for that request's event on
// their own stream and reuse the centres.
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

// Device bytes of one request and the offsets of its buffers inside them
// (a volume that is resident takes no room here).
struct Footprint {
    size_t ref, flt, sel, stats, centers, disp, ncc, conf, total;
    int64_t k;
    int32_t grid[3];
};

bool footprint(const nrr_request &r, bool ref_resident, bool flt_resident, Footprint *f) {
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
    f->ref = at, at += ref_resident ? 0 : up(vb);
    f->flt = at, at += flt_resident ? 0 : up(vb);
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

// A selection cached on a resident volume.
struct CachedSelection {
    int32_t block, stride;
    double fraction;
    int64_t k;
    size_t off;                  // centres, in the server's memory
    hipEvent_t ready = nullptr;  // recorded after the selection that fills them
};

struct Volume {
    nrr_dtype dtype;
    int32_t dims[3];
    size_t off = 0, bytes = 0;
    int users = 0;  // requests submitted and not finished that name it
    std::vector<CachedSelection> sels;
};

struct Request {
    nrr_request r;
    Footprint f;
    int64_t ref_vol = 0, flt_vol = 0;  // resident volumes (0: uploaded)
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
    hipStream_t copy_stream = nullptr;  // uploads of resident volumes
    std::vector<bool> slot_busy;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<std::shared_ptr<Request>> pending;
    std::vector<std::shared_ptr<Request>> running;
    std::map<int64_t, std::shared_ptr<Request>> all;  // until released
    std::vector<hipEvent_t> spare_events;
    std::map<int64_t, Volume> volumes;
    int64_t next_ticket = 1, next_volume = 1;
    int64_t admitted = 0, completed = 0;
    int32_t max_running = 0;
    bool stop = false;
    Clock::time_point t_create, t_busy;
    double busy_ms = 0.0;  // wall time with at least one request running
    std::thread worker;
};

namespace {

hipEvent_t take_event(nrr_server *S) {
    if (!S->spare_events.empty()) {
        hipEvent_t e = S->spare_events.back();
        S->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess ? e : nullptr;
}

// The cached selection of a resident volume for (block, stride, fraction),
// made (its centres allocated, not yet computed) when absent and `make`; null
// when absent and not made.
CachedSelection *cached_selection(nrr_server *S, Volume &v, const nrr_request &r, int64_t k,
                                  bool make, bool *fresh) {
    *fresh = false;
    for (CachedSelection &c : v.sels)
        if (c.block == r.block && c.stride == r.stride && c.fraction == r.fraction) return &c;
    if (!make) return nullptr;
    CachedSelection c{r.block, r.stride, r.fraction, k, 0, nullptr};
    if (!S->arena.alloc((size_t)std::max<int64_t>(k, 1) * 12, &c.off)) return nullptr;
    if (!(c.ready = take_event(S))) {
        S->arena.release(c.off, (size_t)std::max<int64_t>(k, 1) * 12);
        return nullptr;
    }
    v.sels.push_back(c);
    *fresh = true;
    return &v.sels.back();
}

void drop_cached(nrr_server *S, Volume &v, CachedSelection *c) {
    S->arena.release(c->off, (size_t)std::max<int64_t>(c->k, 1) * 12);
    S->spare_events.push_back(c->ready);
    v.sels.erase(v.sels.begin() + (c - v.sels.data()));
}

// Enqueue one request on its slot stream.
hipError_t enqueue(nrr_server *S, Request &q) {
    hipStream_t st = S->streams[q.slot];
    char *b = S->base + q.off;
    const nrr_request &r = q.r;
    const Footprint &f = q.f;
    const size_t vb = (size_t)r.dims[0] * r.dims[1] * r.dims[2] * (r.dtype == NRR_U16 ? 2 : 4);
    Volume *rv = q.ref_vol ? &S->volumes.at(q.ref_vol) : nullptr;
    Volume *fv = q.flt_vol ? &S->volumes.at(q.flt_vol) : nullptr;
    char *ref = rv ? S->base + rv->off : b + f.ref;
    char *flt = fv ? S->base + fv->off : b + f.flt;
    hipError_t e = hipSuccess;
    if (!rv) e = hipMemcpyAsync(ref, r.ref, vb, hipMemcpyDefault, st);
    if (e == hipSuccess && !fv) e = hipMemcpyAsync(flt, r.flt, vb, hipMemcpyDefault, st);
    if (e != hipSuccess) return e;
    if (f.k > 0) {
        int32_t *centers = reinterpret_cast<int32_t *>(b + f.centers);
        bool fresh = false;
        CachedSelection *cs = rv ? cached_selection(S, *rv, r, f.k, true, &fresh) : nullptr;
        if (cs) centers = reinterpret_cast<int32_t *>(S->base + cs->off);
        if (!cs || fresh) {
            e = nrr::launch_select(ref, r.dtype, r.dims, r.block, r.stride, f.grid, f.k, centers,
                                   b + f.sel, st);
            if (e == hipSuccess && cs) e = hipEventRecord(cs->ready, st);
            if (e != hipSuccess && cs) drop_cached(S, *rv, cs);  // never filled
        } else {
            e = hipStreamWaitEvent(st, cs->ready, 0);  // made by an earlier request
        }
        if (e != hipSuccess) return e;
        const nrr::StatsLayout L = nrr::stats_layout(r.dtype, r.dims, r.block);
        nrr::MatchArgs a;
        a.ref = ref;
        a.flt = flt;
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
        // window statistics, with the plane-pair volume only for the dot2 form
        nrr::TileShape t;
        const bool pairs = r.dtype == NRR_U16 && (!nrr::match_plan(r.dtype, a, &t) || t.arith == 0);
        const int32_t b3[3] = {r.block, r.block, r.block};
        if ((e = nrr::launch_stats(flt, r.dtype, r.dims, b3, pairs, b + f.stats, st)) != hipSuccess)
            return e;
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

void note_running(nrr_server *S, size_t before) {
    const size_t now_running = S->running.size();
    if (before == 0 && now_running > 0) S->t_busy = Clock::now();
    if (before > 0 && now_running == 0) S->busy_ms += ms_between(S->t_busy, Clock::now());
}

void finish(nrr_server *S, Request &q, int32_t state, int32_t status) {
    S->arena.release(q.off, q.f.total);
    S->slot_busy[q.slot] = false;
    if (q.ref_vol) --S->volumes.at(q.ref_vol).users;
    if (q.flt_vol) --S->volumes.at(q.flt_vol).users;
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
            if (e != hipSuccess) hipStreamSynchronize(S->streams[q.slot]);
            finish(S, q, e == hipSuccess ? 2 : 3, e == hipSuccess ? NRR_OK : NRR_ERR_HIP);
            const size_t before = S->running.size();
            S->running.erase(S->running.begin() + i);
            note_running(S, before);
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
                        // work already queued on the slot may still use the
                        // request's memory: let it drain before the memory
                        // is handed out again
                        hipStreamSynchronize(S->streams[slot]);
                        hipGetLastError();
                        finish(S, q, 3, NRR_ERR_HIP);
                        S->cv_done.notify_all();
                    } else {
                        const size_t before = S->running.size();
                        S->running.push_back(S->pending[i]);
                        note_running(S, before);
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

nrr_status check_request(const nrr_request *r, bool ref_resident, bool flt_resident,
                         Footprint *f) {
    if (!r) return nrr::set_error(NRR_ERR_INVALID_ARG, "request is NULL");
    if (r->dtype != NRR_U16 && r->dtype != NRR_F32)
        return nrr::set_error(NRR_ERR_INVALID_ARG, "unknown dtype %d", (int)r->dtype);
    if ((!ref_resident && !r->ref) || (!flt_resident && !r->flt))
        return nrr::set_error(NRR_ERR_INVALID_ARG, "volume pointer is NULL");
    if (!(r->fraction > 0.0 && r->fraction <= 1.0) || r->window < 0)
        return nrr::set_error(NRR_ERR_INVALID_ARG, "fraction must be in (0, 1], window >= 0");
    if (!footprint(*r, ref_resident, flt_resident, f))
        return nrr::set_error(NRR_ERR_INVALID_ARG, "invalid volume, block or stride");
    if (f->k > 0 && r->capacity < f->k)
        return nrr::set_error(NRR_ERR_BUFFER_TOO_SMALL, "capacity %lld < K = %lld",
                              (long long)r->capacity, (long long)f->k);
    return NRR_OK;
}

// The resident volume `id` for a request (0: none); INVALID_ARG when unknown
// or of another dtype or shape.
nrr_status resident(nrr_server *S, int64_t id, const nrr_request &r) {
    if (id == 0) return NRR_OK;
    auto it = S->volumes.find(id);
    if (it == S->volumes.end())
        return nrr::set_error(NRR_ERR_INVALID_ARG, "unknown volume %lld", (long long)id);
    const Volume &v = it->second;
    if (v.dtype != r.dtype || v.dims[0] != r.dims[0] || v.dims[1] != r.dims[1] ||
        v.dims[2] != r.dims[2])
        return nrr::set_error(NRR_ERR_INVALID_ARG, "volume %lld has another dtype or shape",
                              (long long)id);
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
    const nrr_status s = check_request(r, false, false, &f);
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
    if (hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking) != hipSuccess) {
        for (hipStream_t x : S->streams) hipStreamDestroy(x);
        hipFree(S->base);
        return NRR_ERR_HIP;
    }
    S->slot_busy.assign(slots, false);
    S->t_create = Clock::now();
    nrr_server *raw = S.release();
    raw->worker = std::thread(scheduler, raw);
    *out = raw;
    return NRR_OK;
}

nrr_status nrr_server_submit_resident(nrr_server *S, const nrr_request *r, int64_t ref_volume,
                                      int64_t flt_volume, int64_t *ticket) {
    if (!S || !ticket) return nrr::set_error(NRR_ERR_INVALID_ARG, "server or ticket is NULL");
    if (ref_volume < 0 || flt_volume < 0)
        return nrr::set_error(NRR_ERR_INVALID_ARG, "volume ids are >= 0");
    auto q = std::make_shared<Request>();
    nrr_status s = check_request(r, ref_volume != 0, flt_volume != 0, &q->f);
    if (s != NRR_OK) return s;
    if (q->f.total > S->budget)  // could never be admitted
        return nrr::set_error(NRR_ERR_UNSUPPORTED, "request needs %zu bytes, the server holds %zu",
                              q->f.total, S->budget);
    if (q->f.k > 0 && nrr_match_supported(r->dtype, r->block, r->window) != NRR_OK)
        return NRR_ERR_UNSUPPORTED;
    q->r = *r;
    q->ref_vol = ref_volume;
    q->flt_vol = flt_volume;
    q->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return nrr::set_error(NRR_ERR_INVALID_ARG, "server is shutting down");
        if ((s = resident(S, ref_volume, *r)) != NRR_OK) return s;
        if ((s = resident(S, flt_volume, *r)) != NRR_OK) return s;
        if (!(q->done = take_event(S))) return nrr::set_error(NRR_ERR_HIP, "hipEventCreate failed");
        if (ref_volume) ++S->volumes.at(ref_volume).users;
        if (flt_volume) ++S->volumes.at(flt_volume).users;
        q->ticket = S->next_ticket++;
        S->all[q->ticket] = q;
        S->pending.push_back(q);
    }
    S->cv.notify_all();
    *ticket = q->ticket;
    return NRR_OK;
}

nrr_status nrr_server_submit(nrr_server *S, const nrr_request *r, int64_t *ticket) {
    return nrr_server_submit_resident(S, r, 0, 0, ticket);
}

nrr_status nrr_server_release(nrr_server *S, int64_t ticket) {
    if (!S) return nrr::set_error(NRR_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end())
        return nrr::set_error(NRR_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    if (it->second->state < 2)
        return nrr::set_error(NRR_ERR_INVALID_ARG, "ticket %lld has not finished",
                              (long long)ticket);
    S->spare_events.push_back(it->second->done);
    S->all.erase(it);
    return NRR_OK;
}

nrr_status nrr_server_add_volume(nrr_server *S, const void *data, nrr_dtype dtype,
                                 const int32_t dims[3], int64_t *volume) {
    if (!S || !data || !dims || !volume)
        return nrr::set_error(NRR_ERR_INVALID_ARG, "server, data, dims and volume are non-NULL");
    if (dtype != NRR_U16 && dtype != NRR_F32)
        return nrr::set_error(NRR_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1)
        return nrr::set_error(NRR_ERR_INVALID_ARG, "dims must be >= 1");
    Volume v;
    v.dtype = dtype;
    std::memcpy(v.dims, dims, sizeof v.dims);
    v.bytes = (size_t)dims[0] * dims[1] * dims[2] * (dtype == NRR_U16 ? 2 : 4);
    int64_t id = 0;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return nrr::set_error(NRR_ERR_INVALID_ARG, "server is shutting down");
        if (!S->arena.alloc(v.bytes, &v.off))
            return nrr::set_error(NRR_ERR_BUFFER_TOO_SMALL,
                                  "no room for a %zu-byte volume in the server's memory", v.bytes);
        id = S->next_volume++;
        v.users = 1;  // held until the copy below is done
        S->volumes[id] = v;
    }
    // the id is not published before the copy completes, so no request reads
    // the memory while it is written
    hipError_t e = hipMemcpyAsync(S->base + v.off, data, v.bytes, hipMemcpyDefault, S->copy_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->copy_stream);
    std::lock_guard<std::mutex> lk(S->mu);
    if (e != hipSuccess) {
        hipGetLastError();
        S->arena.release(v.off, v.bytes);
        S->volumes.erase(id);
        return nrr::set_error(NRR_ERR_HIP, "volume upload failed");
    }
    S->volumes[id].users = 0;
    *volume = id;
    return NRR_OK;
}

nrr_status nrr_server_remove_volume(nrr_server *S, int64_t volume) {
    if (!S) return nrr::set_error(NRR_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->volumes.find(volume);
    if (it == S->volumes.end())
        return nrr::set_error(NRR_ERR_INVALID_ARG, "unknown volume %lld", (long long)volume);
    Volume &v = it->second;
    if (v.users > 0)
        return nrr::set_error(NRR_ERR_INVALID_ARG, "volume %lld is used by %d unfinished requests",
                              (long long)volume, v.users);
    for (CachedSelection &c : v.sels) {
        S->arena.release(c.off, (size_t)std::max<int64_t>(c.k, 1) * 12);
        S->spare_events.push_back(c.ready);
    }
    S->arena.release(v.off, v.bytes);
    S->volumes.erase(it);
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
    const auto now = Clock::now();
    info->wall_ms = ms_between(S->t_create, now);
    info->busy_ms = S->busy_ms + (S->running.empty() ? 0.0 : ms_between(S->t_busy, now));
    info->volumes = (int64_t)S->volumes.size();
    info->records = (int64_t)S->all.size();
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
    for (hipEvent_t e : S->spare_events) hipEventDestroy(e);
    for (auto &kv : S->volumes)
        for (CachedSelection &c : kv.second.sels) hipEventDestroy(c.ready);
    for (hipStream_t st : S->streams) hipStreamDestroy(st);
    hipStreamDestroy(S->copy_stream);
    hipFree(S->base);
    delete S;
    return NRR_OK;
}

}  // extern "C"
