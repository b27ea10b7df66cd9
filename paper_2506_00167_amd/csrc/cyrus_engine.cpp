// Serving engine: continuous batching of codebook requests from many cells.
//
// Iteration-level scheduling: every step enqueues ONE batched level launch in
// which each running request contributes the evaluated nodes of its current
// level (requests are at different levels and have different shapes). Between
// steps, finished requests are retired and waiting requests are admitted in
// FIFO order while the device pool, the pinned host pool and the batch slots
// allow, so a request that arrives while others are on the GPU joins the next
// launch instead of waiting for the current batch to drain.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

#include "cyrus.h"
#include "cyrus_host.h"
#include "cyrus_kernels.h"

using namespace cyrus;

namespace {

double now_us()
{
    using namespace std::chrono;
    return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

int hip_err(hipError_t e, const char* what)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s failed: %s", what, hipGetErrorString(e));
    return set_error(CYRUS_EDEVICE, buf);
}

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Pool {
  public:
    void init(size_t size, size_t align)
    {
        align_ = align;
        free_.clear();
        if (size)
            free_[0] = size;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = (bytes + align_ - 1) / align_ * align_;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest)
                    free_[start] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + align_ - 1) / align_ * align_;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

  private:
    std::map<size_t, size_t> free_;
    size_t align_ = 256, used_ = 0, peak_ = 0;
};

constexpr int kSlots = 4;      // descriptor slots (launches) in flight
constexpr int kSingleMax = 2;  // new single-launch requests per step served one launch each

struct Request {
    int64_t ticket;
    cyrus_codebook* cell;
    int status = CYRUS_REQ_WAITING;
    int level = 0;  // next level to launch (1..M)
    int drain_slot = -1;
    double t_submit = 0, t_done = 0;
    std::vector<int32_t> ue;  // rb[E], mcs[E], sinr bits[E]
    uint64_t seed = 0, tti = 0;  // Gaussian head: the cell's Philox key and TTI at submit
    int wslot = 0;               // the cell's weight buffer, fixed at admission
    size_t dev_off = 0, dev_bytes = 0, host_off = 0, host_bytes = 0;
    bool has_dev = false, has_host = false;
};

size_t slot_bytes()
{
    return (sizeof(DevTree) * kMaxBatch + 255) / 256 * 256 + (size_t)(3 * kMaxBatch + 1) * 4;
}

// Pool bytes one request of `s` holds: its tree (allocations, states) and UE
// state on the device; its codebook mirror and UE staging on the host.
size_t request_dev_bytes(const Shape& s)
{
    const size_t tree = ((size_t)s.nodes * s.E + 255) / 256 * 256;
    return 2 * tree + 3 * kMaxUE * 4;
}
size_t request_host_bytes(const Shape& s) { return (size_t)s.nodes * s.E + 3 * kMaxUE * 4 + 64; }

}  // namespace

struct cyrus_engine {
    uint8_t* dpool = nullptr;
    uint8_t* hpool = nullptr;
    Pool dfree, hfree;
    size_t dcap = 0, hcap = 0;  // pool bytes left for requests after the descriptor slots
    int max_active = 0;
    int levels_per_step = 1;
    hipStream_t stream = nullptr;
    int device = 0;
    int prec = -1;
    std::deque<Request*> waiting;
    std::vector<Request*> running, draining;
    std::unordered_map<int64_t, Request*> by_ticket;
    int64_t next_ticket = 0;
    hipEvent_t ev[kSlots] = {};
    bool slot_used[kSlots] = {};
    size_t slot_doff[kSlots] = {}, slot_hoff[kSlots] = {};
    int next_slot = 0;
    int64_t counters[7] = {};
    std::deque<Request*> newly_done;
};

namespace {

void release_request_device(cyrus_engine* e, Request* r)
{
    if (r->has_dev) {
        e->dfree.release(r->dev_off, r->dev_bytes);
        r->has_dev = false;
    }
}

int retire(cyrus_engine* e)
{
    for (size_t i = 0; i < e->draining.size();) {
        Request* r = e->draining[i];
        const hipError_t q = hipEventQuery(e->ev[r->drain_slot]);
        if (q == hipSuccess) {
            r->status = CYRUS_REQ_DONE;
            r->t_done = now_us();
            r->cell->engine_refs[r->wslot]--;
            release_request_device(e, r);
            e->newly_done.push_back(r);
            e->counters[1]++;
            e->draining[i] = e->draining.back();
            e->draining.pop_back();
        } else if (q == hipErrorNotReady) {
            ++i;
        } else {
            return hip_err(q, "hipEventQuery");
        }
    }
    return CYRUS_OK;
}

int admit(cyrus_engine* e)
{
    while (!e->waiting.empty()) {
        if ((int)e->running.size() >= e->max_active) {
            e->counters[4]++;
            break;
        }
        Request* r = e->waiting.front();
        const Shape& s = codebook_shape(r->cell);
        const size_t tree = ((size_t)s.nodes * s.E + 255) / 256 * 256;
        r->dev_bytes = request_dev_bytes(s);
        r->host_bytes = request_host_bytes(s);
        if (!e->dfree.alloc(r->dev_bytes, &r->dev_off)) {
            e->counters[3]++;
            break;
        }
        if (!e->hfree.alloc(r->host_bytes, &r->host_off)) {
            e->dfree.release(r->dev_off, r->dev_bytes);
            e->counters[3]++;
            break;
        }
        r->has_dev = r->has_host = true;
        uint8_t* dbase = e->dpool + r->dev_off;
        uint8_t* hbase = e->hpool + r->host_off;
        // UE staging sits after the codebook mirror in the host block
        uint8_t* hue = hbase + (((size_t)s.nodes * s.E + 63) / 64 * 64);
        std::memcpy(hue, r->ue.data(), r->ue.size() * 4);
        hipError_t err = hipMemcpyAsync(dbase + 2 * tree, hue, r->ue.size() * 4, hipMemcpyHostToDevice, e->stream);
        if (err == hipSuccess)
            err = hipMemsetAsync(dbase, 0, s.E, e->stream);  // root punctures nothing
        if (err == hipSuccess)
            err = hipMemsetAsync(dbase + tree, 0, s.E, e->stream);  // root state
        if (err != hipSuccess)
            return hip_err(err, "request admission copies");
        r->status = CYRUS_REQ_RUNNING;
        r->level = 1;
        r->wslot = r->cell->active;
        r->cell->engine_refs[r->wslot]++;
        e->running.push_back(r);
        e->waiting.pop_front();
    }
    return CYRUS_OK;
}

int launch_step(cyrus_engine* e)
{
    if (e->running.empty())
        return CYRUS_OK;
    const int slot = e->next_slot;
    if (e->slot_used[slot]) {
        hipError_t err = hipEventSynchronize(e->ev[slot]);
        if (err != hipSuccess)
            return hip_err(err, "hipEventSynchronize(slot)");
    }
    auto tree_of = [&](const Request* r) {
        const Shape& s = codebook_shape(r->cell);
        const size_t tree = ((size_t)s.nodes * s.E + 255) / 256 * 256;
        uint8_t* dbase = e->dpool + r->dev_off;
        DevTree t = make_devtree(r->cell, reinterpret_cast<const int32_t*>(dbase + 2 * tree), r->wslot);
        t.alloc = dbase;
        t.state = dbase + tree;
        t.logits = nullptr;
        t.seed = r->seed;
        t.tti = r->tti;
        return t;
    };
    // Under light load, new requests on cells that take the single-launch
    // path (the whole tree in one launch, one workgroup per subtree, all CUs)
    // run it at their first step and are done in this step. Each such launch
    // holds the whole GPU, so with more new arrivals than kSingleMax in one
    // step they all join the batched level launch instead, which serves many
    // requests for the price of one.
    std::vector<Request*> lvl;
    std::vector<bool> whole(e->running.size(), false);
    int fresh = 0;
    for (const Request* r : e->running)
        fresh += (r->level == 1 && codebook_path(r->cell) == 1) ? 1 : 0;
    const bool single = fresh <= kSingleMax;
    for (size_t i = 0; i < e->running.size(); ++i) {
        Request* r = e->running[i];
        if (single && r->level == 1 && codebook_path(r->cell) == 1) {
            const hipError_t err = launch_subtree(tree_of(r), e->prec, e->stream);
            if (err != hipSuccess)
                return hip_err(err, "single-launch build");
            whole[i] = true;
        } else {
            lvl.push_back(r);
        }
    }
    hipError_t err = hipSuccess;
    if (!lvl.empty()) {
        const int n = (int)lvl.size();
        DevTree trees[kMaxBatch];
        for (int i = 0; i < n; ++i)
            trees[i] = tree_of(lvl[i]);
        int rtt = 0, buf = 0;
        size_t lds = 0;
        if (!plan_level_batch(trees, n, e->prec, &rtt, &buf, &lds))
            return set_error(CYRUS_EUNSUPPORTED, "batch does not fit the level kernel's LDS");
        uint8_t* h = e->hpool + e->slot_hoff[slot];
        uint8_t* d = e->dpool + e->slot_doff[slot];
        const size_t ent_off = (sizeof(DevTree) * kMaxBatch + 255) / 256 * 256;
        std::memcpy(h, trees, sizeof(DevTree) * n);
        int32_t* ent = reinterpret_cast<int32_t*>(h + ent_off);
        int total = 0;
        for (int i = 0; i < n; ++i) {
            const Request* r = lvl[i];
            const int64_t n_eval = trees[i].K * ipow(trees[i].K + 1, r->level - 1);
            ent[i] = i;
            ent[kMaxBatch + i] = r->level;
            ent[2 * kMaxBatch + i] = total;
            total += (int)((n_eval + 16 * rtt - 1) / (16 * rtt));
        }
        ent[2 * kMaxBatch + n] = total;
        err = hipMemcpyAsync(d, h, sizeof(DevTree) * n, hipMemcpyHostToDevice, e->stream);
        if (err == hipSuccess)
            err = hipMemcpyAsync(d + ent_off, h + ent_off, (size_t)(3 * kMaxBatch + 1) * 4, hipMemcpyHostToDevice,
                                 e->stream);
        if (err != hipSuccess)
            return hip_err(err, "descriptor copy");
        const int32_t* dent = reinterpret_cast<const int32_t*>(d + ent_off);
        err = launch_level_batch(reinterpret_cast<const DevTree*>(d), dent, dent + kMaxBatch, dent + 2 * kMaxBatch, n,
                                 total, e->prec, rtt, buf, lds, e->stream);
        if (err != hipSuccess)
            return hip_err(err, "batched level launch");
    }
    // requests that reached their last level: codebook to the host pool
    std::vector<Request*> still;
    for (size_t i = 0; i < e->running.size(); ++i) {
        Request* r = e->running[i];
        const Shape& s = codebook_shape(r->cell);
        if (whole[i] || r->level == s.M) {
            err = hipMemcpyAsync(e->hpool + r->host_off, e->dpool + r->dev_off, (size_t)s.nodes * s.E,
                                 hipMemcpyDeviceToHost, e->stream);
            if (err != hipSuccess)
                return hip_err(err, "codebook copy");
            r->drain_slot = slot;
            e->draining.push_back(r);
        } else {
            r->level++;
            still.push_back(r);
        }
    }
    // every weight buffer this step read: its cell's use event on the stream
    std::vector<std::pair<cyrus_codebook*, int>> used;
    for (const Request* r : e->running) {
        const std::pair<cyrus_codebook*, int> u(r->cell, r->wslot);
        if (std::find(used.begin(), used.end(), u) == used.end()) {
            used.push_back(u);
            err = note_slot_use(r->cell, r->wslot, e->stream);
            if (err != hipSuccess)
                return hip_err(err, "weight-buffer use event");
        }
    }
    e->running.swap(still);
    err = hipEventRecord(e->ev[slot], e->stream);
    if (err != hipSuccess)
        return hip_err(err, "hipEventRecord");
    e->slot_used[slot] = true;
    e->next_slot = (slot + 1) % kSlots;
    e->counters[2]++;
    return CYRUS_OK;
}

}  // namespace

extern "C" {

int cyrus_engine_create(void* device_pool, size_t device_bytes, void* host_pool, size_t host_bytes,
                        int32_t max_active, void* stream, cyrus_engine** out)
{
    if (!device_pool || !host_pool || !out)
        return set_error(CYRUS_EINVAL, "NULL argument");
    if (max_active < 1 || max_active > kMaxBatch)
        return set_error(CYRUS_ERANGE, "max_active outside [1, 128]");
    if (reinterpret_cast<uintptr_t>(device_pool) % 256 || reinterpret_cast<uintptr_t>(host_pool) % 64)
        return set_error(CYRUS_EWORKSPACE, "pools must be 256-byte (device) and 64-byte (host) aligned");
    const size_t dslots = kSlots * ((slot_bytes() + 255) / 256 * 256), hslots = kSlots * ((slot_bytes() + 63) / 64 * 64);
    if (device_bytes < dslots || host_bytes < hslots)
        return set_error(CYRUS_EWORKSPACE, "pools smaller than the descriptor slots");
    cyrus_engine* e = new (std::nothrow) cyrus_engine();
    if (!e)
        return set_error(CYRUS_EINVAL, "out of host memory");
    e->dpool = static_cast<uint8_t*>(device_pool);
    e->hpool = static_cast<uint8_t*>(host_pool);
    e->dfree.init(device_bytes, 256);
    e->hfree.init(host_bytes, 64);
    e->max_active = max_active;
    e->dcap = device_bytes - dslots;
    e->hcap = host_bytes - hslots;
    e->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&e->device) != hipSuccess) {
        delete e;
        return set_error(CYRUS_EDEVICE, "hipGetDevice failed");
    }
    for (int i = 0; i < kSlots; ++i) {
        e->dfree.alloc(slot_bytes(), &e->slot_doff[i]);
        e->hfree.alloc(slot_bytes(), &e->slot_hoff[i]);
        if (hipEventCreateWithFlags(&e->ev[i], hipEventDisableTiming) != hipSuccess) {
            for (int j = 0; j < i; ++j)
                (void)hipEventDestroy(e->ev[j]);
            delete e;
            return set_error(CYRUS_EDEVICE, "event creation failed");
        }
    }
    *out = e;
    return CYRUS_OK;
}

int cyrus_engine_submit(cyrus_engine* e, cyrus_codebook* cell, const cyrus_ue_state* ue, int64_t* ticket)
{
    if (!e || !cell || !ue || !ue->rb || !ue->mcs || !ue->sinr_db || !ticket)
        return set_error(CYRUS_EINVAL, "NULL argument");
    const Shape& s = codebook_shape(cell);
    if (e->prec >= 0 && s.prec != e->prec)
        return set_error(CYRUS_EINVAL, "all cells of an engine must share one precision");
    if (cell->device != e->device)
        return set_error(CYRUS_EINVAL, "cell lives on another device");
    for (int i = 0; i < s.E; ++i)
        if (ue->rb[i] < 0 || ue->rb[i] > 255)
            return set_error(CYRUS_ERANGE, "rb outside [0, 255]");
    // a request that can never fit the pools would block the FIFO forever
    if (request_dev_bytes(s) > e->dcap || request_host_bytes(s) > e->hcap)
        return set_error(CYRUS_EWORKSPACE, "the request's tree does not fit the engine's pools");
    e->prec = s.prec;
    Request* r = new (std::nothrow) Request();
    if (!r)
        return set_error(CYRUS_EINVAL, "out of host memory");
    r->ticket = e->next_ticket++;
    r->cell = cell;
    r->seed = cell->rng_seed;
    r->tti = cell->rng_tti;
    r->t_submit = now_us();
    r->ue.resize(3 * s.E);
    for (int i = 0; i < s.E; ++i) {
        r->ue[i] = ue->rb[i];
        r->ue[s.E + i] = ue->mcs[i];
        std::memcpy(&r->ue[2 * s.E + i], &ue->sinr_db[i], 4);
    }
    e->waiting.push_back(r);
    e->by_ticket[r->ticket] = r;
    e->counters[0]++;
    *ticket = r->ticket;
    return CYRUS_OK;
}

int cyrus_engine_set_levels_per_step(cyrus_engine* e, int32_t levels)
{
    if (!e)
        return set_error(CYRUS_EINVAL, "NULL engine");
    if (levels < 1 || levels > 7)
        return set_error(CYRUS_ERANGE, "levels per step outside [1, 7]");
    e->levels_per_step = levels;
    return CYRUS_OK;
}

int cyrus_engine_step(cyrus_engine* e, int32_t* running, int32_t* waiting)
{
    if (!e)
        return set_error(CYRUS_EINVAL, "NULL engine");
    if (hipSetDevice(e->device) != hipSuccess)
        return set_error(CYRUS_EDEVICE, "hipSetDevice failed");
    int rc = retire(e);
    if (rc == CYRUS_OK)
        rc = admit(e);
    for (int i = 0; rc == CYRUS_OK && i < e->levels_per_step && !e->running.empty(); ++i)
        rc = launch_step(e);
    if (running)
        *running = (int32_t)e->running.size();
    if (waiting)
        *waiting = (int32_t)e->waiting.size();
    return rc;
}

int cyrus_engine_poll(cyrus_engine* e, int64_t ticket, int32_t* status, double* latency_us)
{
    if (!e || !status)
        return set_error(CYRUS_EINVAL, "NULL argument");
    auto it = e->by_ticket.find(ticket);
    if (it == e->by_ticket.end())
        return set_error(CYRUS_ERANGE, "unknown or released ticket");
    *status = it->second->status;
    if (latency_us)
        *latency_us = it->second->status == CYRUS_REQ_DONE ? it->second->t_done - it->second->t_submit : -1.0;
    return CYRUS_OK;
}

int cyrus_engine_completed(cyrus_engine* e, int64_t* tickets, double* latency_us, int32_t cap, int32_t* n)
{
    if (!e || !tickets || !n || cap < 0)
        return set_error(CYRUS_EINVAL, "NULL argument");
    int32_t k = 0;
    while (k < cap && !e->newly_done.empty()) {
        Request* r = e->newly_done.front();
        e->newly_done.pop_front();
        tickets[k] = r->ticket;
        if (latency_us)
            latency_us[k] = r->t_done - r->t_submit;
        ++k;
    }
    *n = k;
    return CYRUS_OK;
}

int cyrus_engine_result(cyrus_engine* e, int64_t ticket, uint8_t* alloc, size_t bytes)
{
    if (!e || !alloc)
        return set_error(CYRUS_EINVAL, "NULL argument");
    auto it = e->by_ticket.find(ticket);
    if (it == e->by_ticket.end())
        return set_error(CYRUS_ERANGE, "unknown or released ticket");
    Request* r = it->second;
    if (r->status != CYRUS_REQ_DONE)
        return set_error(CYRUS_ENOTREADY, "request not finished");
    const Shape& s = codebook_shape(r->cell);
    const size_t need = (size_t)s.nodes * s.E;
    if (bytes < need)
        return set_error(CYRUS_ERANGE, "result buffer too small");
    std::memcpy(alloc, e->hpool + r->host_off, need);
    e->hfree.release(r->host_off, r->host_bytes);
    e->by_ticket.erase(it);
    auto nd = std::find(e->newly_done.begin(), e->newly_done.end(), r);
    if (nd != e->newly_done.end())
        e->newly_done.erase(nd);
    delete r;
    return CYRUS_OK;
}

int cyrus_engine_stats(const cyrus_engine* e, int64_t* c, int32_t n)
{
    if (!e || !c)
        return set_error(CYRUS_EINVAL, "NULL argument");
    int64_t all[7];
    std::memcpy(all, e->counters, sizeof all);
    all[5] = (int64_t)e->dfree.used();
    all[6] = (int64_t)e->dfree.peak();
    for (int i = 0; i < n && i < 7; ++i)
        c[i] = all[i];
    return CYRUS_OK;
}

void cyrus_engine_destroy(cyrus_engine* e)
{
    if (!e)
        return;
    (void)hipSetDevice(e->device);
    (void)hipStreamSynchronize(e->stream);
    for (Request* r : e->running)
        r->cell->engine_refs[r->wslot]--;
    for (Request* r : e->draining)
        r->cell->engine_refs[r->wslot]--;
    for (int i = 0; i < kSlots; ++i)
        (void)hipEventDestroy(e->ev[i]);
    for (auto& kv : e->by_ticket)
        delete kv.second;
    delete e;
}

}  // extern "C"
