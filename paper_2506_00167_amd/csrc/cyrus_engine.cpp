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
#include <atomic>
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
    int rslot = -1;     // resident worker: slot of the request
    uint32_t gen = 0;   // resident worker: admission generation (nonzero, 20 bits)
    bool copying = false;  // resident worker: codebook copy to the host pool enqueued
    bool device_copy = false;  // resident worker: the worker writes the codebook to the host pool
    bool subtree = false;      // resident worker: built as subtree units
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
    int level_lag = kServeLevelLag;  // resident worker: lag of requests built by level tiles
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
    // resident worker (cyrus_engine_set_resident)
    bool resident = false;
    ServeRequest* d_recs = nullptr;   // device record table of the resident worker
    ServeCtl* d_ctl = nullptr;        // device counters
    ServeHost* h_shared = nullptr;    // pinned shared block, host address
    ServeHost* h_shared_dev = nullptr;  // and its device address
    uint8_t* hpool_dev = nullptr;     // device address of the pinned pool
    std::vector<int> free_rslots;
    uint32_t tail = 0;
    uint32_t next_gen = 0;
    bool worker_live = false;
    hipEvent_t worker_ev = nullptr;
    hipStream_t copy_stream = nullptr;      // codebooks to the host pool, beside the worker
    hipEvent_t copy_ev[kServeSlots] = {};   // per slot: its request's copy
    std::vector<cyrus_codebook*> cells;  // every cell seen by submit
    bool plan_dirty = false, have_plan = false;
    int plan_rtt = 0, plan_buf = 0;
    size_t plan_bias = 0, plan_lds = 0;
    int ncu = 256;
    uint64_t wall_khz = 100000;  // device wall clock (s_memrealtime) rate
    // weights each cell had when last admitted; a change (or a first
    // sight) bumps the epoch, and the workers invalidate their caches once
    std::unordered_map<cyrus_codebook*, uint64_t> seen_wversion;
    uint32_t wepoch = 0;
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

// ------------------------------------------------------------ resident worker

constexpr double kWorkerIdleMs = 20.0;    // the worker leaves after this long with nothing in flight
constexpr double kWorkerStallMs = 2000.0;  // and after this long with requests in flight but no progress

uint32_t host_load(const volatile uint32_t* p)
{
    const uint32_t v = *p;
    std::atomic_thread_fence(std::memory_order_acquire);
    return v;
}

// Whether the current LDS plan covers every cell seen so far; if not, the
// plan that does.
bool plan_covers(const cyrus_engine* e, const DevTree& t)
{
    return e->have_plan && level_buf_bytes(t, e->prec, e->plan_rtt) <= (size_t)e->plan_buf &&
           level_bias_bytes(t) <= e->plan_bias;
}

int replan(cyrus_engine* e)
{
    std::vector<DevTree> trees;
    for (cyrus_codebook* c : e->cells)
        trees.push_back(make_devtree(c, nullptr));
    int rtt = 0, buf = 0;
    size_t lds = 0;
    if (!plan_level_batch(trees.data(), (int)trees.size(), e->prec, &rtt, &buf, &lds))
        return set_error(CYRUS_EUNSUPPORTED, "the engine's cells do not fit one level-kernel LDS plan");
    size_t bias = 0;
    for (const DevTree& t : trees)
        bias = std::max(bias, level_bias_bytes(t));
    e->plan_rtt = rtt;
    e->plan_buf = buf;
    e->plan_bias = bias;
    e->plan_lds = level_lds_for_buf((size_t)buf, bias, rtt);
    e->have_plan = true;
    e->plan_dirty = false;
    return CYRUS_OK;
}

// Request running[i] has its codebook in its host block: done.
void finish_resident(cyrus_engine* e, size_t i)
{
    Request* r = e->running[i];
    r->status = CYRUS_REQ_DONE;
    r->t_done = now_us();
    r->cell->engine_refs[r->wslot]--;
    release_request_device(e, r);
    e->free_rslots.push_back(r->rslot);
    e->newly_done.push_back(r);
    e->counters[1]++;
    e->running[i] = e->running.back();
    e->running.pop_back();
}

int retire_resident(cyrus_engine* e)
{
    for (size_t i = 0; i < e->running.size();) {
        Request* r = e->running[i];
        if (!r->copying) {
            // the worker has finished the tree: its codebook (device pool) goes to
            // the request's block of the host pool on the copy stream, unless
            // the worker has delivered it there itself
            if (host_load(&e->h_shared->finished[r->rslot]) == r->gen && r->device_copy) {
                finish_resident(e, i);
                continue;
            }
            if (host_load(&e->h_shared->finished[r->rslot]) == r->gen) {
                const Shape& s = codebook_shape(r->cell);
                hipError_t err = hipMemcpyAsync(e->hpool + r->host_off, e->dpool + r->dev_off, (size_t)s.nodes * s.E,
                                                hipMemcpyDeviceToHost, e->copy_stream);
                if (err == hipSuccess)
                    err = hipEventRecord(e->copy_ev[r->rslot], e->copy_stream);
                if (err != hipSuccess)
                    return hip_err(err, "codebook copy");
                r->copying = true;
            }
            ++i;
            continue;
        }
        const hipError_t q = hipEventQuery(e->copy_ev[r->rslot]);
        if (q == hipErrorNotReady) {
            ++i;
            continue;
        }
        if (q != hipSuccess)
            return hip_err(q, "hipEventQuery(codebook copy)");
        finish_resident(e, i);
    }
    return CYRUS_OK;
}

bool worker_running(cyrus_engine* e)
{
    if (e->worker_live && hipEventQuery(e->worker_ev) == hipSuccess)
        e->worker_live = false;
    return e->worker_live;
}

int admit_resident(cyrus_engine* e)
{
    if (e->plan_dirty) {
        bool covered = e->have_plan;
        for (cyrus_codebook* c : e->cells)
            covered = covered && plan_covers(e, make_devtree(c, nullptr));
        if (covered) {
            e->plan_dirty = false;
        } else if (!worker_running(e) && e->running.empty()) {
            // (requests in flight keep the tiling they were admitted with)
            const int rc = replan(e);
            if (rc)
                return rc;
        } else {
            // a wider plan needs a new launch: let the worker drain and leave
            if (e->running.empty())
                e->h_shared->stop = 1;
            return CYRUS_OK;
        }
    }
    while (!e->waiting.empty()) {
        if ((int)e->running.size() >= e->max_active || e->free_rslots.empty()) {
            e->counters[4]++;
            break;
        }
        Request* r = e->waiting.front();
        const Shape& s = codebook_shape(r->cell);
        const size_t tree = ((size_t)s.nodes * s.E + 255) / 256 * 256;
        r->dev_bytes = 2 * tree;  // codebook, then node states
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
        r->rslot = e->free_rslots.back();
        e->free_rslots.pop_back();
        r->wslot = r->cell->active;
        r->cell->engine_refs[r->wslot]++;
        e->next_gen = e->next_gen % (kServeGenMask - 1) + 1;
        r->gen = e->next_gen;
        ServeRequest& q = e->h_shared->ring[e->tail % kServeRing];
        DevTree t = make_devtree(r->cell, nullptr, r->wslot);  // the device points t.ue at its record
        t.alloc = e->dpool + r->dev_off;
        t.state = e->dpool + r->dev_off + tree;
        t.logits = nullptr;
        t.seed = r->seed;
        t.tti = r->tti;
        int32_t nt[8] = {0};
        for (int tau = 1; tau <= s.M; ++tau) {
            const int64_t n_eval = (int64_t)s.K * ipow(s.K + 1, tau - 1);
            // in [1, kServeMaxTiles]: K, M <= 7 give at most 7 * 8^6 / 16 = 114,688 tiles
            nt[tau] = (int32_t)((n_eval + 16 * e->plan_rtt - 1) / (16 * e->plan_rtt));
        }
        // A tree the worker's subtree units cover (BF16, two hidden layers of
        // 256) is built as (K+1)^L units with roots at level L = min(3, M-1):
        // each unit is a register-resident pass over its ancestors and its
        // subtree, so the request takes one round of units instead of M
        // dependent level steps, for about the same work (the ancestors are
        // recomputed per unit) as the level tiles.
        int sub_split = 0, sub_buf = 0, sub_st = 0;
        {
            const int L = std::min(3, s.M - 1);
            size_t sub_lds = 0;
            if (L >= 1 && plan_subtree_units(t, e->prec, L, &sub_buf, &sub_st, &sub_lds) && sub_lds <= e->plan_lds) {
                sub_split = L;
                std::memset(nt, 0, sizeof nt);
                nt[1] = (int32_t)ipow(s.K + 1, L);
            }
        }
        r->subtree = sub_split > 0;
        auto seen = e->seen_wversion.find(r->cell);
        if (seen == e->seen_wversion.end() || seen->second != r->cell->wversion) {
            ++e->wepoch;  // new or refreshed weights: the workers drop their cached lines once
            e->seen_wversion[r->cell] = r->cell->wversion;
        }
        std::memcpy(&q.t, &t, sizeof t);
        std::memcpy(q.ntiles, nt, sizeof nt);
        q.slot = r->rslot;
        q.gen = r->gen;
        q.wepoch = e->wepoch;
        // a small codebook is delivered by the worker into the request's host block
        const size_t cb_bytes = (size_t)s.nodes * s.E;
        r->device_copy = cb_bytes <= kServeDeviceCopyBytes;
        q.cb_words = r->device_copy ? (uint32_t)((cb_bytes + 3) / 4) : 0u;
        q.cb_host = r->device_copy ? (uint64_t)(uintptr_t)(e->hpool_dev + r->host_off) : 0u;
        q.sub_split = sub_split;
        q.sub_bufsize = sub_buf;
        q.sub_stbytes = sub_st;
        q.lag = sub_split > 0 ? 0 : e->level_lag;
        std::memset(q.ue, 0, sizeof q.ue);
        std::memcpy(q.ue, r->ue.data(), r->ue.size() * 4);
        std::atomic_thread_fence(std::memory_order_release);
        *reinterpret_cast<volatile uint32_t*>(&e->h_shared->tail) = ++e->tail;
        r->status = CYRUS_REQ_RUNNING;
        r->copying = false;
        e->running.push_back(r);
        e->waiting.pop_front();
    }
    return CYRUS_OK;
}

int ensure_worker(cyrus_engine* e)
{
    if (worker_running(e))
        return CYRUS_OK;
    const uint32_t consumed = host_load(&e->h_shared->consumed);
    if (consumed == e->tail)
        return CYRUS_OK;  // nothing waits in the ring
    if (!e->have_plan) {
        const int rc = replan(e);
        if (rc)
            return rc;
    }
    e->h_shared->stop = 0;
    std::atomic_thread_fence(std::memory_order_release);
    ServeArgs a{};
    a.recs = e->d_recs;
    a.ctl = e->d_ctl;
    a.host = e->h_shared_dev;
    a.head0 = consumed;
    a.bufsize = e->plan_buf;
    a.idle_ticks = (uint64_t)(kWorkerIdleMs * (double)e->wall_khz);
    a.stall_ticks = (uint64_t)(kWorkerStallMs * (double)e->wall_khz);
    // quit is the only counter a finished launch leaves set
    hipError_t err = hipMemsetAsync(&e->d_ctl->quit, 0, sizeof(int32_t), e->stream);
    if (err == hipSuccess)
        err = launch_serve(a, e->prec, e->plan_rtt, e->ncu, e->plan_lds, e->stream);
    if (err == hipSuccess)
        err = hipEventRecord(e->worker_ev, e->stream);
    if (err != hipSuccess)
        return hip_err(err, "resident worker launch");
    e->worker_live = true;
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
    const size_t dev_need = e->resident ? 2 * (((size_t)s.nodes * s.E + 255) / 256 * 256) : request_dev_bytes(s);
    if (dev_need > e->dcap || request_host_bytes(s) > e->hcap)
        return set_error(CYRUS_EWORKSPACE, "the request's tree does not fit the engine's pools");
    if (e->resident && std::find(e->cells.begin(), e->cells.end(), cell) == e->cells.end()) {
        int rtt = 0, buf = 0;
        size_t lds = 0;
        const DevTree t = make_devtree(cell, nullptr);
        if (!plan_level_batch(&t, 1, s.prec, &rtt, &buf, &lds))
            return set_error(CYRUS_EUNSUPPORTED, "the cell does not fit the level kernel's LDS");
        e->cells.push_back(cell);
        e->plan_dirty = true;
    }
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

int cyrus_engine_set_level_lag(cyrus_engine* e, int32_t lag)
{
    if (!e)
        return set_error(CYRUS_EINVAL, "NULL engine");
    if (lag < 0 || lag > kServeMaxLag)
        return set_error(CYRUS_ERANGE, "lag outside [0, 65536]");
    e->level_lag = lag;
    return CYRUS_OK;
}

int cyrus_engine_set_resident(cyrus_engine* e, int32_t on)
{
    if (!e)
        return set_error(CYRUS_EINVAL, "NULL engine");
    if (on != 0 && on != 1)
        return set_error(CYRUS_EINVAL, "on must be 0 or 1");
    if (e->next_ticket != 0)
        return set_error(CYRUS_EINVAL, "the worker mode is chosen before the first submit");
    if (on == (int)e->resident)
        return CYRUS_OK;
    if (!on)
        return set_error(CYRUS_EINVAL, "the resident worker cannot be switched off once chosen");
    if (hipSetDevice(e->device) != hipSuccess)
        return set_error(CYRUS_EDEVICE, "hipSetDevice failed");
    if (hipHostGetDevicePointer(reinterpret_cast<void**>(&e->hpool_dev), e->hpool, 0) != hipSuccess ||
        !e->hpool_dev) {
        (void)hipGetLastError();
        return set_error(CYRUS_EUNSUPPORTED, "the host pool is not mapped into the device address space");
    }
    size_t doff_slots = 0, doff_ctl = 0, hoff = 0;
    const size_t slots_bytes = sizeof(ServeRequest) * kServeRecords;
    if (!e->dfree.alloc(slots_bytes, &doff_slots))
        return set_error(CYRUS_EWORKSPACE, "device pool too small for the worker's record table");
    if (!e->dfree.alloc(sizeof(ServeCtl), &doff_ctl)) {
        e->dfree.release(doff_slots, slots_bytes);
        return set_error(CYRUS_EWORKSPACE, "device pool too small for the worker's counters");
    }
    if (!e->hfree.alloc(sizeof(ServeHost), &hoff)) {
        e->dfree.release(doff_ctl, sizeof(ServeCtl));
        e->dfree.release(doff_slots, slots_bytes);
        return set_error(CYRUS_EWORKSPACE, "host pool too small for the worker's ring");
    }
    e->d_recs = reinterpret_cast<ServeRequest*>(e->dpool + doff_slots);
    e->d_ctl = reinterpret_cast<ServeCtl*>(e->dpool + doff_ctl);
    e->h_shared = reinterpret_cast<ServeHost*>(e->hpool + hoff);
    e->h_shared_dev = reinterpret_cast<ServeHost*>(e->hpool_dev + hoff);
    std::memset(e->h_shared, 0, sizeof(ServeHost));
    hipError_t err = hipMemsetAsync(e->d_ctl, 0, sizeof(ServeCtl), e->stream);
    if (err == hipSuccess)
        err = hipStreamSynchronize(e->stream);
    if (err == hipSuccess && !e->worker_ev)
        err = hipEventCreateWithFlags(&e->worker_ev, hipEventDisableTiming);
    if (err == hipSuccess && !e->copy_stream)
        err = hipStreamCreateWithFlags(&e->copy_stream, hipStreamNonBlocking);
    for (int i = 0; err == hipSuccess && i < kServeSlots; ++i)
        if (!e->copy_ev[i])
            err = hipEventCreateWithFlags(&e->copy_ev[i], hipEventDisableTiming);
    if (err != hipSuccess)
        return hip_err(err, "resident worker set-up");
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, e->device) == hipSuccess && n > 1)
        e->ncu = n;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeWallClockRate, e->device) == hipSuccess && n > 0)
        e->wall_khz = (uint64_t)n;
    e->free_rslots.clear();
    for (int i = kServeSlots - 1; i >= 0; --i)
        e->free_rslots.push_back(i);
    e->dcap -= std::min(e->dcap, (slots_bytes + 255) / 256 * 256 + (sizeof(ServeCtl) + 255) / 256 * 256);
    e->hcap -= std::min(e->hcap, (sizeof(ServeHost) + 63) / 64 * 64);
    e->resident = true;
    return CYRUS_OK;
}

int cyrus_engine_step(cyrus_engine* e, int32_t* running, int32_t* waiting)
{
    if (!e)
        return set_error(CYRUS_EINVAL, "NULL engine");
    if (hipSetDevice(e->device) != hipSuccess)
        return set_error(CYRUS_EDEVICE, "hipSetDevice failed");
    int rc;
    if (e->resident) {
        rc = retire_resident(e);
        if (rc == CYRUS_OK)
            rc = admit_resident(e);
        if (rc == CYRUS_OK)
            rc = ensure_worker(e);
    } else {
        rc = retire(e);
        if (rc == CYRUS_OK)
            rc = admit(e);
        for (int i = 0; rc == CYRUS_OK && i < e->levels_per_step && !e->running.empty(); ++i)
            rc = launch_step(e);
    }
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

}  // extern "C"

namespace {

// Copy a finished request's codebook to alloc (NULL: no copy) and release it.
int release_result(cyrus_engine* e, int64_t ticket, uint8_t* alloc, size_t bytes)
{
    auto it = e->by_ticket.find(ticket);
    if (it == e->by_ticket.end())
        return set_error(CYRUS_ERANGE, "unknown or released ticket");
    Request* r = it->second;
    if (r->status != CYRUS_REQ_DONE)
        return set_error(CYRUS_ENOTREADY, "request not finished");
    const Shape& s = codebook_shape(r->cell);
    const size_t need = (size_t)s.nodes * s.E;
    if (alloc && bytes < need)
        return set_error(CYRUS_ERANGE, "result buffer too small");
    if (alloc)
        std::memcpy(alloc, e->hpool + r->host_off, need);
    e->hfree.release(r->host_off, r->host_bytes);
    e->by_ticket.erase(it);
    auto nd = std::find(e->newly_done.begin(), e->newly_done.end(), r);
    if (nd != e->newly_done.end())
        e->newly_done.erase(nd);
    delete r;
    return CYRUS_OK;
}

}  // namespace

extern "C" {

int cyrus_engine_result(cyrus_engine* e, int64_t ticket, uint8_t* alloc, size_t bytes)
{
    if (!e || !alloc)
        return set_error(CYRUS_EINVAL, "NULL argument");
    return release_result(e, ticket, alloc, bytes);
}

int cyrus_engine_run(cyrus_engine* e, int32_t n, cyrus_codebook* const* cells, const cyrus_ue_state* ues,
                     const double* arrival_us, uint8_t* const* results, double* latency_us)
{
    if (!e || n < 0 || (n > 0 && (!cells || !ues || !arrival_us)))
        return set_error(CYRUS_EINVAL, "NULL argument");
    for (int32_t i = 0; i < n; ++i) {
        if (!cells[i])
            return set_error(CYRUS_EINVAL, "a cell handle is NULL");
        if (!(arrival_us[i] >= 0.0) || (i > 0 && arrival_us[i] < arrival_us[i - 1]))
            return set_error(CYRUS_ERANGE, "arrival_us must be non-negative and non-decreasing");
    }
    std::unordered_map<int64_t, int32_t> index;  // ticket -> request
    index.reserve((size_t)n * 2);
    const double t0 = now_us();
    int32_t next = 0, done = 0;
    while (done < n) {
        // submit what has arrived
        const double now = now_us() - t0;
        while (next < n && arrival_us[next] <= now) {
            int64_t ticket = 0;
            const int rc = cyrus_engine_submit(e, cells[next], &ues[next], &ticket);
            if (rc)
                return rc;
            index[ticket] = next++;
        }
        int32_t running = 0, waiting = 0;
        int rc = cyrus_engine_step(e, &running, &waiting);
        if (rc)
            return rc;
        // collect what has finished (requests of earlier submits are left alone)
        for (auto it = e->newly_done.begin(); it != e->newly_done.end();) {
            Request* r = *it;
            auto f = index.find(r->ticket);
            if (f == index.end()) {
                ++it;
                continue;
            }
            const int32_t i = f->second;
            index.erase(f);
            if (latency_us)
                latency_us[i] = r->t_done - (t0 + arrival_us[i]);
            it = e->newly_done.erase(it);
            const Shape& s = codebook_shape(r->cell);
            rc = release_result(e, r->ticket, results ? results[i] : nullptr, (size_t)s.nodes * s.E);
            if (rc)
                return rc;
            ++done;
        }
        // nothing in flight: wait for the next arrival
        if (running == 0 && waiting == 0 && done == next && next < n)
            while (now_us() - t0 < arrival_us[next]) {
            }
    }
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
    if (e->resident && e->h_shared) {
        e->h_shared->stop = 1;  // the worker leaves; requests still in flight are abandoned
        std::atomic_thread_fence(std::memory_order_seq_cst);
    }
    (void)hipStreamSynchronize(e->stream);
    if (e->copy_stream) {
        (void)hipStreamSynchronize(e->copy_stream);
        (void)hipStreamDestroy(e->copy_stream);
    }
    for (hipEvent_t ev : e->copy_ev)
        if (ev)
            (void)hipEventDestroy(ev);
    if (e->worker_ev)
        (void)hipEventDestroy(e->worker_ev);
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
