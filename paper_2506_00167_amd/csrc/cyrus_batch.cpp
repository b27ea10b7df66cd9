// Several cells' codebooks built in shared launches: one batched level launch
// per mini-slot level covers the evaluated nodes of every codebook at that
// level, so small trees of many cells fill the GPU together.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>

#include "cyrus.h"
#include "cyrus_host.h"
#include "cyrus_kernels.h"

using namespace cyrus;

namespace {

int hip_fail(hipError_t e, const char* what)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s failed: %s", what, hipGetErrorString(e));
    return set_error(CYRUS_EDEVICE, buf);
}

}  // namespace

namespace cyrus {

// Level-launch descriptors of one batch, in the pinned staging area of the
// first handle: DevTree[kMaxBatch], then per level slot the entry lists.
struct BatchLayout {
    size_t trees, slot0, slot_bytes;
};

static BatchLayout batch_layout()
{
    BatchLayout b;
    b.trees = 0;
    b.slot0 = (sizeof(DevTree) * kMaxBatch + 255) / 256 * 256;
    b.slot_bytes = (size_t)(3 * kMaxBatch + 1) * 4;
    return b;
}

// The level launches of a batch. The first handle's staging event (its
// descriptor tables in pinned memory may be rewritten once the copy out of
// them is done) follows that copy; done (nullable) completes with the last
// launch. (A start event carried by the first launch instead of the staging
// marker measured slower on the latency path.)
int build_batch_levels(cyrus_codebook* const* cbs, const DevTree* trees, int n, hipStream_t st, hipEvent_t done)
{
    cyrus_codebook* host_cb = cbs[0];
    const int prec = host_cb->s.prec;
    // one row-tile count and LDS size valid for every member
    int rtt = 0, buf = 0;
    size_t lds = 0;
    if (!plan_level_batch(trees, n, prec, &rtt, &buf, &lds))
        return set_error(CYRUS_EUNSUPPORTED, "batch does not fit the level kernel's LDS");

    const BatchLayout L = batch_layout();
    uint8_t* hbase = host_cb->host + host_cb->s.hoff_batch;
    uint8_t* dbase = host_cb->ws + host_cb->s.off_batch;
    if (host_cb->staged_recorded) {
        hipError_t e = hipEventSynchronize(host_cb->ev_staged);
        if (e != hipSuccess)
            return hip_fail(e, "hipEventSynchronize");
    }
    std::memcpy(hbase + L.trees, trees, sizeof(DevTree) * n);
    int max_m = 0;
    for (int i = 0; i < n; ++i)
        max_m = std::max(max_m, trees[i].M);
    int blocks[8] = {0}, entries[8] = {0};
    for (int tau = 1; tau <= max_m; ++tau) {
        int32_t* slot = reinterpret_cast<int32_t*>(hbase + L.slot0 + (tau - 1) * L.slot_bytes);
        int32_t* ent_tree = slot;
        int32_t* ent_tau = slot + kMaxBatch;
        int32_t* prefix = slot + 2 * kMaxBatch;
        int j = 0, total = 0;
        for (int i = 0; i < n; ++i) {
            if (trees[i].M < tau)
                continue;
            const int64_t n_eval = trees[i].K * ipow(trees[i].K + 1, tau - 1);
            ent_tree[j] = i;
            ent_tau[j] = tau;
            prefix[j] = total;
            total += (int)((n_eval + 16 * rtt - 1) / (16 * rtt));
            ++j;
        }
        prefix[j] = total;
        blocks[tau] = total;
        entries[tau] = j;
    }
    const size_t bytes = L.slot0 + (size_t)max_m * L.slot_bytes;
    hipError_t e = hipMemcpyAsync(dbase, hbase, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(batch descriptors)");
    e = hipEventRecord(host_cb->ev_staged, st);
    if (e != hipSuccess)
        return hip_fail(e, "hipEventRecord");
    host_cb->staged_recorded = true;
    const DevTree* dtrees = reinterpret_cast<const DevTree*>(dbase + L.trees);
    for (int tau = 1; tau <= max_m; ++tau) {
        const int32_t* slot = reinterpret_cast<const int32_t*>(dbase + L.slot0 + (tau - 1) * L.slot_bytes);
        e = launch_level_batch(dtrees, slot, slot + kMaxBatch, slot + 2 * kMaxBatch, entries[tau], blocks[tau], prec,
                               rtt, buf, lds, st, tau == max_m ? done : nullptr);
        if (e != hipSuccess)
            return hip_fail(e, "level batch launch");
    }
    return CYRUS_OK;
}

}  // namespace cyrus

namespace {

// Checks shared by both batch entry points.
int check_batch(cyrus_codebook* const* cbs, int32_t n)
{
    if (!cbs)
        return set_error(CYRUS_EINVAL, "NULL argument");
    if (n < 1 || n > kMaxBatch)
        return set_error(CYRUS_ERANGE, "batch size outside [1, 128]");
    for (int i = 0; i < n; ++i) {
        if (!cbs[i])
            return set_error(CYRUS_EINVAL, "NULL handle in the batch");
        if (cbs[i]->s.prec != cbs[0]->s.prec)
            return set_error(CYRUS_EINVAL, "all codebooks of a batch must share a precision");
        if (cbs[i]->device != cbs[0]->device)
            return set_error(CYRUS_EINVAL, "all codebooks of a batch must live on one device");
        for (int j = 0; j < i; ++j)
            if (cbs[j] == cbs[i])
                return set_error(CYRUS_EINVAL, "a codebook appears twice in one batch");
    }
    return CYRUS_OK;
}

}  // namespace

extern "C" int cyrus_codebook_build_batch_device(cyrus_codebook* const* cbs, const void* const* ue_device, int32_t n,
                                                 void* stream)
{
    int rc = check_batch(cbs, n);
    if (rc)
        return rc;
    if (!ue_device)
        return set_error(CYRUS_EINVAL, "NULL argument");
    DevTree trees[kMaxBatch];
    for (int i = 0; i < n; ++i) {
        if (!ue_device[i])
            return set_error(CYRUS_EINVAL, "NULL UE pointer in the batch");
        if (reinterpret_cast<uintptr_t>(ue_device[i]) % 4)
            return set_error(CYRUS_EINVAL, "UE state must be 4-byte aligned");
        trees[i] = make_devtree(cbs[i], static_cast<const int32_t*>(ue_device[i]));
    }
    hipError_t e = hipSetDevice(cbs[0]->device);
    if (e != hipSuccess)
        return hip_fail(e, "hipSetDevice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // one completion event for the whole batch, carried by its last launch
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess)
        return hip_fail(e, "hipEventCreateWithFlags");
    std::shared_ptr<std::remove_pointer_t<hipEvent_t>> done(ev, [](hipEvent_t x) { (void)hipEventDestroy(x); });
    rc = build_batch_levels(cbs, trees, n, st, ev);
    if (rc)
        return rc;
    for (int i = 0; i < n; ++i) {
        e = note_build_use(cbs[i], cbs[i]->active, st);
        if (e != hipSuccess)
            return hip_fail(e, "weight buffer use");
        cbs[i]->batch_done = done;
        cbs[i]->built = cbs[i]->pending = true;
        cbs[i]->mirror_valid = false;
    }
    return CYRUS_OK;
}

extern "C" int cyrus_codebook_build_batch(cyrus_codebook* const* cbs, const cyrus_ue_state* ue, int32_t n,
                                          void* stream)
{
    int rc = check_batch(cbs, n);
    if (rc)
        return rc;
    if (!ue)
        return set_error(CYRUS_EINVAL, "NULL argument");
    hipError_t e = hipSetDevice(cbs[0]->device);
    if (e != hipSuccess)
        return hip_fail(e, "hipSetDevice");
    // every UE state is validated and staged before anything is enqueued
    for (int i = 0; i < n; ++i) {
        rc = stage_ue_host(cbs[i], &ue[i]);
        if (rc)
            return rc;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    DevTree trees[kMaxBatch];
    for (int i = 0; i < n; ++i)
        trees[i] = make_devtree(cbs[i], reinterpret_cast<const int32_t*>(cbs[i]->ws + cbs[i]->s.off_ue));
    {
        int rtt = 0, buf = 0;
        size_t lds = 0;
        if (!plan_level_batch(trees, n, cbs[0]->s.prec, &rtt, &buf, &lds))
            return set_error(CYRUS_EUNSUPPORTED, "batch does not fit the level kernel's LDS");
    }
    for (int i = 0; i < n; ++i) {
        const Shape& s = cbs[i]->s;
        e = hipMemcpyAsync(cbs[i]->ws + s.off_ue, cbs[i]->host + s.hoff_ue, (size_t)3 * s.E * 4, hipMemcpyHostToDevice,
                           st);
        if (e != hipSuccess)
            return hip_fail(e, "hipMemcpyAsync(UE state)");
    }
    rc = build_batch_levels(cbs, trees, n, st, nullptr);
    if (rc)
        return rc;
    for (int i = 0; i < n; ++i) {
        cyrus_codebook* cb = cbs[i];
        cb->batch_done.reset();  // ev_done, recorded after this handle's copies, completes the build
        const Shape& s = cb->s;
        e = hipEventRecord(cb->ev_staged, st);  // the UE copy out of the pinned buffer
        if (e == hipSuccess)
            e = hipMemcpyAsync(cb->host + s.hoff_alloc, cb->ws + s.off_alloc, (size_t)s.nodes * s.E,
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && s.export_logits)
            e = hipMemcpyAsync(cb->host + s.hoff_logits, cb->ws + s.off_logits, (size_t)s.nodes * s.E * 4,
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = note_build_use(cb, cb->active, st);
        if (e == hipSuccess)
            e = hipEventRecord(cb->ev_done, st);
        if (e != hipSuccess)
            return hip_fail(e, "codebook copy to the pinned mirror");
        cb->staged_recorded = true;
        cb->staged_is_done = false;
        cb->built = cb->pending = cb->mirror_valid = true;
    }
    return CYRUS_OK;
}
