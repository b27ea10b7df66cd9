// Shared host/device layout of the resident serving worker.
#pragma once

#include <stdint.h>

#include "cyrus_internal.h"

namespace cyrus {

// ---------------------------------------------------------------- serving
// The resident serving worker (serve_kernel): one control workgroup admits
// requests that the host appends to a ring in pinned memory; every other
// workgroup repeatedly claims one row tile of some admitted request's current
// level, runs it, and the workgroup that finishes a level's last tile opens
// the next level (or, after level M, flags the request done in pinned memory).
constexpr int kServeSlots = 128;  // requests in flight (engine slots)

// One request as the host hands it over (pinned ring entry) and as the device
// keeps it (record table): the tree descriptor (t.ue is set by the device to
// this record's UE copy; t.alloc and t.state point at the request's codebook
// and node states in the device pool), the row tiles of each level, the
// admission generation (nonzero, 20 bits), for a small codebook where the
// worker itself delivers it in the pinned pool, and the subtree-unit plan.
constexpr uint32_t kServeDeviceCopyBytes = 128 * 1024;  // larger codebooks go by copy engine
struct alignas(128) ServeRequest {
    DevTree t;
    int32_t ntiles[8];  // [tau], tau = 1..M
    int32_t slot;
    uint32_t gen;
    uint32_t wepoch;    // weight-refresh epoch of the host at admission
    uint32_t cb_words;  // codebook words the worker copies to cb_host (0: the host copies it)
    uint64_t cb_host;   // device address of the request's codebook block in the pinned pool
    // subtree units (sub_split > 0): the whole request is (K+1)^sub_split
    // units, claimed as the tiles of level 1, each the subtree algorithm
    // for one root of level sub_split (LDS plan: sub_bufsize, sub_stbytes)
    int32_t sub_split;
    int32_t sub_bufsize;
    int32_t sub_stbytes;
    int32_t lag;  // generations added to the request's age when workgroups pick tiles
    int32_t ue[3 * kMaxUE];
};

// Scheduling words of one slot, alone on a 128-byte line (the workers'
// atomics on one slot do not contend with another's):
//   claim = [gen 20 | level 3 | tiles of the level 17 | tiles claimed 24] bits,
//           level 0 meaning nothing to do; a worker claims a tile with one
//           fetch-and-add and owns tile `claimed` if it is below `tiles`
//   done  = tiles of the current level finished
struct alignas(128) ServeSlotCtl {
    uint64_t claim;
    uint32_t done;
    int32_t M;
    int32_t ntiles[8];  // [tau]
    int32_t rec;        // the request's record in the launch's record table
    int32_t lag;        // generations added to this request's age when tiles are claimed
};
// Default lag of a request built by level tiles (M dependent steps, well over
// a slot for the 512-wide cells): it ranks, when workgroups pick the oldest
// request with tiles left, as if it had been admitted this many requests
// later, so that the requests of subtree units, which can finish within the
// slot, do not queue behind its level tiles, while it cannot be passed over
// indefinitely. 0 is first come, first served.
constexpr int kServeLevelLag = 64;
constexpr int kServeMaxLag = 1 << 16;

// Request records of one worker launch: the control workgroup copies the k-th
// request it admits into record k, so within a launch every record is written
// once, before any workgroup reads it, and the tile workgroups can read the
// tree descriptor through the scalar cache (as a kernel argument). Records
// are whole 128-byte lines (the L2 line), so reading one never caches part of
// the next. A
// launch that has used every record stops admitting and leaves; the host
// relaunches it for the rest.
constexpr int kServeRecords = 2048;

__host__ __device__ inline uint64_t serve_claim_word(uint32_t gen, int level, int ntiles)
{
    return ((uint64_t)(gen & 0xFFFFFu) << 44) | ((uint64_t)(level & 7) << 41) | ((uint64_t)(ntiles & 0x1FFFF) << 24);
}
constexpr uint32_t kServeGenMask = 0xFFFFFu;  // generations are 20-bit, nonzero
constexpr int kServeMaxTiles = 0x1FFFF;       // row tiles of one level
static_assert(7 * 8 * 8 * 8 * 8 * 8 * 8 / 16 <= kServeMaxTiles, "the largest level (K = M = 7) fits the claim word");

struct ServeCtl {
    ServeSlotCtl slot[kServeSlots];
    int32_t active;   // admitted, unfinished requests
    int32_t quit;     // the control workgroup has exited: workers leave when idle
    int32_t hi;       // 1 + the highest slot index admitted so far
    uint32_t wepoch;  // latest weight-refresh epoch admitted
    uint32_t opened;  // bumped after each level that others may claim tiles of is opened
};

// Pinned host memory shared with the worker.
constexpr int kServeRing = kServeSlots;
struct ServeHost {
    uint32_t tail;      // host: ring entries written so far
    uint32_t stop;      // host: leave now (in-flight requests are abandoned)
    uint32_t consumed;  // control workgroup: ring entries admitted so far
    uint32_t launches;  // unused by the device
    uint32_t finished[kServeSlots];  // worker: gen of the last request finished in each slot
    ServeRequest ring[kServeRing];
};

struct ServeArgs {
    ServeRequest* recs;    // device record table [kServeRecords] (written by the control workgroup)
    ServeCtl* ctl;         // device counters
    ServeHost* host;       // device address of the pinned shared block
    uint32_t head0;        // ring entries admitted before this launch
    int bufsize;           // activation buffer bytes of the level plan
    uint64_t idle_ticks;   // wall-clock ticks with nothing in flight before the worker leaves
    uint64_t stall_ticks;  // wall-clock ticks without progress before any workgroup leaves anyway
};

}  // namespace cyrus
