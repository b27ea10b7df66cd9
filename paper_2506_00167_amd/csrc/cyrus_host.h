// Host-side internals shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdint.h>

#include <memory>
#include <type_traits>
#include <utility>
#include <vector>

#include "cyrus.h"
#include "cyrus_internal.h"

struct cyrus_codebook;

namespace cyrus {

constexpr int kMaxBatch = kMaxEntries;  // codebooks per batched launch

// Derived sizes and the workspace carving of one configuration.
struct Shape {
    int E, K, M, prec, n_layers;
    int dims[kMaxLayers + 1];
    int in_pad[kMaxLayers], out_pad[kMaxLayers];
    size_t w_off[kMaxLayers], b_off[kMaxLayers];
    int in_pad_d;            // per-node inputs of layer 1 (E + 2), padded
    size_t w1d_off;          // their fragments, within one weight buffer
    size_t w_bytes;          // one weight buffer (packed weights + biases)
    size_t staging_floats;   // FP32 staging for the largest layer
    int64_t nodes;
    bool export_logits;
    // device workspace offsets
    size_t off_w[2], off_staging, off_ue, off_alloc, off_state, off_logits, off_batch, device_bytes;
    // pinned host offsets
    size_t hoff_ue, hoff_alloc, hoff_logits, hoff_batch, host_bytes;
};

int validate_config(const cyrus_config* cfg);
Shape make_shape(const cyrus_config* cfg);
size_t batch_area_bytes();
void pack_fragments(const float* w, int out, int in, int out_pad, int in_pad, int prec, float* dst);
float e4m3_weight_scale(const float* w, size_t n);
int choose_rtt(const DevTree& t, int prec, int max_rtt);
// Kernel descriptor of cb with UE state ue_dev, reading weight buffer `slot`
// (-1: the current one).
DevTree make_devtree(const cyrus_codebook* cb, const int32_t* ue_dev, int slot = -1);
int codebook_path(const cyrus_codebook* cb);
int codebook_rtt(const cyrus_codebook* cb);
const Shape& codebook_shape(const cyrus_codebook* cb);
int set_error(int status, const char* msg);
// Mark weight buffer `slot` of cb as read by the work enqueued so far on
// `stream` (records that stream's use event for the slot).
hipError_t note_slot_use(cyrus_codebook* cb, int slot, hipStream_t stream);
// Before a build of cb that reads weight buffer `slot` records ev_done on
// `stream`: keeps the use ev_done marked so far if ev_done moves elsewhere.
hipError_t note_build_use(cyrus_codebook* cb, int slot, hipStream_t stream);
// Validate one host UE state and copy it into cb's pinned staging area (after
// the previous copy out of it has finished).
int stage_ue_host(cyrus_codebook* cb, const cyrus_ue_state* ue);

// Subtree (single-launch latency) path.
bool subtree_supported(const DevTree& t, int prec);
// The resident worker's subtree units (roots at level `split`): whether the
// tree has the shape the worker's instantiation carries, and its LDS plan.
bool plan_subtree_units(const DevTree& t, int prec, int split, int* bufsize, int* stbytes, size_t* lds);
// done (nullable): an event that completes with the launch (the kernel's own
// completion signal, so no separate marker follows it in the stream)
hipError_t launch_subtree(const DevTree& t, int prec, hipStream_t s, hipEvent_t done = nullptr);

}  // namespace cyrus

// The opaque handle of the C ABI.
struct cyrus_codebook {
    cyrus_config cfg;
    cyrus::Shape s;
    int device = 0;
    uint8_t* ws = nullptr;
    uint8_t* host = nullptr;
    uint8_t* host_dev = nullptr;  // device-side address of the pinned buffer (null: not mapped)
    int active = 0;
    float deq[2][cyrus::kMaxLayers];     // per weight buffer: FP8 weight scale * input scale, else 1
    float inv_in[2][cyrus::kMaxLayers];  // per weight buffer: FP8 1 / input scale, else 1
    hipEvent_t ev_staged = nullptr;
    hipEvent_t ev_done = nullptr;
    // A device batch completes all its codebooks with one event, carried by
    // its last launch and shared by the handles it built (recording one
    // event per codebook after the batch put a marker into the stream for
    // each, several microseconds of GPU time apiece); a single build clears it.
    std::shared_ptr<std::remove_pointer_t<hipEvent_t>> batch_done;
    // The event that completes with the handle's last build.
    hipEvent_t done_event() const { return batch_done ? batch_done.get() : ev_done; }
    bool staged_recorded = false;
    bool built = false;
    mutable bool pending = false;       // a build may still run (cleared by a wait)
    mutable bool mirror_valid = false;  // the pinned mirror holds the last build
    // Last use of each weight buffer: one event per stream that enqueued work
    // reading it. set_weights waits for these before overwriting a buffer.
    // The builds of the handle itself mark their use with done_event() (the
    // weight buffer done_slot on stream done_stream), so a build needs no
    // event of its own for it; an entry in slot_use is recorded only when
    // builds move to another stream or buffer.
    std::vector<std::pair<hipStream_t, hipEvent_t>> slot_use[2];
    hipStream_t done_stream = nullptr;
    int done_slot = -1;  // -1: done_event() marks no build
    bool staged_is_done = false;  // the last host build's staging is released by ev_done
    // Serving-engine requests admitted with each weight buffer and not yet
    // retired (their next launches are not enqueued yet, so no event covers
    // them); set_weights refuses to overwrite a buffer while this is nonzero.
    int engine_refs[2] = {0, 0};
    uint64_t wversion = 0;  // incremented by every weight load (create, set_weights)
    int path = 0;  // 0 level, 1 subtree
    int rtt = 1;
    uint64_t rng_seed = 0, rng_tti = 0;  // Gaussian head: Philox key and TTI of the next builds
    std::vector<float> pack;  // host FP32 fragment staging
};

