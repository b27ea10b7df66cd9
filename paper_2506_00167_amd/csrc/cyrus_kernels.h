// Host-callable launchers of the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "cyrus_internal.h"
#include "cyrus_serve.h"

namespace cyrus {

// Level path: one launch per level tau. rtt = row tiles of 16 per workgroup.
size_t level_buf_bytes(const DevTree& t, int prec, int rtt);
size_t level_lds_bytes(const DevTree& t, int prec, int rtt);
// Row tiles per workgroup (rtt), activation-buffer bytes and LDS bytes of one
// batched level launch over trees[0..n): the largest rtt whose LDS fits.
bool plan_level_batch(const DevTree* trees, int n, int prec, int* rtt, int* buf, size_t* lds);
// done (nullable): an event that completes with this launch (the kernel's own
// completion signal, so no separate marker follows it in the stream)
hipError_t launch_level(const DevTree& t, int prec, int rtt, int tau, hipStream_t s, hipEvent_t done = nullptr);
// Batched: entry j is codebook ent_tree[j] at level ent_tau[j], owning
// workgroups [prefix[j], prefix[j+1]) of an nblocks = prefix[n] launch.
// done (nullable): an event that completes when the launch ends (carried by
// the dispatch itself; recorded in the stream instead if the launch has no
// workgroups).
hipError_t launch_level_batch(const DevTree* trees, const int* ent_tree, const int* ent_tau, const int* prefix, int n,
                              int nblocks, int prec, int rtt, int buf, size_t lds, hipStream_t s,
                              hipEvent_t done = nullptr);

// Resident serving worker over `grid` workgroups (workgroup 0 admits, the
// others run row tiles), with the LDS plan (rtt, a.bufsize, lds) of a batched
// level launch covering every request it will be handed.
hipError_t launch_serve(const ServeArgs& a, int prec, int rtt, int grid, size_t lds, hipStream_t s);
size_t level_bias_bytes(const DevTree& t);
size_t level_lds_for_buf(size_t buf, size_t bias_bytes, int rtt);

// Critic pass (kernels_critic.hip). nets: actor, Q1, Q2, Qtarg1, Qtarg2 as
// FP32 MLP descriptors (E = number of outputs, softmax head = raw outputs).
struct CriticArgs {
    const DevTree* nets;
    const int32_t* ue;
    const int32_t* k;
    const uint8_t* c;
    const float* y;
    const float* reward;
    float* q;
    float* qhat;
    float* loss;
    float* tq;   // [2][H M] target critics at step tau+1 (workspace scratch)
    float* tlp;  // [H M] log pi of the fresh action (workspace scratch)
    int E, M, H;
    float discount, entropy_coef;
    uint64_t seed, episode;
    int bufsize;
    int bias_off[5];
    int bias_total;
};
size_t critic_lds_bytes(int bufsize, int bias_total, int rtt);
// regs_t > 0: the register-resident kernel (regs_t neuron tiles per wave,
// regs_ch1 first-layer chunks, rtt = 2); else the streamed-weight kernel.
hipError_t launch_critic(const CriticArgs& a, int rtt, int regs_t, int regs_ch1, size_t lds, hipStream_t s);

// FP32 fragment-ordered weights -> packed storage of `prec`.
hipError_t launch_convert_weights(int prec, const float* src, uint8_t* dst, int64_t n_floats, float inv_w_scale,
                                  hipStream_t s);

}  // namespace cyrus
