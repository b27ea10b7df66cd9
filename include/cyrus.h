/*
 * cyrus.h - C ABI of the MI355X puncturing-codebook builder.
 *
 * The builder is the real-time O-DU step of Cyrus+ (arXiv 2506.00167,
 * Sec. IV-C "RT O-DU", Sec. V-B, Alg. 2): once per slot it evaluates the
 * actor network f_a on every node of the tree of URLLC arrival sequences over
 * the slot's M mini-slots (arrival counts k in {0..K}, K = floor(N/L),
 * Sec. III-A), carries each eMBB UE's punctured-RB state down the tree, and
 * turns every node's output into an integer per-UE puncturing vector
 * (softmax, the KL projection of Eqs. (6)-(7), largest-remainder rounding).
 * The O-RU then reads one row per mini-slot (Alg. 3): cyrus_codebook_lookup.
 *
 * Conventions for every entry point:
 *  - Status: int, CYRUS_OK (0) or a negative CYRUS_E* code. On error nothing
 *    is enqueued on the stream, outputs are left untouched, and
 *    cyrus_last_error() returns a thread-local message.
 *  - No exceptions or aborts cross this boundary.
 *  - Host pointers are plain CPU memory; "device" pointers are HIP device
 *    memory of the current device. Streams are hipStream_t passed as void*
 *    (NULL = the default stream).
 *  - The library never allocates device memory: the caller provides one
 *    device workspace and one pinned host buffer per codebook, sized by
 *    cyrus_codebook_workspace_size, which must outlive the handle.
 *  - A handle is used by one host thread at a time.
 *
 * Node order (BFS): level tau (1..M) starts at O_tau = ((K+1)^tau - 1)/K;
 * the node for arrival prefix (k_1..k_tau) is O_tau + sum_t k_t (K+1)^(tau-t).
 * Node 0 is the root (start of the slot). nodes = ((K+1)^(M+1) - 1)/K.
 */
#ifndef CYRUS_H
#define CYRUS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define CYRUS_OK 0
#define CYRUS_EINVAL (-1)      /* null pointer or malformed argument */
#define CYRUS_ERANGE (-2)      /* a size or value outside the supported range */
#define CYRUS_EWORKSPACE (-3)  /* workspace or pinned buffer too small / misaligned */
#define CYRUS_EDEVICE (-4)     /* a HIP runtime call failed */
#define CYRUS_ENOTREADY (-5)   /* lookup/export before any build */
#define CYRUS_EUNSUPPORTED (-6)/* shape/precision combination not provided */

/* ------------------------------------------------------------ precisions */
#define CYRUS_FP32 0     /* layer GEMMs in FP32 on MFMA */
#define CYRUS_BF16 1     /* BF16 operands, FP32 accumulation */
#define CYRUS_FP8_E4M3 2 /* OCP E4M3 operands, power-of-two per-tensor scales,
                            FP32 accumulation */

/* ------------------------------------------------------------ flags */
#define CYRUS_FLAG_EXPORT_LOGITS 1u      /* keep the FP32 logits of every node */
#define CYRUS_FLAG_LEVEL_KERNEL 2u       /* force the one-launch-per-level path */
/* Integer step of the enforcer: Huntington-Hill apportionment (the rounding
 * the paper names, Sec. IV-B) instead of the default largest remainder. Units
 * go by priority x_e / sqrt(n (n+1)) within the caps, ties to the larger share
 * then the lower UE index; when T is below the number of UEs with a positive
 * share (no Huntington-Hill allocation exists then) the T largest shares get
 * one unit each. */
#define CYRUS_FLAG_HUNTINGTON_HILL 4u
/* The paper's stochastic policy head (Sec. IV-B): the actor has 2E outputs,
 * means mu_e then log standard deviations (clamped to [-20, 2]); every
 * evaluated node draws eps_e ~ N(0, 1) (Philox4x32-10, key = seed, counter =
 * (node, e, tti); Box-Muller on the first two words), samples u = mu + sigma
 * eps, maps it through tanh to b_e = (1 + tanh u_e) / 2 and hands the
 * enforcer the log-shares log b_e in place of logits. Seed and TTI come from
 * cyrus_codebook_set_rng. Without it the actor has E outputs (logits). */
#define CYRUS_FLAG_GAUSSIAN_HEAD 8u

#define CYRUS_MAX_HIDDEN 4
#define CYRUS_MAX_LAYERS (CYRUS_MAX_HIDDEN + 1)
#define CYRUS_MAX_UE 32

/* Tree and actor shape.
 *   num_ue        E in [1, 32]: eMBB UEs of the cell (Sec. III-A).
 *   max_arrival   K in [1, 7]: floor(N/L), the largest number of URLLC
 *                 packets punctured in one mini-slot (Sec. III-A).
 *   num_minislots M in [1, 7]: mini-slots per slot (7 in NR, Sec. III-A).
 *   rb_per_unit   U >= 1: RBs one URLLC packet needs (L in RB units).
 *                 M*K*U must not exceed 255 (the carried state is 8-bit).
 *   num_hidden    hidden layers of f_a, in [1, 4]; hidden[i] their widths,
 *                 each a multiple of 32 in [32, 512] (the kernels compute
 *                 128 neurons at a time; other widths are zero-padded to the
 *                 next multiple of 128, which leaves the results unchanged).
 *   precision     CYRUS_FP32, CYRUS_BF16 or CYRUS_FP8_E4M3.
 *   flags         CYRUS_FLAG_*.
 * The actor's input width is 4E+2 and its output width is E. */
typedef struct {
    int32_t num_ue;
    int32_t max_arrival;
    int32_t num_minislots;
    int32_t rb_per_unit;
    int32_t num_hidden;
    int32_t hidden[CYRUS_MAX_HIDDEN];
    int32_t precision;
    uint32_t flags;
} cyrus_config;

/* Actor parameters f_a in canonical FP32, host memory, read during the call.
 *   w[l]  row-major [out_l][in_l] (in_0 = 4E+2, out_last = E)
 *   b[l]  [out_l]
 *   act_scale  FP8 only: num_hidden+1 positive powers of two, the scale of each
 *              layer's input (input / scale is rounded to E4M3); NULL otherwise.
 * Weight scales for FP8 are derived by the library (smallest power of two that
 * keeps max|w|/scale <= 448). Each layer's combined output scale, weight scale
 * x act_scale[l] / act_scale[l+1] (the last layer: weight scale x
 * act_scale[l]), must lie in 2^-126..2^127, else CYRUS_ERANGE. */
typedef struct {
    const float* w[CYRUS_MAX_LAYERS];
    const float* b[CYRUS_MAX_LAYERS];
    const float* act_scale;
} cyrus_weights;

/* Per-UE scheduling state of one TTI, host arrays of E entries (Sec. III-A:
 * the eMBB scheduling vector s(t), here in RBs, plus channel features).
 *   rb       RBs scheduled to UE e in this TTI, in [0, 255] (0 = unscheduled)
 *   mcs      MCS index
 *   sinr_db  SINR in dB */
typedef struct {
    const int32_t* rb;
    const int32_t* mcs;
    const float* sinr_db;
} cyrus_ue_state;

typedef struct cyrus_codebook cyrus_codebook;

/* Sizes of the two caller-owned buffers for `cfg`: device workspace (align 256)
 * and pinned host buffer (align 64). */
int cyrus_codebook_workspace_size(const cyrus_config* cfg, size_t* device_bytes, size_t* host_bytes);

/* Create a builder bound to the current device. Copies (and for BF16/FP8
 * rounds) the weights into the workspace; blocks until that copy is done.
 * device_ws / host_pinned: caller-owned, at least the sizes above; host_pinned
 * must be page-locked memory. *out receives the handle. */
int cyrus_codebook_create(const cyrus_config* cfg, const cyrus_weights* w, void* device_ws, size_t ws_bytes,
                          void* host_pinned, size_t host_bytes, void* stream, cyrus_codebook** out);

/* Policy refresh from the Near-RT RIC (Alg. 1 pushes the updated f_a to the
 * O-DU): loads new weights into the idle half of a double buffer on `stream`,
 * waits for the copy, then makes them current. Builds enqueued before the call
 * keep the old weights: before overwriting a half, the call blocks until every
 * build, batch and engine request enqueued earlier that reads that half has
 * finished (on whatever stream it runs). Engine requests keep the weights
 * that were current when they were admitted. */
int cyrus_codebook_set_weights(cyrus_codebook* cb, const cyrus_weights* w, void* stream);

/* Alg. 2 for one TTI: s(t) in, codebook B*(t) out. Asynchronous on `stream`:
 * host UE arrays are copied into the pinned buffer before returning; then, on
 * the single-launch path, one kernel reads them from the pinned buffer and
 * writes the codebook (and the logits if exported) straight into the pinned
 * mirror; on the level path, the UE state is copied to the device and the
 * level kernels write the codebook (and logits) straight into the pinned
 * mirror too (when the pinned buffer is mapped for the device; else device-to-
 * host copies follow them). The handle's completion event, which
 * cyrus_codebook_wait waits for, completes with the last kernel (or copy).
 * The device array (cyrus_codebook_device_alloc) is only written by device
 * builds. */
int cyrus_codebook_build(cyrus_codebook* cb, const cyrus_ue_state* ue, void* stream);

/* Device-resident variant: the UE state is already in device memory as
 * int32 rb[E], int32 mcs[E], float sinr_db[E] (contiguous, 4-byte aligned) and
 * the codebook stays in the device workspace (cyrus_codebook_device_alloc);
 * nothing is copied to the host. The completion event completes with the
 * last kernel. */
int cyrus_codebook_build_device(cyrus_codebook* cb, const void* ue_device, void* stream);

/* Build n codebooks in shared launches on one stream (cells batched per
 * launch: one batched level launch per mini-slot level covers every member's
 * nodes at that level); the serving and stress extension of Alg. 2. All
 * handles must share a precision and a device, and no handle may appear
 * twice. ue: n host UE states (as for cyrus_codebook_build), validated and
 * copied into each handle's pinned buffer before the call returns; the calls
 * enqueue the UE copies, the level launches, then each codebook's (and
 * logits') copy into its pinned mirror, and record each handle's event, so
 * lookup/export read the new codebooks after it. CYRUS_ERANGE for n outside
 * [1, 128]; CYRUS_EUNSUPPORTED (nothing enqueued) when the batch does not fit
 * the level kernel's LDS. */
int cyrus_codebook_build_batch(cyrus_codebook* const* cbs, const cyrus_ue_state* ue, int32_t n, void* stream);

/* Device-resident batch: ue_device holds n pointers to device UE states laid
 * out as for cyrus_codebook_build_device (4-byte aligned). Results stay in
 * each handle's workspace (cyrus_codebook_device_alloc); one event, which
 * completes with the batch's last launch, serves as every member's completion
 * event (until the member's next build). Same checks as
 * cyrus_codebook_build_batch. */
int cyrus_codebook_build_batch_device(cyrus_codebook* const* cbs, const void* const* ue_device, int32_t n,
                                      void* stream);

/* Block until the last build of this handle has finished. */
int cyrus_codebook_wait(cyrus_codebook* cb);

/* Alg. 3, one mini-slot: the puncturing vector (E bytes, RBs per UE) for
 * mini-slot tau in [1, M] after arrivals k_1..k_tau (arrivals[0..tau-1], each
 * in [0, K], already capped by the O-RU controller). Waits for the last host
 * build once, then reads the pinned mirror. */
int cyrus_codebook_lookup(const cyrus_codebook* cb, const uint8_t* arrivals, int32_t tau, uint8_t* alloc_out);

/* O-RU side of one slot: the controller caps the URLLC packets punctured in
 * a mini-slot at K and carries the rest to the next one (Sec. III-A:
 * k_tau = min(K, a_tau + q_{tau-1}), q_tau = a_tau + q_{tau-1} - k_tau,
 * q_0 = carry_in), and Alg. 3 reads each mini-slot's puncturing vector from the
 * codebook for the served prefix.
 *   raw_arrivals  [num_minislots] packets arriving per mini-slot (>= 0)
 *   served        [num_minislots] out: packets punctured per mini-slot
 *   y             [num_minislots][E] out: the puncturing matrix Y(t)
 *   carry_out     out: packets still buffered after the slot
 * Waits for the last build like lookup. */
int cyrus_codebook_assemble(const cyrus_codebook* cb, const int32_t* raw_arrivals, int32_t carry_in, uint8_t* served,
                            uint8_t* y, int32_t* carry_out);

/* Copy the whole codebook to host memory: alloc [nodes][E] bytes; logits
 * [nodes][E] FP32 or NULL (needs CYRUS_FLAG_EXPORT_LOGITS). Waits for the
 * last build; after a device build it copies from the workspace. */
int cyrus_codebook_export(const cyrus_codebook* cb, uint8_t* alloc, float* logits);

/* Device address of the codebook array [nodes][E] inside the workspace. */
const uint8_t* cyrus_codebook_device_alloc(const cyrus_codebook* cb);

/* Number of tree nodes (root included); -1 for a NULL handle. */
int64_t cyrus_codebook_num_nodes(const cyrus_codebook* cb);

/* Which kernel family builds this codebook: "subtree" (one launch, one
 * workgroup per subtree, actor weights held in registers) or "level" (one
 * launch per mini-slot level). */
const char* cyrus_codebook_kernel_path(const cyrus_codebook* cb);

/* Gaussian head only: the Philox key (`seed`) and the TTI number that the
 * following builds of this handle use (engine requests take them at submit).
 * Builds with the same seed, TTI, weights and UE state are identical. Default
 * 0, 0. CYRUS_EINVAL if cb is NULL. */
int cyrus_codebook_set_rng(cyrus_codebook* cb, uint64_t seed, uint64_t tti);

/* Release the handle (not the caller-owned buffers). Waits for pending work. */
void cyrus_codebook_destroy(cyrus_codebook* cb);

const char* cyrus_status_string(int status);
const char* cyrus_last_error(void);

/* Hash (16 hex digits) of the source files this library was compiled from,
 * fixed at build time, so a binding can refuse a library older than the
 * sources beside it. A static string; never NULL. */
const char* cyrus_build_source_hash(void);

/* ------------------------------------------------------------------------
 * Near-RT RIC critic pass (Sec. IV-B, Eqs. (3) and (4)): the batched forward
 * evaluation that the critics' update needs, for H buffer samples of M steps
 * (the backward pass and the optimiser are not part of this library).
 *
 * For sample h and step tau (1..M) the critic input is the actor's state
 * features at that step (R/32, MCS/32, SINR/32, c/64 per UE, tau/8, k/8) followed
 * by the action y, dimension 5E+2. The pass computes
 *   q[i][h][tau] = Q_i(state, y),  i = 0, 1                      (Eq. (3) input)
 *   qhat[h][tau] = discount * (min_i Qtarg_i(state at tau+1, y~)
 *                              - entropy_coef * log pi(y~))      (Eq. (4), tau < M)
 *                = reward[h]                                      (tau = M)
 * where y~ is a fresh action of the actor (Gaussian head, the draws of
 * CYRUS_FLAG_GAUSSIAN_HEAD with counter node = h M + tau and TTI = episode,
 * y~ = (1 + tanh u) / 2) and log pi its log density; when no packet arrives at
 * step tau+1 the policy does not act (y~ = 0, log pi = 0). Then
 *   loss[i] = mean over h, tau of (q[i][h][tau] - qhat[h][tau])^2      (Eq. (3)).
 * All arithmetic is FP32 with FP32 accumulation. */
typedef struct {
    int32_t num_ue;                         /* E in [1, 16] */
    int32_t num_minislots;                  /* M in [1, 7]: steps per sample */
    int32_t num_samples;                    /* H >= 1, H*M <= 2^24 */
    int32_t actor_hidden_layers;            /* in [1, 4] */
    int32_t actor_hidden[CYRUS_MAX_HIDDEN]; /* multiples of 32 in [32, 512] (zero-padded
                                               to the next multiple of 128 inside) */
    int32_t critic_hidden_layers;           /* in [1, 4] */
    int32_t critic_hidden[CYRUS_MAX_HIDDEN]; /* as actor_hidden */
    float discount;                         /* lambda of Eq. (4) */
    float entropy_coef;                     /* zeta of Eq. (4) */
} cyrus_critic_config;

/* FP32 host weights, row-major [out][in] per layer (act_scale is ignored).
 *   actor     4E+2 -> actor_hidden -> 2E (means, then log standard deviations)
 *   q, q_targ 5E+2 -> critic_hidden -> 1 */
typedef struct {
    cyrus_weights actor;
    cyrus_weights q[2];
    cyrus_weights q_targ[2];
} cyrus_critic_weights;

/* One batch of buffer samples, device arrays read during the pass. */
typedef struct {
    const int32_t* ue;    /* [H][3E]: rb, mcs, sinr_db (float bits) per UE */
    const int32_t* k;     /* [H][M]: URLLC arrivals of each step, in [0, 255] */
    const uint8_t* c;     /* [H][M][E]: punctured RBs carried into each step */
    const float* y;       /* [H][M][E]: the stored actions */
    const float* reward;  /* [H]: r(t) of each sample */
} cyrus_critic_batch;

typedef struct cyrus_critic cyrus_critic;

/* Device workspace bytes (align 256) for `cfg`: the five networks' packed
 * weights, their descriptors, and 12 bytes per row (H M rows) of scratch for
 * the per-row targets, which cyrus_critic_evaluate overwrites. */
int cyrus_critic_workspace_size(const cyrus_critic_config* cfg, size_t* device_bytes);

/* Bind a critic evaluator to the current device: validates cfg, packs the
 * weights into the caller-owned workspace on `stream` and waits for the copy.
 * *out receives the handle. The library allocates no device memory. */
int cyrus_critic_create(const cyrus_critic_config* cfg, const cyrus_critic_weights* w, void* device_ws,
                        size_t ws_bytes, void* stream, cyrus_critic** out);

/* One pass over a batch, asynchronous on `stream`. Outputs are device arrays:
 * q [2][H][M], qhat [H][M], loss [2]. Same inputs, seed and episode give the
 * same outputs bit for bit. Passes on one handle share its workspace scratch,
 * so passes that overlap in time (other streams) race; order them on one
 * stream. CYRUS_EINVAL for NULL pointers. */
int cyrus_critic_evaluate(cyrus_critic* cr, const cyrus_critic_batch* batch, uint64_t seed, uint64_t episode,
                          float* q, float* qhat, float* loss, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * pass as cyrus_critic_evaluate with the same kernels and outputs, but the
 * per-row targets go to a static device array inside the library (one per
 * GPU, held until the process ends, at most 65,536 rows = num_samples x
 * num_minislots, 768 KiB) instead of the handle's workspace scratch. It calls
 * no allocating routine. CYRUS_ERANGE (nothing enqueued) for more rows.
 * Every call on one GPU shares that array: calls that overlap in time on one
 * GPU (other streams, other handles) race; order them on one stream. */
int cyrus_critic_evaluate_noalloc(cyrus_critic* cr, const cyrus_critic_batch* batch, uint64_t seed, uint64_t episode,
                                  float* q, float* qhat, float* loss, void* stream);

/* Release the handle (not the workspace). */
void cyrus_critic_destroy(cyrus_critic* cr);

/* ------------------------------------------------------------------------
 * Serving engine: continuous batching of codebook requests from many cells.
 *
 * Each cell is a cyrus_codebook handle (its actor weights stay resident in its
 * workspace). A request is one TTI of one cell (Alg. 2 for that cell). The
 * engine advances every admitted request by one tree level per step, in ONE
 * batched launch whatever the requests' shapes and current levels, and admits
 * waiting requests (FIFO) between steps as device-pool memory and batch slots
 * free up, so requests that arrive while others are on the GPU join the next
 * launch. A request's tree (allocations and states) lives in the engine's
 * device pool until its codebook has been copied to the engine's pinned host
 * pool; results are bit-identical to the same request built alone by the
 * engine. All cells of an engine must share one precision; every step uses the
 * level kernel.
 *
 * device_pool / host_pool: caller-owned device memory (align 256) and pinned
 * host memory (align 64) from which requests are admitted.
 * max_active: requests batched per step, in [1, 128].
 * A handle is used by one host thread at a time. */
typedef struct cyrus_engine cyrus_engine;

#define CYRUS_REQ_WAITING 0  /* queued, not admitted (memory or batch full) */
#define CYRUS_REQ_RUNNING 1  /* admitted, levels in flight */
#define CYRUS_REQ_DONE 2     /* codebook in the host pool, result() may copy it */

int cyrus_engine_create(void* device_pool, size_t device_bytes, void* host_pool, size_t host_bytes,
                        int32_t max_active, void* stream, cyrus_engine** out);

/* Queue one request for `cell`; the UE arrays are copied before returning.
 * *ticket receives an id (increasing from 0). CYRUS_EWORKSPACE (nothing
 * queued) when the request's tree could never fit the engine's pools, so an
 * oversize request cannot block the FIFO. */
int cyrus_engine_submit(cyrus_engine* eng, cyrus_codebook* cell, const cyrus_ue_state* ue, int64_t* ticket);

/* One engine iteration: retire requests whose codebook copy finished, admit
 * waiting requests that fit, then enqueue batched level launches for all
 * running requests, each launch advancing every running request by one level
 * (and queueing the host copies of the ones that reached level M): one launch
 * per step by default (iteration-level batching: requests join between
 * levels), up to levels_per_step launches (see below). Under light load (at
 * most two new such requests in the step) a request whose cell takes the
 * single-launch path (cyrus_codebook_kernel_path: "subtree") is built whole
 * by one launch at its first step instead. Never blocks on the GPU
 * except to reuse a descriptor slot still in flight. Outputs (nullable):
 * running and waiting request counts after the step. */
int cyrus_engine_step(cyrus_engine* eng, int32_t* running, int32_t* waiting);

/* Level launches per cyrus_engine_step, in [1, 7] (default 1). With 7, every
 * request admitted in a step completes in that step's launches: one host step
 * per request instead of one per level, so a request's latency is one step's
 * GPU time plus its wait for the step, at the cost of new arrivals waiting for
 * the next step. CYRUS_ERANGE outside [1, 7]. */
int cyrus_engine_set_levels_per_step(cyrus_engine* eng, int32_t levels);

/* Resident worker (on = 1), chosen before the first submit: instead of
 * host-stepped launches, ONE resident kernel serves every request. Its
 * workgroup 0 takes requests from a ring in the host pool (pinned memory that
 * the device reads and writes directly); every other workgroup repeatedly
 * claims one row tile of the oldest admitted request whose current level has
 * tiles left, runs it (the batched level kernel's tile), and the workgroup
 * that finishes a level's last tile opens the next level; after level M that
 * workgroup writes a codebook of up to 128 KiB into the request's block of
 * the host pool itself and sets the request's completion flag in pinned
 * memory. Levels of different requests overlap freely and no host step is
 * needed between levels: cyrus_engine_step retires finished requests (it
 * reads the flags, and copies each larger codebook from the device pool into
 * the request's block of the host pool on a copy stream of the engine's
 * own), admits waiting ones
 * into free slots and pool memory, and relaunches the worker when it has
 * exited with requests waiting. The worker leaves after 20 ms with nothing to
 * do, after 2 s without progress, after admitting 2,048 requests (the host then
 * relaunches it), or when the engine is destroyed; it first finishes every
 * request it has admitted (on destroy, their results are dropped). Up to 128 requests are in flight. Results are bit-identical
 * to the same request alone (every request runs the same tile code whatever
 * the mix). CYRUS_EINVAL after a submit or for on = 0 once resident;
 * CYRUS_EWORKSPACE if the pools cannot hold the worker's tables (about
 * 1.6 MiB device, 100 KiB host); CYRUS_EUNSUPPORTED if the host pool is not
 * mapped for the device. */
int cyrus_engine_set_resident(cyrus_engine* eng, int32_t on);

/* Resident worker's tile order: its workgroups take tiles of the oldest
 * request with tiles left, a request built by level tiles (one that the
 * worker cannot build as register-resident subtree units, such as the 512-wide
 * cells, which take M dependent steps) ranking as if admitted `lag` requests
 * later. Requests that can finish within the slot then do not queue behind
 * the long ones, and a long one is passed over by at most `lag` later
 * admissions. 0 is first come, first served; default 64. Applies to requests
 * admitted after the call; results do not depend on it. CYRUS_ERANGE outside
 * [0, 65536]. */
int cyrus_engine_set_level_lag(cyrus_engine* eng, int32_t lag);

/* Status of a ticket (CYRUS_REQ_*); *latency_us (nullable) receives, once
 * done, the time from submit to the step that observed completion. */
int cyrus_engine_poll(cyrus_engine* eng, int64_t ticket, int32_t* status, double* latency_us);

/* Tickets that became done since the previous call (at most `cap`), with
 * their latencies in microseconds (nullable); *n receives the count. */
int cyrus_engine_completed(cyrus_engine* eng, int64_t* tickets, double* latency_us, int32_t cap, int32_t* n);

/* Copy a finished request's codebook ([nodes][E] bytes) and release its slot. */
int cyrus_engine_result(cyrus_engine* eng, int64_t ticket, uint8_t* alloc, size_t bytes);

/* A native request loop (Sec. VII's serving timing, without a host
 * interpreter between steps): request i, for cells[i] with UE state ues[i],
 * is submitted once arrival_us[i] microseconds have passed since the call
 * began (non-negative and non-decreasing; all zero submits everything at
 * once). The loop submits what has arrived, steps the engine, and copies each
 * finished request's codebook ([nodes][E] bytes) to results[i] and releases
 * it (results NULL, or results[i] NULL: released without a copy), until all n
 * are done. latency_us[i] (nullable) receives the time from the request's
 * arrival to the step that observed its completion, so that a wait before
 * the submit counts. Requests of earlier submits stay in the engine. Returns
 * the first error of a submit or step (CYRUS_EINVAL for a NULL array or cell,
 * CYRUS_ERANGE for arrival times out of order); requests already submitted
 * then stay in the engine. */
int cyrus_engine_run(cyrus_engine* eng, int32_t n, cyrus_codebook* const* cells, const cyrus_ue_state* ues,
                     const double* arrival_us, uint8_t* const* results, double* latency_us);

/* Counters: [0] submitted, [1] completed, [2] steps launched (resident worker:
 * worker launches), [3] admissions
 * deferred for memory, [4] admissions deferred for batch slots,
 * [5] device-pool bytes in use, [6] peak device-pool bytes in use. */
int cyrus_engine_stats(const cyrus_engine* eng, int64_t* counters, int32_t n);

/* Waits for all enqueued work, then frees the engine (not the pools). */
void cyrus_engine_destroy(cyrus_engine* eng);

#ifdef __cplusplus
}
#endif

#endif /* CYRUS_H */
