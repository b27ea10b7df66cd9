// Host side of the C ABI declared in include/cyrus.h: validation, workspace
// carving, weight packing, build orchestration on HIP streams, lookup.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cyrus.h"
#include "cyrus_internal.h"
#include "cyrus_kernels.h"
#include "cyrus_host.h"

using namespace cyrus;

namespace {

thread_local std::string g_err;

int fail(int status, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return status;
}

#define HIP_TRY(call)                                                                                                  \
    do {                                                                                                               \
        hipError_t e_ = (call);                                                                                        \
        if (e_ != hipSuccess)                                                                                          \
            return fail(CYRUS_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));                                 \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Waits for a build's event by polling it for up to 2 ms, then blocks. A
// codebook takes tens of microseconds, and a blocking wait can hand the
// thread to the OS scheduler, whose wake-up alone may cost more than a slot.
hipError_t wait_event(hipEvent_t ev)
{
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t e = hipEventQuery(ev);
        if (e != hipErrorNotReady)
            return e;
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2))
            return hipEventSynchronize(ev);
    }
}

bool is_pow2_float(float v)
{
    if (!(v > 0.f) || !std::isfinite(v))
        return false;
    int e;
    return std::frexp(v, &e) == 0.5f;
}

}  // namespace

namespace cyrus {

int validate_config(const cyrus_config* cfg)
{
    if (!cfg)
        return fail(CYRUS_EINVAL, "config is NULL");
    if (cfg->num_ue < 1 || cfg->num_ue > CYRUS_MAX_UE)
        return fail(CYRUS_ERANGE, "num_ue %d outside [1, %d]", cfg->num_ue, CYRUS_MAX_UE);
    if (cfg->max_arrival < 1 || cfg->max_arrival > 7)
        return fail(CYRUS_ERANGE, "max_arrival %d outside [1, 7]", cfg->max_arrival);
    if (cfg->num_minislots < 1 || cfg->num_minislots > 7)
        return fail(CYRUS_ERANGE, "num_minislots %d outside [1, 7]", cfg->num_minislots);
    if (cfg->rb_per_unit < 1)
        return fail(CYRUS_ERANGE, "rb_per_unit %d < 1", cfg->rb_per_unit);
    if ((int64_t)cfg->num_minislots * cfg->max_arrival * cfg->rb_per_unit > 255)
        return fail(CYRUS_ERANGE, "M*K*U = %d exceeds the 8-bit state range",
                    cfg->num_minislots * cfg->max_arrival * cfg->rb_per_unit);
    if (cfg->num_hidden < 1 || cfg->num_hidden > CYRUS_MAX_HIDDEN)
        return fail(CYRUS_ERANGE, "num_hidden %d outside [1, %d]", cfg->num_hidden, CYRUS_MAX_HIDDEN);
    for (int i = 0; i < cfg->num_hidden; ++i)
        if (cfg->hidden[i] < 32 || cfg->hidden[i] > 512 || cfg->hidden[i] % 32 != 0)
            return fail(CYRUS_ERANGE, "hidden[%d] = %d is not a multiple of 32 in [32, 512]", i, cfg->hidden[i]);
    if (cfg->precision != CYRUS_FP32 && cfg->precision != CYRUS_BF16 && cfg->precision != CYRUS_FP8_E4M3)
        return fail(CYRUS_EINVAL, "unknown precision %d", cfg->precision);
    if (cfg->flags &
        ~(CYRUS_FLAG_EXPORT_LOGITS | CYRUS_FLAG_LEVEL_KERNEL | CYRUS_FLAG_HUNTINGTON_HILL | CYRUS_FLAG_GAUSSIAN_HEAD))
        return fail(CYRUS_EINVAL, "unknown flags 0x%x", cfg->flags);
    return CYRUS_OK;
}

Shape make_shape(const cyrus_config* cfg)
{
    Shape s{};
    s.E = cfg->num_ue;
    s.K = cfg->max_arrival;
    s.M = cfg->num_minislots;
    s.prec = cfg->precision;
    s.n_layers = cfg->num_hidden + 1;
    s.dims[0] = 4 * s.E + 2;
    for (int i = 0; i < cfg->num_hidden; ++i)
        s.dims[i + 1] = cfg->hidden[i];
    s.dims[s.n_layers] = (cfg->flags & CYRUS_FLAG_GAUSSIAN_HEAD) ? 2 * s.E : s.E;
    const int kc = prec_chunk(s.prec);
    s.w_bytes = 0;
    s.staging_floats = 0;
    for (int l = 0; l < s.n_layers; ++l) {
        // FP8 reads its input in pairs of chunks (one 16x16x128 MFMA step).
        // Hidden layers are computed 128 neurons at a time (8 waves x 16): a
        // width that is a multiple of 32 is zero-padded to the next multiple
        // of 128 (zero weights and bias, so the padded neurons are ReLU(0) = 0
        // and add nothing to the next layer).
        s.in_pad[l] = (int)(l == 0 ? align_up(s.dims[l], s.prec == kFP8 ? 2 * kc : kc) : align_up(s.dims[l], 128));
        s.out_pad[l] = (int)align_up(s.dims[l + 1], l + 1 < s.n_layers ? 128 : 16);
        s.w_off[l] = s.w_bytes;
        s.w_bytes += align_up((size_t)s.in_pad[l] * s.out_pad[l] * prec_esize(s.prec), 256);
        s.staging_floats = std::max(s.staging_floats, (size_t)s.in_pad[l] * s.out_pad[l]);
    }
    s.in_pad_d = (int)align_up(s.E + 2, s.prec == kFP8 ? 2 * kc : kc);
    s.w1d_off = s.w_bytes;
    s.w_bytes += align_up((size_t)s.in_pad_d * s.out_pad[0] * prec_esize(s.prec), 256);
    s.staging_floats = std::max(s.staging_floats, (size_t)s.in_pad_d * s.out_pad[0]);
    for (int l = 0; l < s.n_layers; ++l) {
        s.b_off[l] = s.w_bytes;
        s.w_bytes += align_up((size_t)s.out_pad[l] * 4, 256);
    }
    s.nodes = (ipow(s.K + 1, s.M + 1) - 1) / s.K;
    s.export_logits = (cfg->flags & CYRUS_FLAG_EXPORT_LOGITS) != 0;

    size_t off = 0;
    s.off_w[0] = off;
    off += align_up(s.w_bytes, 256);
    s.off_w[1] = off;
    off += align_up(s.w_bytes, 256);
    s.off_staging = off;
    off += align_up(s.staging_floats * 4, 256);
    s.off_ue = off;
    off += align_up(3 * kMaxUE * 4, 256);
    s.off_alloc = off;
    off += align_up((size_t)s.nodes * s.E, 256);
    s.off_state = off;
    off += align_up((size_t)s.nodes * s.E, 256);
    s.off_logits = off;
    if (s.export_logits)
        off += align_up((size_t)s.nodes * s.E * 4, 256);
    s.off_batch = off;
    off += align_up(batch_area_bytes(), 256);
    s.device_bytes = off;

    size_t h = 0;
    s.hoff_ue = h;
    h += align_up(3 * kMaxUE * 4, 64);
    s.hoff_alloc = h;
    h += align_up((size_t)s.nodes * s.E, 64);
    s.hoff_logits = h;
    if (s.export_logits)
        h += align_up((size_t)s.nodes * s.E * 4, 64);
    s.hoff_batch = h;
    h += align_up(batch_area_bytes(), 64);
    s.host_bytes = h;
    return s;
}

size_t batch_area_bytes() { return align_up(sizeof(DevTree) * kMaxBatch, 256) + (size_t)7 * (3 * kMaxBatch + 1) * 4; }

void pack_fragments(const float* w, int out, int in, int out_pad, int in_pad, int prec, float* dst)
{
    const int kc = prec_chunk(prec), per = kc / 4, nch = in_pad / kc, ntiles = out_pad / 16;
    for (int nt = 0; nt < ntiles; ++nt)
        for (int ch = 0; ch < nch; ++ch)
            for (int lane = 0; lane < 64; ++lane) {
                const int n = nt * 16 + (lane & 15);
                for (int j = 0; j < per; ++j) {
                    const int k = ch * kc + (lane >> 4) * per + j;
                    dst[(((size_t)nt * nch + ch) * 64 + lane) * per + j] =
                        (n < out && k < in) ? w[(size_t)n * in + k] : 0.f;
                }
            }
}

float e4m3_weight_scale(const float* w, size_t n)
{
    float amax = 0.f;
    for (size_t i = 0; i < n; ++i)
        amax = std::max(amax, std::fabs(w[i]));
    if (amax == 0.f)
        return 1.f;
    float s = 1.f;
    while (amax / s > 448.f)
        s *= 2.f;
    while (amax / (s * 0.5f) <= 448.f)
        s *= 0.5f;
    return s;
}

int choose_rtt(const DevTree& t, int prec, int max_rtt)
{
    const int cands[] = {6, 4, 2, 1};
    for (int r : cands) {
        if (r > max_rtt || (prec == kFP32 && r > 4))
            continue;
        if (level_lds_bytes(t, prec, r) <= 160 * 1024)
            return r;
    }
    return 0;
}

}  // namespace cyrus


namespace cyrus {

DevTree make_devtree(const cyrus_codebook* cb, const int32_t* ue_dev, int slot)
{
    const Shape& s = cb->s;
    if (slot < 0)
        slot = cb->active;
    DevTree t{};
    t.E = s.E;
    t.K = s.K;
    t.M = s.M;
    t.U = cb->cfg.rb_per_unit;
    t.rounding = (cb->cfg.flags & CYRUS_FLAG_HUNTINGTON_HILL) ? kHuntingtonHill : kLargestRemainder;
    t.head = (cb->cfg.flags & CYRUS_FLAG_GAUSSIAN_HEAD) ? kGaussianHead : kSoftmaxHead;
    t.seed = cb->rng_seed;
    t.tti = cb->rng_tti;
    t.n_layers = s.n_layers;
    t.in_dim0 = s.dims[0];
    const uint8_t* wb = cb->ws + s.off_w[slot];
    for (int l = 0; l < s.n_layers; ++l) {
        t.in_pad[l] = s.in_pad[l];
        t.out_pad[l] = s.out_pad[l];
        t.w[l] = wb + s.w_off[l];
        t.b[l] = reinterpret_cast<const float*>(wb + s.b_off[l]);
        t.deq[l] = cb->deq[slot][l];
        t.inv_in_scale[l] = cb->inv_in[slot][l];
    }
    t.in_pad_d = s.in_pad_d;
    t.w1d = wb + s.w1d_off;
    t.ue = ue_dev;
    t.alloc = cb->ws + s.off_alloc;
    t.state = cb->ws + s.off_state;
    t.logits = s.export_logits ? reinterpret_cast<float*>(cb->ws + s.off_logits) : nullptr;
    return t;
}

hipError_t note_slot_use(cyrus_codebook* cb, int slot, hipStream_t stream)
{
    for (auto& u : cb->slot_use[slot])
        if (u.first == stream)
            return hipEventRecord(u.second, stream);
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess)
        return e;
    e = hipEventRecord(ev, stream);
    if (e != hipSuccess) {
        (void)hipEventDestroy(ev);
        return e;
    }
    cb->slot_use[slot].emplace_back(stream, ev);
    return hipSuccess;
}

hipError_t note_build_use(cyrus_codebook* cb, int slot, hipStream_t stream)
{
    if (cb->done_slot >= 0 && (cb->done_stream != stream || cb->done_slot != slot)) {
        // an event recorded now on the old stream follows every build
        // enqueued there, the one ev_done marked included
        const hipError_t e = note_slot_use(cb, cb->done_slot, cb->done_stream);
        if (e != hipSuccess)
            return e;
    }
    cb->done_stream = stream;
    cb->done_slot = slot;
    return hipSuccess;
}

int codebook_path(const cyrus_codebook* cb) { return cb->path; }
int codebook_rtt(const cyrus_codebook* cb) { return cb->rtt; }
const Shape& codebook_shape(const cyrus_codebook* cb) { return cb->s; }

}  // namespace cyrus

static int load_weights(cyrus_codebook* cb, const cyrus_weights* w, hipStream_t stream, int target)
{
    const Shape& s = cb->s;
    if (!w)
        return fail(CYRUS_EINVAL, "weights are NULL");
    for (int l = 0; l < s.n_layers; ++l)
        if (!w->w[l] || !w->b[l])
            return fail(CYRUS_EINVAL, "weights or bias of layer %d is NULL", l);
    float a_scale[kMaxLayers], w_scale[kMaxLayers];
    for (int l = 0; l < s.n_layers; ++l) {
        a_scale[l] = 1.f;
        w_scale[l] = 1.f;
    }
    if (s.prec == CYRUS_FP8_E4M3) {
        if (!w->act_scale)
            return fail(CYRUS_EINVAL, "FP8 needs act_scale (one power of two per layer input)");
        for (int l = 0; l < s.n_layers; ++l) {
            if (!is_pow2_float(w->act_scale[l]))
                return fail(CYRUS_ERANGE, "act_scale[%d] = %g is not a positive power of two", l,
                            (double)w->act_scale[l]);
            a_scale[l] = w->act_scale[l];
            w_scale[l] = e4m3_weight_scale(w->w[l], (size_t)s.dims[l] * s.dims[l + 1]);
        }
        // the kernels apply each layer's output scale (deq, times the next
        // layer's inverse input scale for a hidden layer) as an E8M0 block
        // scale, which holds the powers of two from 2^-126 to 2^127
        for (int l = 0; l < s.n_layers; ++l) {
            const float c = w_scale[l] * a_scale[l] / (l + 1 < s.n_layers ? a_scale[l + 1] : 1.f);
            if (!(c >= 0x1p-126f && c <= 0x1p127f))
                return fail(CYRUS_ERANGE, "layer %d: weight scale x act_scale[%d] / act_scale[%d] = %g is outside "
                            "2^-126..2^127", l, l, l + 1, (double)c);
        }
    }
    for (int l = 0; l < s.n_layers; ++l)
        for (size_t i = 0; i < (size_t)s.dims[l] * s.dims[l + 1]; ++i)
            if (!std::isfinite(w->w[l][i]))
                return fail(CYRUS_EINVAL, "weight %zu of layer %d is not finite", i, l);

    // builds, batches and engine launches enqueued earlier may still read the
    // buffer about to be overwritten: wait for each stream's last use of it.
    // Engine requests admitted with it may have levels still to enqueue.
    if (cb->engine_refs[target] > 0)
        return fail(CYRUS_ENOTREADY, "%d serving-engine requests still use the weight buffer to be replaced; step "
                    "the engine until they finish", cb->engine_refs[target]);
    for (auto& u : cb->slot_use[target])
        HIP_TRY(hipEventSynchronize(u.second));
    if (cb->done_slot == target)
        HIP_TRY(hipEventSynchronize(cb->done_event()));
    uint8_t* wb = cb->ws + s.off_w[target];
    float* staging = reinterpret_cast<float*>(cb->ws + s.off_staging);
    cb->pack.assign(s.staging_floats, 0.f);
    std::vector<float> bias;
    for (int l = 0; l < s.n_layers; ++l) {
        const size_t n = (size_t)s.in_pad[l] * s.out_pad[l];
        pack_fragments(w->w[l], s.dims[l + 1], s.dims[l], s.out_pad[l], s.in_pad[l], s.prec, cb->pack.data());
        HIP_TRY(hipMemcpyAsync(staging, cb->pack.data(), n * 4, hipMemcpyHostToDevice, stream));
        HIP_TRY(launch_convert_weights(s.prec, staging, wb + s.w_off[l], (int64_t)n, 1.f / w_scale[l], stream));
        bias.assign(s.out_pad[l], 0.f);
        std::memcpy(bias.data(), w->b[l], sizeof(float) * s.dims[l + 1]);
        HIP_TRY(hipMemcpyAsync(wb + s.b_off[l], bias.data(), bias.size() * 4, hipMemcpyHostToDevice, stream));
        // the host staging vectors are reused by the next layer
        HIP_TRY(hipStreamSynchronize(stream));
    }
    {
        // the per-node columns of layer 1 (c, tau, k: the last E + 2), packed
        // on their own with the layer's weight scale
        const int nd = s.E + 2, in0 = s.dims[0], h1 = s.dims[1];
        std::vector<float> wd((size_t)h1 * nd);
        for (int n = 0; n < h1; ++n)
            for (int j = 0; j < nd; ++j)
                wd[(size_t)n * nd + j] = w->w[0][(size_t)n * in0 + 3 * s.E + j];
        const size_t n = (size_t)s.in_pad_d * s.out_pad[0];
        pack_fragments(wd.data(), h1, nd, s.out_pad[0], s.in_pad_d, s.prec, cb->pack.data());
        HIP_TRY(hipMemcpyAsync(staging, cb->pack.data(), n * 4, hipMemcpyHostToDevice, stream));
        HIP_TRY(launch_convert_weights(s.prec, staging, wb + s.w1d_off, (int64_t)n, 1.f / w_scale[0], stream));
        HIP_TRY(hipStreamSynchronize(stream));
    }
    for (int l = 0; l < s.n_layers; ++l) {
        cb->deq[target][l] = w_scale[l] * a_scale[l];
        cb->inv_in[target][l] = 1.f / a_scale[l];
    }
    cb->active = target;
    cb->wversion++;
    return CYRUS_OK;
}

// The launches of one build. done (nullable) completes with the last launch
// (it rides on that dispatch rather than following it as a separate marker).
static int enqueue_tree(cyrus_codebook* cb, const DevTree& t, hipStream_t stream, hipEvent_t done)
{
    if (cb->path == 1)
        HIP_TRY(launch_subtree(t, cb->s.prec, stream, done));
    else
        for (int tau = 1; tau <= cb->s.M; ++tau)
            HIP_TRY(launch_level(t, cb->s.prec, cb->rtt, tau, stream, tau == cb->s.M ? done : nullptr));
    return CYRUS_OK;
}

// The kernels of one build, `done` completing with the last of them.
static int enqueue_kernels(cyrus_codebook* cb, const int32_t* ue_dev, hipStream_t stream, hipEvent_t done)
{
    int rc = enqueue_tree(cb, make_devtree(cb, ue_dev), stream, done);
    if (rc)
        return rc;
    HIP_TRY(note_build_use(cb, cb->active, stream));
    return CYRUS_OK;
}

extern "C" {

int cyrus_codebook_workspace_size(const cyrus_config* cfg, size_t* device_bytes, size_t* host_bytes)
{
    int rc = validate_config(cfg);
    if (rc)
        return rc;
    if (!device_bytes || !host_bytes)
        return fail(CYRUS_EINVAL, "output pointers are NULL");
    const Shape s = make_shape(cfg);
    *device_bytes = s.device_bytes;
    *host_bytes = s.host_bytes;
    return CYRUS_OK;
}

int cyrus_codebook_create(const cyrus_config* cfg, const cyrus_weights* w, void* device_ws, size_t ws_bytes,
                          void* host_pinned, size_t host_bytes, void* stream, cyrus_codebook** out)
{
    int rc = validate_config(cfg);
    if (rc)
        return rc;
    if (!out || !device_ws || !host_pinned)
        return fail(CYRUS_EINVAL, "out, device_ws or host_pinned is NULL");
    const Shape s = make_shape(cfg);
    if (ws_bytes < s.device_bytes || host_bytes < s.host_bytes)
        return fail(CYRUS_EWORKSPACE, "workspace %zu/%zu bytes, need %zu/%zu", ws_bytes, host_bytes, s.device_bytes,
                    s.host_bytes);
    if (reinterpret_cast<uintptr_t>(device_ws) % 256 || reinterpret_cast<uintptr_t>(host_pinned) % 64)
        return fail(CYRUS_EWORKSPACE, "workspace must be 256-byte aligned and the host buffer 64-byte aligned");
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, device_ws) != hipSuccess ||
        (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged && attr.type != hipMemoryTypeUnified)) {
        (void)hipGetLastError();
        return fail(CYRUS_EWORKSPACE, "device_ws is not device memory known to this HIP runtime");
    }
    if (hipPointerGetAttributes(&attr, host_pinned) != hipSuccess || attr.type != hipMemoryTypeHost) {
        (void)hipGetLastError();
        return fail(CYRUS_EWORKSPACE, "host_pinned is not page-locked host memory known to this HIP runtime");
    }
    cyrus_codebook* cb = new (std::nothrow) cyrus_codebook();
    if (!cb)
        return fail(CYRUS_EINVAL, "out of host memory");
    cb->cfg = *cfg;
    cb->s = s;
    cb->ws = static_cast<uint8_t*>(device_ws);
    cb->host = static_cast<uint8_t*>(host_pinned);
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto cleanup = [&](int status) {
        if (cb->ev_staged)
            (void)hipEventDestroy(cb->ev_staged);
        if (cb->ev_done)
            (void)hipEventDestroy(cb->ev_done);
        delete cb;
        return status;
    };
    if (hipHostGetDevicePointer(reinterpret_cast<void**>(&cb->host_dev), host_pinned, 0) != hipSuccess) {
        (void)hipGetLastError();
        cb->host_dev = nullptr;
    }
    if (hipGetDevice(&cb->device) != hipSuccess || hipEventCreateWithFlags(&cb->ev_staged, hipEventDisableTiming) ||
        hipEventCreateWithFlags(&cb->ev_done, hipEventDisableTiming))
        return cleanup(fail(CYRUS_EDEVICE, "event creation failed"));
    // root row: punctures nothing, state zero
    if (hipMemsetAsync(cb->ws + s.off_alloc, 0, s.E, st) != hipSuccess ||
        hipMemsetAsync(cb->ws + s.off_state, 0, s.E, st) != hipSuccess ||
        (s.export_logits && hipMemsetAsync(cb->ws + s.off_logits, 0, (size_t)s.E * 4, st) != hipSuccess))
        return cleanup(fail(CYRUS_EDEVICE, "workspace clear failed"));
    // the pinned mirror starts as an all-zero codebook: the single-launch path
    // writes it directly and never writes the root row
    std::memset(cb->host + s.hoff_alloc, 0, (size_t)s.nodes * s.E);
    if (s.export_logits)
        std::memset(cb->host + s.hoff_logits, 0, (size_t)s.nodes * s.E * 4);
    rc = load_weights(cb, w, st, 0);
    if (rc)
        return cleanup(rc);
    const DevTree t = make_devtree(cb, nullptr);
    cb->path = (!(cfg->flags & CYRUS_FLAG_LEVEL_KERNEL) && subtree_supported(t, s.prec)) ? 1 : 0;
    cb->rtt = choose_rtt(t, s.prec, 4);
    if (cb->rtt == 0)
        return cleanup(fail(CYRUS_EUNSUPPORTED, "shape does not fit the level kernel's LDS"));
    *out = cb;
    return CYRUS_OK;
}

int cyrus_codebook_set_weights(cyrus_codebook* cb, const cyrus_weights* w, void* stream)
{
    if (!cb)
        return fail(CYRUS_EINVAL, "handle is NULL");
    HIP_TRY(hipSetDevice(cb->device));
    return load_weights(cb, w, static_cast<hipStream_t>(stream), 1 - cb->active);
}

static int stage_ue(cyrus_codebook* cb, const cyrus_ue_state* ue)
{
    const int E = cb->s.E;
    if (!ue || !ue->rb || !ue->mcs || !ue->sinr_db)
        return fail(CYRUS_EINVAL, "UE state or one of its arrays is NULL");
    for (int e = 0; e < E; ++e) {
        if (ue->rb[e] < 0 || ue->rb[e] > 255)
            return fail(CYRUS_ERANGE, "rb[%d] = %d outside [0, 255]", e, ue->rb[e]);
        if (!std::isfinite(ue->sinr_db[e]))
            return fail(CYRUS_EINVAL, "sinr_db[%d] is not finite", e);
    }
    if (cb->staged_is_done)
        HIP_TRY(wait_event(cb->done_event()));
    else if (cb->staged_recorded)
        HIP_TRY(hipEventSynchronize(cb->ev_staged));
    int32_t* st = reinterpret_cast<int32_t*>(cb->host + cb->s.hoff_ue);
    for (int e = 0; e < E; ++e) {
        st[e] = ue->rb[e];
        st[E + e] = ue->mcs[e];
        std::memcpy(&st[2 * E + e], &ue->sinr_db[e], 4);
    }
    return CYRUS_OK;
}

int cyrus_codebook_build(cyrus_codebook* cb, const cyrus_ue_state* ue, void* stream)
{
    if (!cb)
        return fail(CYRUS_EINVAL, "handle is NULL");
    HIP_TRY(hipSetDevice(cb->device));
    int rc = stage_ue(cb, ue);
    if (rc)
        return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Shape& s = cb->s;
    if (cb->path == 1 && cb->host_dev) {
        // one launch, no copies: the kernel reads s(t) from the pinned buffer
        // and writes the codebook (and logits) straight into the pinned mirror
        DevTree t = make_devtree(cb, reinterpret_cast<const int32_t*>(cb->host_dev + s.hoff_ue));
        t.alloc = cb->host_dev + s.hoff_alloc;
        t.logits = s.export_logits ? reinterpret_cast<float*>(cb->host_dev + s.hoff_logits) : nullptr;
        // ev_done completes with the launch; the kernel reads the staged UE
        // state, so ev_done also releases it
        cb->batch_done.reset();
        rc = enqueue_tree(cb, t, st, cb->ev_done);
        if (rc)
            return rc;
        HIP_TRY(note_build_use(cb, cb->active, st));
        cb->staged_is_done = true;
        cb->built = cb->pending = cb->mirror_valid = true;
        return CYRUS_OK;
    }
    int32_t* ue_dev = reinterpret_cast<int32_t*>(cb->ws + s.off_ue);
    HIP_TRY(hipMemcpyAsync(ue_dev, cb->host + s.hoff_ue, (size_t)3 * s.E * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(cb->ev_staged, st));
    cb->staged_recorded = true;
    cb->staged_is_done = false;
    cb->batch_done.reset();
    if (cb->host_dev) {
        // level path, no copies back: the UE state goes to the device once
        // (every tile of every level reads it), and the level kernels write
        // the codebook (and logits) straight into the pinned mirror, whose
        // root row is zero from create; ev_done completes with the last level
        DevTree t = make_devtree(cb, ue_dev);
        t.alloc = cb->host_dev + s.hoff_alloc;
        t.logits = s.export_logits ? reinterpret_cast<float*>(cb->host_dev + s.hoff_logits) : nullptr;
        rc = enqueue_tree(cb, t, st, cb->ev_done);
        if (rc)
            return rc;
        HIP_TRY(note_build_use(cb, cb->active, st));
        cb->built = cb->pending = cb->mirror_valid = true;
        return CYRUS_OK;
    }
    rc = enqueue_kernels(cb, ue_dev, st, nullptr);
    if (rc)
        return rc;
    HIP_TRY(hipMemcpyAsync(cb->host + s.hoff_alloc, cb->ws + s.off_alloc, (size_t)s.nodes * s.E,
                           hipMemcpyDeviceToHost, st));
    if (s.export_logits)
        HIP_TRY(hipMemcpyAsync(cb->host + s.hoff_logits, cb->ws + s.off_logits, (size_t)s.nodes * s.E * 4,
                               hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(cb->ev_done, st));
    cb->built = cb->pending = cb->mirror_valid = true;
    return CYRUS_OK;
}

int cyrus_codebook_build_device(cyrus_codebook* cb, const void* ue_device, void* stream)
{
    if (!cb || !ue_device)
        return fail(CYRUS_EINVAL, "handle or UE pointer is NULL");
    if (reinterpret_cast<uintptr_t>(ue_device) % 4)
        return fail(CYRUS_EINVAL, "UE state must be 4-byte aligned");
    HIP_TRY(hipSetDevice(cb->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    cb->batch_done.reset();
    int rc = enqueue_kernels(cb, static_cast<const int32_t*>(ue_device), st, cb->ev_done);  // ev_done rides on the last launch
    if (rc)
        return rc;
    cb->built = cb->pending = true;
    cb->mirror_valid = false;
    return CYRUS_OK;
}

int cyrus_codebook_wait(cyrus_codebook* cb)
{
    if (!cb)
        return fail(CYRUS_EINVAL, "handle is NULL");
    if (cb->pending) {
        HIP_TRY(wait_event(cb->done_event()));
        cb->pending = false;
    }
    return CYRUS_OK;
}

// Wait for the last build, then make sure the pinned mirror holds it (a
// device build leaves the codebook in the workspace only).
static int sync_mirror(const cyrus_codebook* cb)
{
    if (!cb->built)
        return fail(CYRUS_ENOTREADY, "no build has been enqueued on this handle");
    if (cb->pending) {
        HIP_TRY(wait_event(cb->done_event()));
        cb->pending = false;
    }
    if (!cb->mirror_valid) {
        const Shape& s = cb->s;
        HIP_TRY(hipSetDevice(cb->device));
        HIP_TRY(hipMemcpy(cb->host + s.hoff_alloc, cb->ws + s.off_alloc, (size_t)s.nodes * s.E,
                          hipMemcpyDeviceToHost));
        if (s.export_logits)
            HIP_TRY(hipMemcpy(cb->host + s.hoff_logits, cb->ws + s.off_logits, (size_t)s.nodes * s.E * 4,
                              hipMemcpyDeviceToHost));
        cb->mirror_valid = true;
    }
    return CYRUS_OK;
}

int cyrus_codebook_lookup(const cyrus_codebook* cb, const uint8_t* arrivals, int32_t tau, uint8_t* alloc_out)
{
    if (!cb || !alloc_out || (tau > 0 && !arrivals))
        return fail(CYRUS_EINVAL, "NULL argument");
    const Shape& s = cb->s;
    if (tau < 1 || tau > s.M)
        return fail(CYRUS_ERANGE, "tau %d outside [1, %d]", tau, s.M);
    int64_t idx = 0;
    for (int i = 0; i < tau; ++i) {
        if (arrivals[i] > s.K)
            return fail(CYRUS_ERANGE, "arrivals[%d] = %d exceeds K = %d", i, arrivals[i], s.K);
        idx = idx * (s.K + 1) + arrivals[i];
    }
    int rc = sync_mirror(cb);
    if (rc)
        return rc;
    const int64_t node = (ipow(s.K + 1, tau) - 1) / s.K + idx;
    std::memcpy(alloc_out, cb->host + s.hoff_alloc + node * s.E, s.E);
    return CYRUS_OK;
}

int cyrus_codebook_assemble(const cyrus_codebook* cb, const int32_t* raw_arrivals, int32_t carry_in, uint8_t* served,
                            uint8_t* y, int32_t* carry_out)
{
    if (!cb || !raw_arrivals || !served || !y || !carry_out)
        return fail(CYRUS_EINVAL, "NULL argument");
    const Shape& s = cb->s;
    if (carry_in < 0)
        return fail(CYRUS_ERANGE, "carry_in %d < 0", carry_in);
    for (int tau = 0; tau < s.M; ++tau)
        if (raw_arrivals[tau] < 0)
            return fail(CYRUS_ERANGE, "raw_arrivals[%d] = %d < 0", tau, raw_arrivals[tau]);
    int rc = sync_mirror(cb);
    if (rc)
        return rc;
    int64_t backlog = carry_in, idx = 0;
    for (int tau = 1; tau <= s.M; ++tau) {
        const int64_t want = raw_arrivals[tau - 1] + backlog;
        const int k = (int)std::min<int64_t>(want, s.K);
        backlog = want - k;
        served[tau - 1] = (uint8_t)k;
        idx = idx * (s.K + 1) + k;
        const int64_t node = (ipow(s.K + 1, tau) - 1) / s.K + idx;
        std::memcpy(y + (size_t)(tau - 1) * s.E, cb->host + s.hoff_alloc + node * s.E, s.E);
    }
    *carry_out = (int32_t)std::min<int64_t>(backlog, INT32_MAX);
    return CYRUS_OK;
}

int cyrus_codebook_export(const cyrus_codebook* cb, uint8_t* alloc, float* logits)
{
    if (!cb || !alloc)
        return fail(CYRUS_EINVAL, "NULL argument");
    const Shape& s = cb->s;
    if (logits && !s.export_logits)
        return fail(CYRUS_EINVAL, "logits requested but CYRUS_FLAG_EXPORT_LOGITS is not set");
    int rc = sync_mirror(cb);
    if (rc)
        return rc;
    std::memcpy(alloc, cb->host + s.hoff_alloc, (size_t)s.nodes * s.E);
    if (logits)
        std::memcpy(logits, cb->host + s.hoff_logits, (size_t)s.nodes * s.E * 4);
    return CYRUS_OK;
}

const uint8_t* cyrus_codebook_device_alloc(const cyrus_codebook* cb)
{
    return cb ? cb->ws + cb->s.off_alloc : nullptr;
}

int64_t cyrus_codebook_num_nodes(const cyrus_codebook* cb) { return cb ? cb->s.nodes : -1; }

const char* cyrus_codebook_kernel_path(const cyrus_codebook* cb)
{
    if (!cb)
        return "none";
    return cb->path == 1 ? "subtree" : "level";
}

int cyrus_codebook_set_rng(cyrus_codebook* cb, uint64_t seed, uint64_t tti)
{
    if (!cb)
        return fail(CYRUS_EINVAL, "handle is NULL");
    cb->rng_seed = seed;
    cb->rng_tti = tti;
    return CYRUS_OK;
}

void cyrus_codebook_destroy(cyrus_codebook* cb)
{
    if (!cb)
        return;
    (void)hipSetDevice(cb->device);
    if (cb->pending)
        (void)hipEventSynchronize(cb->done_event());
    if (cb->staged_recorded)
        (void)hipEventSynchronize(cb->ev_staged);
    (void)hipEventDestroy(cb->ev_staged);
    (void)hipEventDestroy(cb->ev_done);
    for (auto& uses : cb->slot_use)
        for (auto& u : uses) {
            (void)hipEventSynchronize(u.second);
            (void)hipEventDestroy(u.second);
        }
    delete cb;
}

const char* cyrus_status_string(int status)
{
    switch (status) {
    case CYRUS_OK:
        return "ok";
    case CYRUS_EINVAL:
        return "invalid argument";
    case CYRUS_ERANGE:
        return "value out of range";
    case CYRUS_EWORKSPACE:
        return "workspace too small or misplaced";
    case CYRUS_EDEVICE:
        return "HIP runtime error";
    case CYRUS_ENOTREADY:
        return "no build yet";
    case CYRUS_EUNSUPPORTED:
        return "unsupported shape";
    default:
        return "unknown status";
    }
}

const char* cyrus_last_error(void) { return g_err.c_str(); }

#ifndef CYRUS_SOURCE_HASH
#define CYRUS_SOURCE_HASH "unknown"
#endif
const char* cyrus_build_source_hash(void) { return CYRUS_SOURCE_HASH; }

}  // extern "C"

// Shared with the batch builder.
namespace cyrus {
int set_error(int status, const char* msg) { return fail(status, "%s", msg); }
int stage_ue_host(cyrus_codebook* cb, const cyrus_ue_state* ue) { return stage_ue(cb, ue); }
}  // namespace cyrus
