// Critic pass of the C ABI: configuration checks, the five networks' packed
// FP32 weights and descriptors in the caller's workspace, and the launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "cyrus.h"
#include "cyrus_host.h"
#include "cyrus_kernels.h"

using namespace cyrus;

struct cyrus_critic {
    cyrus_critic_config cfg;
    int device = 0;
    uint8_t* ws = nullptr;
    const DevTree* nets = nullptr;  // in the workspace
    float* tgt = nullptr;           // per-row target scratch in the workspace: [3][H M]
    int rtt = 1;
    int regs_t = 0, regs_ch1 = 0;  // register-resident kernel: tiles per wave, first-layer chunks (0: streamed)
    size_t lds = 0;
    int bufsize = 0;
    int bias_off[5] = {0};
    int bias_total = 0;
};

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int fail_msg(int status, const char* msg) { return set_error(status, msg); }

int hip_fail(hipError_t e, const char* what)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s failed: %s", what, hipGetErrorString(e));
    return set_error(CYRUS_EDEVICE, buf);
}

// Layer widths of net n: 0 actor, 1..4 critics.
struct NetShape {
    int n_layers;
    int dims[kMaxLayers + 1];
    int in_pad[kMaxLayers], out_pad[kMaxLayers];
    size_t w_off[kMaxLayers], b_off[kMaxLayers];
};

struct CriticLayout {
    NetShape net[5];
    int regs_t, regs_ch1;  // register-resident kernel shape, or 0
    size_t nets_off;  // DevTree[5]
    size_t tgt_off;   // float[3][H M]: both target critics and log pi, per row
    size_t bytes;
};

int check_hidden(int n, const int32_t* h, const char* what)
{
    if (n < 1 || n > CYRUS_MAX_HIDDEN) {
        char buf[128];
        snprintf(buf, sizeof buf, "%s_hidden_layers = %d outside [1, %d]", what, n, CYRUS_MAX_HIDDEN);
        return fail_msg(CYRUS_ERANGE, buf);
    }
    for (int i = 0; i < n; ++i)
        if (h[i] < 32 || h[i] > 512 || h[i] % 32) {
            char buf[128];
            snprintf(buf, sizeof buf, "%s_hidden[%d] = %d is not a multiple of 32 in [32, 512]", what, i, h[i]);
            return fail_msg(CYRUS_ERANGE, buf);
        }
    return CYRUS_OK;
}

int validate(const cyrus_critic_config* c)
{
    if (!c)
        return fail_msg(CYRUS_EINVAL, "config is NULL");
    if (c->num_ue < 1 || c->num_ue > 16)
        return fail_msg(CYRUS_ERANGE, "num_ue outside [1, 16]");
    if (c->num_minislots < 1 || c->num_minislots > 7)
        return fail_msg(CYRUS_ERANGE, "num_minislots outside [1, 7]");
    if (c->num_samples < 1 || (int64_t)c->num_samples * c->num_minislots > (1 << 24))
        return fail_msg(CYRUS_ERANGE, "num_samples outside [1, 2^24 / num_minislots]");
    if (!std::isfinite(c->discount) || !std::isfinite(c->entropy_coef))
        return fail_msg(CYRUS_EINVAL, "discount and entropy_coef must be finite");
    int rc = check_hidden(c->actor_hidden_layers, c->actor_hidden, "actor");
    return rc ? rc : check_hidden(c->critic_hidden_layers, c->critic_hidden, "critic");
}

// Hidden layers are computed 128 neurons at a time: a width that is a
// multiple of 32 is zero-padded to the next multiple of 128 (zero weights and
// bias, so a padded neuron is ReLU(0) = 0 and its zero outgoing weights add
// nothing to the next layer).
int hidden_pad(int h) { return (int)align_up(h, 128); }

// The register-resident critic kernel takes two hidden layers of one padded
// width H in {128, 256} in all five networks and at most 16 actor outputs
// (E <= 8); every network's first layer is then padded to the critics' 5E+2
// inputs.
bool regs_shape(const cyrus_critic_config* c, int* H)
{
    const int h = hidden_pad(c->actor_hidden[0]);
    *H = h;
    return c->actor_hidden_layers == 2 && c->critic_hidden_layers == 2 && (h == 128 || h == 256) &&
           hidden_pad(c->actor_hidden[1]) == h && hidden_pad(c->critic_hidden[0]) == h &&
           hidden_pad(c->critic_hidden[1]) == h && 2 * c->num_ue <= 16;
}

CriticLayout layout(const cyrus_critic_config* c)
{
    CriticLayout L{};
    const int E = c->num_ue;
    int H = 0;
    const bool regs = regs_shape(c, &H);
    const int in0 = (int)align_up(5 * E + 2, 16);
    L.regs_t = regs ? H / 128 : 0;
    L.regs_ch1 = regs ? in0 / 16 : 0;
    size_t off = 0;
    for (int n = 0; n < 5; ++n) {
        NetShape& s = L.net[n];
        const bool actor = n == 0;
        const int nh = actor ? c->actor_hidden_layers : c->critic_hidden_layers;
        const int32_t* hw = actor ? c->actor_hidden : c->critic_hidden;
        s.n_layers = nh + 1;
        s.dims[0] = actor ? 4 * E + 2 : 5 * E + 2;
        for (int i = 0; i < nh; ++i)
            s.dims[i + 1] = hw[i];
        s.dims[nh + 1] = actor ? 2 * E : 1;
        for (int l = 0; l < s.n_layers; ++l) {
            s.in_pad[l] = l == 0 ? (regs ? in0 : (int)align_up(s.dims[0], 16)) : hidden_pad(s.dims[l]);
            s.out_pad[l] = l < nh ? hidden_pad(s.dims[l + 1]) : (int)align_up(s.dims[l + 1], 16);
            s.w_off[l] = off;
            off = align_up(off + (size_t)s.in_pad[l] * s.out_pad[l] * 4, 256);
            s.b_off[l] = off;
            off = align_up(off + (size_t)s.out_pad[l] * 4, 256);
        }
    }
    L.nets_off = off;
    L.tgt_off = align_up(off + sizeof(DevTree) * 5, 256);
    L.bytes = align_up(L.tgt_off + (size_t)3 * c->num_samples * c->num_minislots * 4, 256);
    return L;
}

}  // namespace

extern "C" int cyrus_critic_workspace_size(const cyrus_critic_config* cfg, size_t* device_bytes)
{
    int rc = validate(cfg);
    if (rc)
        return rc;
    if (!device_bytes)
        return fail_msg(CYRUS_EINVAL, "device_bytes is NULL");
    *device_bytes = layout(cfg).bytes;
    return CYRUS_OK;
}

extern "C" int cyrus_critic_create(const cyrus_critic_config* cfg, const cyrus_critic_weights* w, void* device_ws,
                                   size_t ws_bytes, void* stream, cyrus_critic** out)
{
    int rc = validate(cfg);
    if (rc)
        return rc;
    if (!w || !device_ws || !out)
        return fail_msg(CYRUS_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(device_ws) % 256)
        return fail_msg(CYRUS_EWORKSPACE, "device_ws must be 256-byte aligned");
    const CriticLayout L = layout(cfg);
    if (ws_bytes < L.bytes)
        return fail_msg(CYRUS_EWORKSPACE, "device workspace smaller than cyrus_critic_workspace_size");
    const cyrus_weights* nets_w[5] = {&w->actor, &w->q[0], &w->q[1], &w->q_targ[0], &w->q_targ[1]};
    for (int n = 0; n < 5; ++n)
        for (int l = 0; l < L.net[n].n_layers; ++l) {
            if (!nets_w[n]->w[l] || !nets_w[n]->b[l])
                return fail_msg(CYRUS_EINVAL, "a weight or bias pointer is NULL");
            const size_t cnt = (size_t)L.net[n].dims[l] * L.net[n].dims[l + 1];
            for (size_t i = 0; i < cnt; ++i)
                if (!std::isfinite(nets_w[n]->w[l][i]))
                    return fail_msg(CYRUS_EINVAL, "a weight is not finite");
        }
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, device_ws) != hipSuccess ||
        (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged && attr.type != hipMemoryTypeUnified))
        return fail_msg(CYRUS_EINVAL, "device_ws is not device memory");

    cyrus_critic* cr = new (std::nothrow) cyrus_critic();
    if (!cr)
        return fail_msg(CYRUS_EINVAL, "out of host memory");
    cr->cfg = *cfg;
    cr->ws = static_cast<uint8_t*>(device_ws);
    hipError_t e = hipGetDevice(&cr->device);
    if (e != hipSuccess) {
        delete cr;
        return hip_fail(e, "hipGetDevice");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    DevTree nets[5];
    std::vector<float> pack, bias;
    int boff = 0;
    size_t stride = 0, part = 0;
    for (int n = 0; n < 5; ++n) {
        const NetShape& s = L.net[n];
        DevTree& t = nets[n];
        t = DevTree{};
        t.E = s.dims[s.n_layers];  // number of outputs
        t.K = 1;
        t.M = 1;
        t.n_layers = s.n_layers;
        t.in_dim0 = s.dims[0];
        t.head = kSoftmaxHead;
        cr->bias_off[n] = boff;
        for (int l = 0; l < s.n_layers; ++l) {
            t.in_pad[l] = s.in_pad[l];
            t.out_pad[l] = s.out_pad[l];
            t.w[l] = cr->ws + s.w_off[l];
            t.b[l] = reinterpret_cast<const float*>(cr->ws + s.b_off[l]);
            t.deq[l] = 1.f;
            t.inv_in_scale[l] = 1.f;
            if (l == 0) {  // the register-resident kernel loads layer 1 through these
                t.w1d = t.w[0];
                t.in_pad_d = t.in_pad[0];
            }
            boff += s.out_pad[l];
            stride = std::max(stride, (size_t)s.in_pad[l] * 4 + 16);
            pack.assign((size_t)s.in_pad[l] * s.out_pad[l], 0.f);
            pack_fragments(nets_w[n]->w[l], s.dims[l + 1], s.dims[l], s.out_pad[l], s.in_pad[l], kFP32, pack.data());
            bias.assign(s.out_pad[l], 0.f);
            std::memcpy(bias.data(), nets_w[n]->b[l], sizeof(float) * s.dims[l + 1]);
            e = hipMemcpyAsync(cr->ws + s.w_off[l], pack.data(), pack.size() * 4, hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(cr->ws + s.b_off[l], bias.data(), bias.size() * 4, hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = hipStreamSynchronize(st);  // the host vectors are reused by the next layer
            if (e != hipSuccess) {
                delete cr;
                return hip_fail(e, "weight upload");
            }
        }
        part = std::max(part, (size_t)s.out_pad[s.n_layers - 1]);
    }
    cr->bias_total = boff;
    cr->nets = reinterpret_cast<const DevTree*>(cr->ws + L.nets_off);
    cr->tgt = reinterpret_cast<float*>(cr->ws + L.tgt_off);
    e = hipMemcpyAsync(cr->ws + L.nets_off, nets, sizeof nets, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete cr;
        return hip_fail(e, "descriptor upload");
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, cr->device) != hipSuccess || ncu < 1)
        ncu = 256;
    const int64_t rows = (int64_t)cfg->num_samples * cfg->num_minislots;
    cr->rtt = 0;
    if (L.regs_t) {
        // register-resident kernel: 32-row tiles; the output partials of a
        // pass take 8 waves x 48 rows x 16 floats of one activation buffer
        const size_t buf = align_up(std::max(stride * 32, (size_t)kWaves * 48 * 16 * 4), 16);
        const size_t lds = critic_lds_bytes((int)buf, cr->bias_total, 2);
        if (lds <= 160 * 1024) {
            cr->rtt = 2;
            cr->bufsize = (int)buf;
            cr->lds = lds;
            cr->regs_t = L.regs_t;
            cr->regs_ch1 = L.regs_ch1;
        }
    }
    // streamed-weight kernel: row tiles per workgroup (four workgroups per
    // tile, one per role): the smallest whose LDS fits and whose grid runs in
    // one round on the CUs; the largest that fits when none gives one round
    for (int r : {1, 2, 4}) {
        if (cr->regs_t)
            break;
        const size_t rt = 16 * (size_t)r;
        const size_t buf = align_up(std::max(stride * rt, (size_t)kWaves * rt * part * 4), 16);
        const size_t lds = critic_lds_bytes((int)buf, cr->bias_total, r);
        if (lds > 160 * 1024)
            continue;
        cr->rtt = r;
        cr->bufsize = (int)buf;
        cr->lds = lds;
        if (4 * ((rows + (int64_t)rt - 1) / (int64_t)rt) <= ncu)
            break;
    }
    if (!cr->rtt) {
        delete cr;
        return fail_msg(CYRUS_EUNSUPPORTED, "critic networks do not fit the kernel's LDS");
    }
    *out = cr;
    return CYRUS_OK;
}

namespace {

// Per-row target scratch of cyrus_critic_evaluate_noalloc, [3][rows] floats
// (both target critics, then log pi), for at most kNoAllocMaxRows rows. Each
// device holds its own copy for the life of the process; host code reaches it
// only through the address hipGetSymbolAddress returns on that device.
constexpr int64_t kNoAllocMaxRows = 1 << 16;
static __device__ __align__(256) float scratch[3 * kNoAllocMaxRows];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// The scratch address on `dev` (which must be current), looked up once.
int scratch_on(int dev, float** out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return fail_msg(CYRUS_ERANGE, "device ordinal beyond the no-alloc scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return CYRUS_OK;
}

// Both critic entry points: the pass over `b` with the per-row targets in
// `tgt` ([3][H M] floats).
int critic_run(cyrus_critic* cr, const cyrus_critic_batch* b, uint64_t seed, uint64_t episode, float* q, float* qhat,
               float* loss, float* tgt, hipStream_t stream)
{
    CriticArgs a{};
    a.nets = cr->nets;
    a.ue = b->ue;
    a.k = b->k;
    a.c = b->c;
    a.y = b->y;
    a.reward = b->reward;
    a.q = q;
    a.qhat = qhat;
    a.loss = loss;
    const int64_t rows = (int64_t)cr->cfg.num_samples * cr->cfg.num_minislots;
    a.tq = tgt;
    a.tlp = tgt + 2 * rows;
    a.E = cr->cfg.num_ue;
    a.M = cr->cfg.num_minislots;
    a.H = cr->cfg.num_samples;
    a.discount = cr->cfg.discount;
    a.entropy_coef = cr->cfg.entropy_coef;
    a.seed = seed;
    a.episode = episode;
    a.bufsize = cr->bufsize;
    for (int n = 0; n < 5; ++n)
        a.bias_off[n] = cr->bias_off[n];
    a.bias_total = cr->bias_total;
    const hipError_t e = launch_critic(a, cr->rtt, cr->regs_t, cr->regs_ch1, cr->lds, stream);
    if (e != hipSuccess)
        return hip_fail(e, "critic launch");
    return CYRUS_OK;
}

}  // namespace

extern "C" int cyrus_critic_evaluate(cyrus_critic* cr, const cyrus_critic_batch* b, uint64_t seed, uint64_t episode,
                                     float* q, float* qhat, float* loss, void* stream)
{
    if (!cr || !b || !b->ue || !b->k || !b->c || !b->y || !b->reward || !q || !qhat || !loss)
        return fail_msg(CYRUS_EINVAL, "NULL argument");
    hipError_t e = hipSetDevice(cr->device);
    if (e != hipSuccess)
        return hip_fail(e, "hipSetDevice");
    return critic_run(cr, b, seed, episode, q, qhat, loss, cr->tgt, static_cast<hipStream_t>(stream));
}

extern "C" int cyrus_critic_evaluate_noalloc(cyrus_critic* cr, const cyrus_critic_batch* b, uint64_t seed,
                                             uint64_t episode, float* q, float* qhat, float* loss, void* stream)
{
    if (!cr || !b || !b->ue || !b->k || !b->c || !b->y || !b->reward || !q || !qhat || !loss)
        return fail_msg(CYRUS_EINVAL, "NULL argument");
    const int64_t rows = (int64_t)cr->cfg.num_samples * cr->cfg.num_minislots;
    if (rows > kNoAllocMaxRows) {
        char buf[160];
        snprintf(buf, sizeof buf, "%lld rows (samples x steps) exceed the no-alloc scratch limit of %lld",
                 (long long)rows, (long long)kNoAllocMaxRows);
        return fail_msg(CYRUS_ERANGE, buf);
    }
    hipError_t e = hipSetDevice(cr->device);
    if (e != hipSuccess)
        return hip_fail(e, "hipSetDevice");
    float* tgt = nullptr;
    const int rc = scratch_on(cr->device, &tgt);
    if (rc)
        return rc;
    // every row's targets are written by the main kernel before the loss
    // kernel reads them, so the scratch needs no clearing between calls
    return critic_run(cr, b, seed, episode, q, qhat, loss, tgt, static_cast<hipStream_t>(stream));
}

extern "C" void cyrus_critic_destroy(cyrus_critic* cr) { delete cr; }
