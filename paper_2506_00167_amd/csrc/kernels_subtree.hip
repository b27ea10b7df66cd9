// Subtree kernel: the whole codebook in ONE launch, for actors whose weights
// fit in the register file of one CU (hidden width 128 or 256, up to two
// hidden layers, E <= 16). The tree is cut at level L: workgroup r (one per
// CU) runs the subtree algorithm (cyrus_subtree.h) for the subtree below node
// r of level L.
#include <hip/hip_ext.h>

#include "cyrus_device.h"
#include "cyrus_host.h"
#include "cyrus_subtree.h"

namespace cyrus {

namespace {

// EXT: the options beyond softmax logits and largest remainder (the Gaussian
// head, whose 2E outputs fit the one output tile for E <= 8, and
// Huntington-Hill rounding) are compiled into a separate kernel, so the
// default kernel carries none of their code or registers.
template <int P, int T, int CH1, int CHH, int NHH, bool EXT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 2))) void subtree_kernel(
    DevTree t, int split, int bufsize, int stbytes)
{
    extern __shared__ __align__(16) uint8_t smem[];
    if (t.E <= 8)
        subtree_body<P, T, CH1, CHH, NHH, 8, EXT, false>(t, split, blockIdx.x, bufsize, stbytes, smem);
    else
        subtree_body<P, T, CH1, CHH, NHH, 16, EXT, false>(t, split, blockIdx.x, bufsize, stbytes, smem);
}

struct SubtreePlan {
    int split;    // level L of the subtree roots
    int grid;     // (K+1)^L workgroups
    int bufsize;  // one ping-pong buffer
    int stbytes;  // one level of subtree states
    size_t lds;
};

int g_num_cu = 0;

int num_cus()
{
    if (g_num_cu == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            g_num_cu = n;
        else
            g_num_cu = 256;
    }
    return g_num_cu;
}

// The LDS plan of the subtree algorithm with its roots at level `split`.
bool plan_subtree_at(const DevTree& t, int prec, int split, SubtreePlan& pl)
{
    if (t.E > 16 || t.n_layers < 2 || t.n_layers > 3 || t.out_pad[t.n_layers - 1] > 16)
        return false;  // one 16-wide output tile (E logits, or mu and log sigma for E <= 8)
    const int H = t.out_pad[0];
    if (H != 128 && H != 256)
        return false;
    if (t.n_layers == 3 && t.out_pad[1] != H)
        return false;
    const int kc = prec_chunk(prec), es = prec_esize(prec);
    // per-node first-layer inputs: one chunk (BF16; FP32 with E <= 14), two
    // (FP32 with E > 14) or one chunk pair (FP8)
    const int nch1 = t.in_pad_d / kc;
    if (!t.w1d || t.in_pad_d % kc != 0 || nch1 < 1 || nch1 > (prec == kFP32 ? 2 : (prec == kBF16 ? 1 : 2)) ||
        (prec == kFP8 && nch1 != 2))
        return false;
    if (split < 0 || split > t.M - 1)
        return false;
    const int64_t width_max = ipow(t.K + 1, t.M - split);
    const int64_t st = width_max * t.E;
    if (st > 16 * 1024)
        return false;
    // the biggest subtree level must not serialise too many passes
    if (t.K * ipow(t.K + 1, t.M - split - 1) > 8 * kRTmax)
        return false;
    size_t stride = (size_t)t.in_pad_d * es + 16;
    stride = std::max(stride, (size_t)H * es + 16);
    size_t buf = std::max(stride * kRTmax, (size_t)kWaves * kRTmax * 16 * 4);
    buf = (buf + 15) & ~(size_t)15;
    pl.split = split;
    pl.grid = (int)ipow(t.K + 1, split);
    pl.bufsize = (int)buf;
    pl.stbytes = (int)((st + 15) & ~15);
    size_t nbias = 0;
    for (int l = 0; l < t.n_layers; ++l)
        nbias += t.out_pad[l];
    pl.lds = 2 * buf + (size_t)kRTmax * kLogitStride * 4 + (kMaxUE + 8) * 4 + 3 * kMaxUE * 4 + nbias * 4 +
             2 * (size_t)pl.stbytes;
    if (t.head == kGaussianHead)  // the precomputed draws, 16-byte aligned
        pl.lds += 16 + (size_t)eps_slots(t.K, t.M, split) * t.E * 4;
    return pl.lds <= 160 * 1024;
}

// One launch: the deepest split whose (K+1)^split roots fit one workgroup per CU.
bool plan_subtree(const DevTree& t, int prec, SubtreePlan& pl)
{
    const int ncu = num_cus();
    int split = 0;
    while (split + 1 <= t.M - 1 && ipow(t.K + 1, split + 1) <= ncu)
        ++split;
    return plan_subtree_at(t, prec, split, pl);
}

template <int P, int T, int CH1, int CHH, int NHH>
hipError_t launch_t(const DevTree& t, const SubtreePlan& pl, hipStream_t s, hipEvent_t done)
{
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&subtree_kernel<P, T, CH1, CHH, NHH, false>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&subtree_kernel<P, T, CH1, CHH, NHH, true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    // with `done`, the event rides on the dispatch itself: an event recorded
    // after the launch would put a marker into the stream that costs about
    // 3 us of GPU time per build between back-to-back launches
    const bool ext = t.head == kGaussianHead || t.rounding == kHuntingtonHill;
    if (ext && done)
        hipExtLaunchKernelGGL((subtree_kernel<P, T, CH1, CHH, NHH, true>), dim3(pl.grid), dim3(kThreads), pl.lds, s,
                              nullptr, done, 0, t, pl.split, pl.bufsize, pl.stbytes);
    else if (ext)
        hipLaunchKernelGGL((subtree_kernel<P, T, CH1, CHH, NHH, true>), dim3(pl.grid), dim3(kThreads), pl.lds, s, t,
                           pl.split, pl.bufsize, pl.stbytes);
    else if (done)
        hipExtLaunchKernelGGL((subtree_kernel<P, T, CH1, CHH, NHH, false>), dim3(pl.grid), dim3(kThreads), pl.lds, s,
                              nullptr, done, 0, t, pl.split, pl.bufsize, pl.stbytes);
    else
        hipLaunchKernelGGL((subtree_kernel<P, T, CH1, CHH, NHH, false>), dim3(pl.grid), dim3(kThreads), pl.lds, s, t,
                           pl.split, pl.bufsize, pl.stbytes);
    return hipGetLastError();
}

template <int P, int CH1>
hipError_t dispatch_width(const DevTree& t, const SubtreePlan& pl, hipStream_t s, hipEvent_t done)
{
    constexpr int kc = Traits<P>::kChunk;
    const int H = t.out_pad[0];
    const bool two = t.n_layers == 3;
    if (H == 256)
        return two ? launch_t<P, 2, CH1, 256 / kc, 1>(t, pl, s, done) : launch_t<P, 2, CH1, 256 / kc, 0>(t, pl, s, done);
    return two ? launch_t<P, 1, CH1, 128 / kc, 1>(t, pl, s, done) : launch_t<P, 1, CH1, 128 / kc, 0>(t, pl, s, done);
}

}  // namespace

bool plan_subtree_units(const DevTree& t, int prec, int split, int* bufsize, int* stbytes, size_t* lds)
{
    // the resident worker carries one instantiation: BF16, two hidden layers
    // of 256, per-node inputs in one chunk, softmax head, largest remainder
    if (prec != kBF16 || t.n_layers != 3 || t.out_pad[0] != 256 || t.out_pad[1] != 256 ||
        t.in_pad_d != prec_chunk(prec) || t.head != kSoftmaxHead || t.rounding != kLargestRemainder)
        return false;
    SubtreePlan pl;
    if (!plan_subtree_at(t, prec, split, pl))
        return false;
    *bufsize = pl.bufsize;
    *stbytes = pl.stbytes;
    *lds = pl.lds;
    return true;
}

bool subtree_supported(const DevTree& t, int prec)
{
    SubtreePlan pl;
    return plan_subtree(t, prec, pl);
}

hipError_t launch_subtree(const DevTree& t, int prec, hipStream_t s, hipEvent_t done)
{
    SubtreePlan pl;
    if (!plan_subtree(t, prec, pl))
        return hipErrorInvalidValue;
    // register arrays are sized by the exact chunk count of the per-node inputs
    const int nch1 = t.in_pad_d / prec_chunk(prec);
    if (prec == kFP32)
        return nch1 == 1 ? dispatch_width<kFP32, 1>(t, pl, s, done) : dispatch_width<kFP32, 2>(t, pl, s, done);
    if (prec == kBF16)
        return dispatch_width<kBF16, 1>(t, pl, s, done);
    return dispatch_width<kFP8, 2>(t, pl, s, done);
}

}  // namespace cyrus
