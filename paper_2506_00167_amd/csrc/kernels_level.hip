// Level kernels: one launch per mini-slot level tau, one workgroup per tile of
// RT = 16*RTT evaluated nodes of that level (the k > 0 children of the nodes
// of level tau-1). Each workgroup assembles the node features, runs the whole
// actor MLP on MFMA with the activations in LDS and the weight fragments read
// from global memory (L2-resident after the first touch), then applies the
// feasibility enforcer and writes the nodes' puncturing vectors and states.
// This is the general path (any width, depth, precision, cells batched per
// launch); the latency path for small trees is kernels_subtree.hip. Within a
// launch, workgroups read only what earlier launches wrote (the parent
// level's states), so waves meet at LDS-only barriers.
#include <algorithm>

#include "cyrus_device.h"
#include "cyrus_kernels.h"

namespace cyrus {

constexpr int kPF = 4;   // output-layer weight chunks loaded per group
constexpr int kTMax = 4; // neuron tiles a wave accumulates at once

__device__ __forceinline__ int64_t dev_level_offset(int K, int tau)
{
    int64_t p = 1;
    for (int i = 0; i < tau; ++i)
        p *= (K + 1);
    return (p - 1) / K;
}

// Enforcer for the rows of a tile, G lanes per row (lane e = UE e). Each
// evaluated node writes its allocation and state; the first child (k = 1) of
// every parent also writes the k = 0 sibling, which punctures nothing and
// passes the parent state on unchanged.
template <int G>
__device__ __forceinline__ void finish_rows_level(const DevTree& t, const float* zl, const int* R, int rsum, int row0,
                                                  int nrows, int64_t off, int64_t poff)
{
    const int E = t.E, K = t.K;
    for (int base = 0; base < nrows; base += kThreads / G) {
        const int row = base + (int)threadIdx.x / G, e = (int)threadIdx.x % G;
        if (row < nrows) {
            const int r = row0 + row, p = r / K, k = r - p * K + 1;
            float* zrow = const_cast<float*>(zl) + row * kLogitStride;
            const float z = e < E ? zrow[e] : 0.f;
            int a;
            if constexpr (G <= 16)
                a = enforce_dpp<G>(E, e, z, e < E ? R[e] : 0, rsum, t.U * k, zrow);  // row reused for ranks
            else
                a = enforce_group<G>(E, e, z, e < E ? R[e] : 0, rsum, t.U * k);
            if (e < E) {
                const int64_t node = off + (int64_t)p * (K + 1) + k, parent = poff + p;
                const uint8_t c = t.state[parent * E + e];
                t.alloc[node * E + e] = (uint8_t)a;
                t.state[node * E + e] = (uint8_t)(c + a);
                if (t.logits)
                    t.logits[node * E + e] = z;
                if (k == 1) {
                    const int64_t sib = off + (int64_t)p * (K + 1);
                    t.alloc[sib * E + e] = 0;
                    t.state[sib * E + e] = c;
                    if (t.logits)
                        t.logits[sib * E + e] = 0.f;
                }
            }
        }
    }
}

// Actor forward pass over `nrows` node rows whose features are in bufA.
// Leaves the FP32 logits in zl[row * kLogitStride + e].
template <int P, int RTT>
__device__ __forceinline__ void run_mlp(const DevTree& t, int nrows, uint8_t* bufA, uint8_t* bufB, float* zl)
{
    constexpr int kc = Traits<P>::kChunk, es = Traits<P>::kEsize, RT = 16 * RTT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, c16 = lane & 15;
    const int art = (nrows + 15) >> 4;
    uint8_t* in = bufA;
    uint8_t* out = bufB;
    for (int l = 0; l + 1 < t.n_layers; ++l) {
        const int nch = t.in_pad[l] / kc;
        const int sin = t.in_pad[l] * es + 16;
        const int sout = t.out_pad[l] * es + 16;
        const int ntile = t.out_pad[l] >> 4;
        const uint4* wl = reinterpret_cast<const uint4*>(t.w[l]);
        const float deq = t.deq[l];
        const float inv_next = t.inv_in_scale[l + 1];
        // this wave owns neuron tiles wave, wave + 8, ...; up to kTMax of them
        // accumulate together so each activation fragment read from LDS feeds
        // every tile of the wave
        const int T = (ntile - wave + kWaves - 1) / kWaves;
        for (int tt0 = 0; tt0 < T; tt0 += kTMax) {
            floatx4 acc[kTMax][RTT];
#pragma unroll
            for (int tt = 0; tt < kTMax; ++tt)
#pragma unroll
                for (int rt = 0; rt < RTT; ++rt)
                    acc[tt][rt] = floatx4{0.f, 0.f, 0.f, 0.f};
            const uint4* wp[kTMax];
#pragma unroll
            for (int tt = 0; tt < kTMax; ++tt)
                wp[tt] = wl + (size_t)(wave + kWaves * min(tt0 + tt, T - 1)) * nch * 64 + lane;
            const uint8_t* bp = in + c16 * sin + g * (kc / 4) * es;
            // weight fragments stream from L2 one chunk pair ahead of the MFMAs
            uint4 a0[kTMax], a1[kTMax];
#pragma unroll
            for (int tt = 0; tt < kTMax; ++tt) {
                a0[tt] = wp[tt][0];
                a1[tt] = (nch > 1) ? wp[tt][64] : uint4{0, 0, 0, 0};
            }
            for (int c = 0; c < nch; c += 2) {
                uint4 n0[kTMax], n1[kTMax];
#pragma unroll
                for (int tt = 0; tt < kTMax; ++tt) {
                    n0[tt] = (c + 2 < nch) ? wp[tt][(size_t)(c + 2) * 64] : uint4{0, 0, 0, 0};
                    n1[tt] = (c + 3 < nch) ? wp[tt][(size_t)(c + 3) * 64] : uint4{0, 0, 0, 0};
                }
#pragma unroll
                for (int rt = 0; rt < RTT; ++rt) {
                    if (rt < art) {
                        const uint8_t* brow = bp + rt * 16 * sin + c * kc * es;
                        const uint4 b0 = *reinterpret_cast<const uint4*>(brow);
                        const uint4 b1 =
                            (c + 1 < nch) ? *reinterpret_cast<const uint4*>(brow + kc * es) : uint4{0, 0, 0, 0};
#pragma unroll
                        for (int tt = 0; tt < kTMax; ++tt)
                            if (tt0 + tt < T)
                                mma_pair<P>(a0[tt], a1[tt], b0, b1, acc[tt][rt]);
                    }
                }
#pragma unroll
                for (int tt = 0; tt < kTMax; ++tt) {
                    a0[tt] = n0[tt];
                    a1[tt] = n1[tt];
                }
            }
#pragma unroll
            for (int tt = 0; tt < kTMax; ++tt) {
                if (tt0 + tt >= T)
                    continue;
                const int nt = wave + kWaves * (tt0 + tt);
                const floatx4 bias = *reinterpret_cast<const floatx4*>(t.b[l] + nt * 16 + g * 4);
#pragma unroll
                for (int rt = 0; rt < RTT; ++rt) {
                    if (rt < art) {
                        const float v0 = fmaxf(acc[tt][rt][0] * deq + bias[0], 0.f);
                        const float v1 = fmaxf(acc[tt][rt][1] * deq + bias[1], 0.f);
                        const float v2 = fmaxf(acc[tt][rt][2] * deq + bias[2], 0.f);
                        const float v3 = fmaxf(acc[tt][rt][3] * deq + bias[3], 0.f);
                        store4<P>(out + (rt * 16 + c16) * sout + (nt * 16 + g * 4) * es, v0, v1, v2, v3, inv_next);
                    }
                }
            }
        }
        lds_barrier();
        uint8_t* tmp = in;
        in = out;
        out = tmp;
    }
    // Output layer: the reduction dimension is split across the waves; each
    // wave leaves a partial logit tile, summed in wave order below.
    {
        const int l = t.n_layers - 1;
        const int nch = t.in_pad[l] / kc;
        const int sin = t.in_pad[l] * es + 16;
        const int opad = t.out_pad[l];
        const int ntile = opad >> 4;
        const int cpw = (nch + kWaves - 1) / kWaves;
        const int c0 = wave * cpw, c1 = min(nch, c0 + cpw);
        float* part = reinterpret_cast<float*>(out);
        const uint4* wl = reinterpret_cast<const uint4*>(t.w[l]);
        for (int nt = 0; nt < ntile; ++nt) {
            floatx4 acc[RTT];
#pragma unroll
            for (int rt = 0; rt < RTT; ++rt)
                acc[rt] = floatx4{0.f, 0.f, 0.f, 0.f};
            const uint4* wp = wl + (size_t)nt * nch * 64 + lane;
            const uint8_t* bp = in + c16 * sin + g * (kc / 4) * es;
            for (int cb = c0; cb < c1; cb += kPF) {
                uint4 a[kPF];
#pragma unroll
                for (int j = 0; j < kPF; ++j)
                    a[j] = (cb + j < c1) ? wp[(size_t)(cb + j) * 64] : uint4{0, 0, 0, 0};
#pragma unroll
                for (int j = 0; j < kPF; ++j) {
                    if (cb + j < c1) {
#pragma unroll
                        for (int rt = 0; rt < RTT; ++rt) {
                            if (rt < art) {
                                const uint4 b =
                                    *reinterpret_cast<const uint4*>(bp + rt * 16 * sin + (cb + j) * kc * es);
                                mma_chunk<P>(a[j], b, acc[rt]);
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int rt = 0; rt < RTT; ++rt)
                if (rt < art)
                    *reinterpret_cast<floatx4*>(part + (size_t)(wave * RT + rt * 16 + c16) * opad + nt * 16 + g * 4) =
                        acc[rt];
        }
        lds_barrier();
        const int E = t.E;
        const float deq = t.deq[l];
        for (int idx = threadIdx.x; idx < nrows * E; idx += kThreads) {
            const int row = idx / E, e = idx - row * E;
            float s = 0.f;
            for (int w = 0; w < kWaves; ++w)
                s += part[(size_t)(w * RT + row) * opad + e];
            zl[row * kLogitStride + e] = s * deq + t.b[l][e];
        }
        lds_barrier();
    }
}

// One tile of evaluated rows [row0, row0 + nrows) of level tau.
template <int P, int RTT>
__device__ __forceinline__ void level_tile(const DevTree& t, int tau, int row0, int nrows, uint8_t* smem, int bufsize)
{
    constexpr int es = Traits<P>::kEsize, RT = 16 * RTT;
    uint8_t* bufA = smem;
    uint8_t* bufB = smem + bufsize;
    float* zl = reinterpret_cast<float*>(smem + 2 * bufsize);
    int* R = reinterpret_cast<int*>(zl + RT * kLogitStride);
    int* rsum_lds = R + kMaxUE;
    float* statf = reinterpret_cast<float*>(rsum_lds + 4);  // R/32, MCS/32, SINR/32
    const int E = t.E, K = t.K;
    if (threadIdx.x < E) {
        const int e = threadIdx.x;
        R[e] = t.ue[e];
        statf[e] = (float)t.ue[e] * (1.f / 32.f);
        statf[E + e] = (float)t.ue[E + e] * (1.f / 32.f);
        statf[2 * E + e] = __int_as_float(t.ue[2 * E + e]) * (1.f / 32.f);
    }
    lds_barrier();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int e = 0; e < E; ++e)
            s += R[e];
        *rsum_lds = s;
    }
    const int64_t off = dev_level_offset(K, tau), poff = dev_level_offset(K, tau - 1);

    // features of every row, zero padded to the k-chunk and to whole row tiles
    const int in0 = t.in_pad[0], d_in = t.in_dim0, s0 = in0 * es + 16;
    const int nrows_pad = ((nrows + 15) >> 4) << 4;
    const float inv0 = t.inv_in_scale[0];
    for (int idx = threadIdx.x; idx < nrows_pad * in0; idx += kThreads) {
        const int row = idx / in0, f = idx - row * in0;
        float v = 0.f;
        if (row < nrows && f < d_in) {
            const int r = row0 + row, p = r / K, k = r - p * K + 1;
            if (f < 3 * E)
                v = statf[f];
            else if (f < 4 * E)
                v = (float)t.state[(poff + p) * E + (f - 3 * E)] * (1.f / 64.f);
            else if (f == 4 * E)
                v = (float)tau * (1.f / 8.f);
            else
                v = (float)k * (1.f / 8.f);
        }
        store1<P>(bufA + row * s0 + f * es, v, inv0);
    }
    lds_barrier();
    run_mlp<P, RTT>(t, nrows, bufA, bufB, zl);

    if (E <= 8)
        finish_rows_level<8>(t, zl, R, *rsum_lds, row0, nrows, off, poff);
    else if (E <= 16)
        finish_rows_level<16>(t, zl, R, *rsum_lds, row0, nrows, off, poff);
    else
        finish_rows_level<32>(t, zl, R, *rsum_lds, row0, nrows, off, poff);
}

template <int P, int RTT>
__global__ __launch_bounds__(kThreads) void level_kernel(DevTree t, int tau, int n_eval, int bufsize)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const int row0 = blockIdx.x * 16 * RTT;
    const int nrows = min(16 * RTT, n_eval - row0);
    if (nrows <= 0)
        return;
    level_tile<P, RTT>(t, tau, row0, nrows, smem, bufsize);
}

// Batched level launch over several codebooks (cells), each at its own level:
// entry j of the launch is codebook ent_tree[j] at level ent_tau[j] and owns
// row tiles [prefix[j], prefix[j+1]) of the prefix[n] tiles of the launch.
// Persistent: a grid of at most one workgroup per CU strides over the tiles.
template <int P, int RTT>
__global__ __launch_bounds__(kThreads) void level_kernel_batch(const DevTree* trees, const int* ent_tree,
                                                               const int* ent_tau, const int* prefix, int n,
                                                               int bufsize)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const int total = prefix[n];
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= b)
                lo = mid;
            else
                hi = mid - 1;
        }
        const DevTree& t = trees[ent_tree[lo]];
        const int tau = ent_tau[lo];
        const int n_eval = (int)(t.K * (dev_level_offset(t.K, tau) - dev_level_offset(t.K, tau - 1)));
        const int row0 = (b - prefix[lo]) * 16 * RTT;
        const int nrows = min(16 * RTT, n_eval - row0);
        if (nrows > 0)
            level_tile<P, RTT>(t, tau, row0, nrows, smem, bufsize);
        lds_barrier();  // LDS is reused by the next tile
    }
}

// Converts FP32 fragment-ordered weights into the storage type of P, in place
// of the packed buffer (elementwise; FP8 with its power-of-two scale).
template <int P>
__global__ void convert_weights(const float* src, uint8_t* dst, int64_t n4, float inv_w_scale)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n4)
        return;
    const floatx4 v = reinterpret_cast<const floatx4*>(src)[i];
    store4<P>(dst + i * 4 * Traits<P>::kEsize, v[0], v[1], v[2], v[3], inv_w_scale);
}

// ------------------------------------------------------------------ launch

size_t level_buf_bytes(const DevTree& t, int prec, int rtt)
{
    const int es = prec_esize(prec), rt = 16 * rtt;
    size_t stride = 0;
    for (int l = 0; l < t.n_layers; ++l) {
        const size_t s = (size_t)t.in_pad[l] * es + 16;
        stride = s > stride ? s : stride;
    }
    size_t buf = stride * rt;
    const size_t part = (size_t)kWaves * rt * t.out_pad[t.n_layers - 1] * 4;
    if (part > buf)
        buf = part;
    return (buf + 15) & ~(size_t)15;
}

size_t level_lds_for_buf(size_t buf, int rtt)
{
    return 2 * buf + (size_t)16 * rtt * kLogitStride * 4 + (kMaxUE + 4) * 4 + 3 * kMaxUE * 4;
}

size_t level_lds_bytes(const DevTree& t, int prec, int rtt) { return level_lds_for_buf(level_buf_bytes(t, prec, rtt), rtt); }

template <int P, int RTT>
static hipError_t launch_level_t(const DevTree& t, int tau, hipStream_t s)
{
    const int n_eval = (int)(t.K * ipow(t.K + 1, tau - 1));
    const int grid = (n_eval + 16 * RTT - 1) / (16 * RTT);
    const int buf = (int)level_buf_bytes(t, P, RTT);
    const size_t lds = level_lds_bytes(t, P, RTT);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&level_kernel<P, RTT>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL((level_kernel<P, RTT>), dim3(grid), dim3(kThreads), lds, s, t, tau, n_eval, buf);
    return hipGetLastError();
}

template <int P, int RTT>
static hipError_t launch_level_batch_t(const DevTree* trees, const int* ent_tree, const int* ent_tau,
                                       const int* prefix, int n, int nblocks, int buf, size_t lds, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&level_kernel_batch<P, RTT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    static int ncu = 0;
    if (ncu == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
            ncu = 256;
    }
    const int grid = std::min(nblocks, ncu * std::max(1, (int)((160 * 1024) / lds)));
    if (grid < 1)
        return hipSuccess;
    hipLaunchKernelGGL((level_kernel_batch<P, RTT>), dim3(grid), dim3(kThreads), lds, s, trees, ent_tree, ent_tau,
                       prefix, n, buf);
    return hipGetLastError();
}

hipError_t launch_level(const DevTree& t, int prec, int rtt, int tau, hipStream_t s)
{
#define CYRUS_LEVEL_CASE(P, R)                                                                                         \
    if (prec == P && rtt == R)                                                                                         \
        return launch_level_t<P, R>(t, tau, s);
    CYRUS_LEVEL_CASE(kFP32, 1) CYRUS_LEVEL_CASE(kFP32, 2) CYRUS_LEVEL_CASE(kFP32, 4)
    CYRUS_LEVEL_CASE(kBF16, 1) CYRUS_LEVEL_CASE(kBF16, 2) CYRUS_LEVEL_CASE(kBF16, 4) CYRUS_LEVEL_CASE(kBF16, 8)
    CYRUS_LEVEL_CASE(kFP8, 1) CYRUS_LEVEL_CASE(kFP8, 2) CYRUS_LEVEL_CASE(kFP8, 4) CYRUS_LEVEL_CASE(kFP8, 8)
#undef CYRUS_LEVEL_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_level_batch(const DevTree* trees, const int* ent_tree, const int* ent_tau, const int* prefix, int n,
                              int nblocks, int prec, int rtt, int buf, size_t lds, hipStream_t s)
{
#define CYRUS_LEVEL_CASE(P, R)                                                                                         \
    if (prec == P && rtt == R)                                                                                         \
        return launch_level_batch_t<P, R>(trees, ent_tree, ent_tau, prefix, n, nblocks, buf, lds, s);
    CYRUS_LEVEL_CASE(kFP32, 1) CYRUS_LEVEL_CASE(kFP32, 2) CYRUS_LEVEL_CASE(kFP32, 4)
    CYRUS_LEVEL_CASE(kBF16, 1) CYRUS_LEVEL_CASE(kBF16, 2) CYRUS_LEVEL_CASE(kBF16, 4) CYRUS_LEVEL_CASE(kBF16, 8)
    CYRUS_LEVEL_CASE(kFP8, 1) CYRUS_LEVEL_CASE(kFP8, 2) CYRUS_LEVEL_CASE(kFP8, 4) CYRUS_LEVEL_CASE(kFP8, 8)
#undef CYRUS_LEVEL_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_convert_weights(int prec, const float* src, uint8_t* dst, int64_t n_floats, float inv_w_scale,
                                  hipStream_t s)
{
    const int64_t n4 = n_floats / 4;
    const int block = 256;
    const int grid = (int)((n4 + block - 1) / block);
    if (grid == 0)
        return hipSuccess;
    if (prec == kFP32)
        hipLaunchKernelGGL(convert_weights<kFP32>, dim3(grid), dim3(block), 0, s, src, dst, n4, inv_w_scale);
    else if (prec == kBF16)
        hipLaunchKernelGGL(convert_weights<kBF16>, dim3(grid), dim3(block), 0, s, src, dst, n4, inv_w_scale);
    else
        hipLaunchKernelGGL(convert_weights<kFP8>, dim3(grid), dim3(block), 0, s, src, dst, n4, inv_w_scale);
    return hipGetLastError();
}

}  // namespace cyrus
