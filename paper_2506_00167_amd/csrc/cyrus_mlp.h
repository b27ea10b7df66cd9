// The actor MLP of a tile of node rows on MFMA, shared by the level kernels
// and the critic kernel: activations in LDS (row-major, the GEMM precision,
// rows padded by 16 bytes), weight fragments streamed from global memory
// (L2-resident after the first touch), biases staged in LDS.
#pragma once

#include "cyrus_device.h"

namespace cyrus {

constexpr int kPF = 8;  // output-layer weight chunks per load group (even: chunk pairs)

// One hidden layer, out = ReLU(W in + b), for the T neuron tiles this wave
// owns (tiles wave, wave + 8, ...). The reduction runs over chunk pairs; the
// weight fragments of the next pair are requested before the MFMAs of the
// current one, and the loop body has no branches (clamped addresses, whole
// row tiles; rows past the tile's live rows are computed and discarded), so
// the loads stay in flight behind the matrix work.
template <int P, int RTT, int T>
__device__ __forceinline__ void hidden_layer(const DevTree& t, int l, const uint8_t* in, uint8_t* out,
                                             const float* bias_l, int art)
{
    constexpr int kc = Traits<P>::kChunk, es = Traits<P>::kEsize;
    const int lane = threadIdx.x & 63, wave = wave_id(), g = lane >> 4, c16 = lane & 15;
    const int nch = t.in_pad[l] / kc;
    const int sin = t.in_pad[l] * es + 16;
    const int sout = t.out_pad[l] * es + 16;
    const guint4* wl = as_global(t.w[l]);
    // The accumulators start at the bias, staged in the next layer's input
    // scale, and the products enter in that scale too: c1 = deq times the
    // next layer's inverse input scale is a power of two (1 outside FP8),
    // applied exactly by the FP8 instruction's block scale. The epilogue is
    // then the activation and the conversion alone.
    const int sc = e8m0_of(t.deq[l] * t.inv_in_scale[l + 1]);
    floatx4 acc[T][RTT];
#pragma unroll
    for (int tt = 0; tt < T; ++tt) {
        const floatx4 b4 = *reinterpret_cast<const floatx4*>(bias_l + (wave + kWaves * tt) * 16 + g * 4);
#pragma unroll
        for (int rt = 0; rt < RTT; ++rt)
            acc[tt][rt] = b4;
    }
    const guint4* wp[T];
#pragma unroll
    for (int tt = 0; tt < T; ++tt)
        wp[tt] = wl + (size_t)(wave + kWaves * tt) * nch * 64 + lane;
    const uint8_t* bp = in + c16 * sin + g * (kc / 4) * es;
    const int npair = nch >> 1;
    // two register sets in ping-pong: while one pair's fragments feed the
    // MFMAs, the other set is being loaded, so each wait only covers loads
    // issued one step earlier
    uint4 x0[T], x1[T], y0[T], y1[T];
#define CYRUS_LOAD_PAIR(D0, D1, Q)                                                                                     \
    {                                                                                                                  \
        const int c_ = min((Q), max(npair - 1, 0)) * 2; /* clamped: past the end reloads the last pair */             \
        _Pragma("unroll") for (int tt = 0; tt < T; ++tt)                                                              \
        {                                                                                                              \
            D0[tt] = gld(wp[tt] + (size_t)c_ * 64);                                                                    \
            D1[tt] = gld(wp[tt] + (size_t)(c_ + 1) * 64);                                                              \
        }                                                                                                              \
    }
    // B fragments: row tile rt + 1's pair is read from LDS while row tile
    // rt's MFMAs run, so each wait covers a load issued one tile earlier
#define CYRUS_MMA_PAIRS(S0, S1, Q)                                                                                     \
    {                                                                                                                  \
        const uint8_t* bq_ = bp + 2 * (Q) * kc * es;                                                                   \
        uint4 n0_ = *reinterpret_cast<const uint4*>(bq_);                                                              \
        uint4 n1_ = *reinterpret_cast<const uint4*>(bq_ + kc * es);                                                    \
        _Pragma("unroll") for (int rt = 0; rt < RTT; ++rt)                                                            \
        {                                                                                                              \
            const uint4 b0_ = n0_, b1_ = n1_;                                                                          \
            if (rt + 1 < RTT) {                                                                                        \
                n0_ = *reinterpret_cast<const uint4*>(bq_ + (rt + 1) * 16 * sin);                                      \
                n1_ = *reinterpret_cast<const uint4*>(bq_ + (rt + 1) * 16 * sin + kc * es);                            \
            }                                                                                                          \
            __builtin_amdgcn_sched_barrier(0);                                                                         \
            _Pragma("unroll") for (int tt = 0; tt < T; ++tt) mma_pair_scaled<P>(S0[tt], S1[tt], b0_, b1_, acc[tt][rt], sc); \
            __builtin_amdgcn_sched_barrier(0);                                                                         \
        }                                                                                                              \
    }
    if (npair > 0)
        CYRUS_LOAD_PAIR(x0, x1, 0)
    int q = 0;
    for (; q + 1 < npair; q += 2) {
        CYRUS_LOAD_PAIR(y0, y1, q + 1)
        __builtin_amdgcn_sched_barrier(0);  // the next pair's loads go out before this pair's MFMAs
        CYRUS_MMA_PAIRS(x0, x1, q)
        CYRUS_LOAD_PAIR(x0, x1, q + 2)
        __builtin_amdgcn_sched_barrier(0);
        CYRUS_MMA_PAIRS(y0, y1, q + 1)
    }
    if (q < npair)
        CYRUS_MMA_PAIRS(x0, x1, q)
#undef CYRUS_LOAD_PAIR
#undef CYRUS_MMA_PAIRS
    if (P != kFP8 && (nch & 1)) {  // odd chunk count (FP32/BF16 first layer; FP8 pads to pairs): one last chunk
        const int c = nch - 1;
        const uint8_t* bq = bp + c * kc * es;
        uint4 a0[T];
#pragma unroll
        for (int tt = 0; tt < T; ++tt)
            a0[tt] = gld(wp[tt] + (size_t)c * 64);
#pragma unroll
        for (int rt = 0; rt < RTT; ++rt) {
            const uint4 b0 = *reinterpret_cast<const uint4*>(bq + rt * 16 * sin);
#pragma unroll
            for (int tt = 0; tt < T; ++tt)
                mma_chunk<P>(a0[tt], b0, acc[tt][rt]);
        }
    }
#pragma unroll
    for (int tt = 0; tt < T; ++tt) {
        const int nt = wave + kWaves * tt;
#pragma unroll
        for (int rt = 0; rt < RTT; ++rt) {
            if (rt < art)
                store_act4<P>(out + (rt * 16 + c16) * sout + (nt * 16 + g * 4) * es, acc[tt][rt][0], acc[tt][rt][1],
                              acc[tt][rt][2], acc[tt][rt][3]);
        }
    }
}

// Actor forward pass over `nrows` node rows whose features are in bufA, with
// the biases of all layers staged in LDS (layer after layer, out_pad each;
// a hidden layer's already in the next layer's input scale).
// Leaves the FP32 logits in zl[row * kLogitStride + e].
// Row `row` of the tile is evaluated node off + p (K+1) + k of its level (r =
// row0 + row = p K + k - 1); the Gaussian head keys its draws by that node.
template <int P, int RTT>
__device__ __forceinline__ void run_mlp(const DevTree& t, int nrows, uint8_t* bufA, uint8_t* bufB, float* zl,
                                        const float* bias, int64_t off, int row0)
{
    constexpr int kc = Traits<P>::kChunk, es = Traits<P>::kEsize;
    static_assert(RTT <= kWaves, "the output layer gives each row tile a wave");
    const int lane = threadIdx.x & 63, wave = wave_id(), g = lane >> 4, c16 = lane & 15;
    const int art = (nrows + 15) >> 4;
    uint8_t* in = bufA;
    uint8_t* out = bufB;
    for (int l = 0; l + 1 < t.n_layers; ++l) {
        if (l > 0)
            lds_barrier();  // the previous layer's outputs are complete and its inputs read
        const int T = (t.out_pad[l] >> 4) / kWaves;  // neuron tiles per wave (hidden widths are multiples of 128)
        switch (T) {
        case 1:
            hidden_layer<P, RTT, 1>(t, l, in, out, bias, art);
            break;
        case 2:
            hidden_layer<P, RTT, 2>(t, l, in, out, bias, art);
            break;
        case 3:
            hidden_layer<P, RTT, 3>(t, l, in, out, bias, art);
            break;
        default:
            hidden_layer<P, RTT, 4>(t, l, in, out, bias, art);
            break;
        }
        bias += t.out_pad[l];
        uint8_t* tmp = in;
        in = out;
        out = tmp;
    }
    // Output layer. Wave w owns row tile w (RTT <= waves) and reduces over
    // the whole input in chunk order, so a row's logits do not depend on the
    // tile it was computed in. The wave's weight fragments arrive in groups
    // of kPF chunks, the next group requested before the current one's MFMAs;
    // the first group is requested before the barrier that completes the
    // last hidden layer. As in the hidden layers, the accumulators start at
    // the bias and FP8 applies deq through the block scale. Softmax head: the
    // lanes write their logits to zl directly; Gaussian head: the outputs go
    // through LDS, since a log-share needs outputs e and E + e, which other
    // lanes may hold.
    {
        const int l = t.n_layers - 1;
        const int nch = t.in_pad[l] / kc;
        const int sin = t.in_pad[l] * es + 16;
        const int opad = t.out_pad[l];
        const int ntile = opad >> 4;
        const int E = t.E, K = t.K;
        const int sc = e8m0_of(t.deq[l]);
        const bool gaussian = t.head == kGaussianHead;
        float* raw = reinterpret_cast<float*>(out);  // [RT][opad], Gaussian head
        const int rt = wave;
        const guint4* wl = as_global(t.w[l]) + lane;
        uint4 a[kPF], an[kPF];
        if (rt < art) {
#pragma unroll
            for (int j = 0; j < kPF; ++j)
                a[j] = j < nch ? gld(wl + (size_t)j * 64) : uint4{0, 0, 0, 0};
        }
        lds_barrier();
        if (rt < art) {
            const int row = rt * 16 + c16;
            const uint8_t* bp = in + row * sin + g * (kc / 4) * es;
            for (int nt = 0; nt < ntile; ++nt) {
                const guint4* wp = wl + (size_t)nt * nch * 64;
                if (nt > 0) {
#pragma unroll
                    for (int j = 0; j < kPF; ++j)
                        a[j] = j < nch ? gld(wp + (size_t)j * 64) : uint4{0, 0, 0, 0};
                }
                floatx4 acc = *reinterpret_cast<const floatx4*>(bias + nt * 16 + g * 4);
                for (int cb = 0; cb < nch; cb += kPF) {
#pragma unroll
                    for (int j = 0; j < kPF; ++j)
                        an[j] = cb + kPF + j < nch ? gld(wp + (size_t)(cb + kPF + j) * 64) : uint4{0, 0, 0, 0};
#pragma unroll
                    for (int j = 0; j < kPF; j += 2) {
                        const int c = cb + j;
                        if (c + 1 < nch) {
                            const uint4 b0 = *reinterpret_cast<const uint4*>(bp + c * kc * es);
                            const uint4 b1 = *reinterpret_cast<const uint4*>(bp + (c + 1) * kc * es);
                            mma_pair_scaled<P>(a[j], a[j + 1], b0, b1, acc, sc);
                        } else if (c < nch) {  // FP32 and BF16 only: FP8 inputs are padded to chunk pairs
                            mma_chunk<P>(a[j], *reinterpret_cast<const uint4*>(bp + c * kc * es), acc);
                        }
                    }
#pragma unroll
                    for (int j = 0; j < kPF; ++j)
                        a[j] = an[j];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int e = nt * 16 + g * 4 + i;
                    if (gaussian)
                        raw[row * opad + e] = acc[i];
                    else if (row < nrows && e < E)
                        zl[row * kLogitStride + e] = acc[i];
                }
            }
        }
        if (gaussian) {
            lds_barrier();
            for (int idx = threadIdx.x; idx < nrows * E; idx += kThreads) {
                const int row = idx / E, e = idx - row * E;
                const int r = row0 + row, p = r / K, k = r - p * K + 1;
                // outputs E..2E-1 are the log standard deviations
                zl[row * kLogitStride + e] = gaussian_log_share(raw[row * opad + e], raw[row * opad + E + e], t.seed,
                                                                t.tti, off + (int64_t)p * (K + 1) + k, e);
            }
        }
        lds_barrier();
    }
}

}  // namespace cyrus
