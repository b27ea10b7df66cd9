// Actor-style MLP with its weights resident in registers, on MFMA: each wave
// holds the A fragments of its output-neuron tiles (hidden layers) and its
// slice of the output layer's reduction, loaded once; activations move
// through LDS in the transposed layer form (weights as the A operand, node
// rows as the B operand), except that in FP32 and BF16 the last hidden
// layer's accumulators feed the output layer straight from registers.
// Shared by the subtree kernel and the critic pass.
#pragma once

#include "cyrus_device.h"

namespace cyrus {

namespace {

typedef short short4v __attribute__((ext_vector_type(4)));

// Row tiles per pass: 64 rows for BF16/FP8; 48 for FP32, whose register-
// resident weights leave room for fewer accumulators.
template <int P>
struct Rows {
    static constexpr int kRTT = (P == kFP32) ? 3 : 4;
    static constexpr int kRT = 16 * kRTT;
};
constexpr int kRTmax = 64;

// Register-resident fragments of one wave.
//   T     output-neuron tiles of 16 per hidden layer owned by this wave
//   CH1   chunks of the first layer's input as held in registers
//         (DevTree::in_pad_d / chunk; DevTree::w1d holds those fragments)
//   CHH   chunks of a hidden layer's input (H / chunk)
//   NHH   hidden->hidden layers (0 or 1)
template <int P, int T, int CH1, int CHH, int NHH>
struct WaveWeights {
    static constexpr int CPW = (CHH + kWaves - 1) / kWaves;  // output-layer chunks per wave
    uint4 w1[T][CH1];
    uint4 wh[NHH > 0 ? T : 1][NHH > 0 ? CHH : 1];
    uint4 wo[CPW];
    // BF16 with a hidden->hidden layer: the output-layer weights of the
    // wave's own last-hidden-layer tiles in the 16x16x16 MFMA layout (lane
    // (g, i): W_o[i][16 nt + 4g .. 16 nt + 4g + 3]), fed from registers
    uint2 wo16[(P == kBF16 && NHH > 0) ? T : 1];
    // FP8 with a hidden->hidden layer: the same, for 16x16x32 FP8 MFMAs over
    // pairs of the wave's tiles (lane (g, i): W_o[i][16 nt + 4g .. + 3] of
    // tile 2p in the low word, of tile 2p + 1 (or zeros) in the high word)
    uint2 wo8[(P == kFP8 && NHH > 0) ? (T + 1) / 2 : 1];
};

template <int P, int T, int CH1, int CHH, int NHH>
__device__ __forceinline__ void load_weights(const DevTree& t, WaveWeights<P, T, CH1, CHH, NHH>& W, int wave,
                                             int lane)
{
    using WW = WaveWeights<P, T, CH1, CHH, NHH>;
    const uint4* g1 = reinterpret_cast<const uint4*>(t.w1d);
#pragma unroll
    for (int tt = 0; tt < T; ++tt) {
        const int nt = wave + kWaves * tt;
#pragma unroll
        for (int c = 0; c < CH1; ++c)
            W.w1[tt][c] = g1[((size_t)nt * CH1 + c) * 64 + lane];
    }
    if constexpr (NHH > 0) {
        const uint4* gh = reinterpret_cast<const uint4*>(t.w[1]);
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            const int nt = wave + kWaves * tt;
#pragma unroll
            for (int c = 0; c < CHH; ++c)
                W.wh[tt][c] = gh[((size_t)nt * CHH + c) * 64 + lane];
        }
    }
    // output-layer chunks wave, wave + kWaves, ...: for FP32 (chunk = one
    // neuron tile) these are the wave's own tiles of the last hidden layer
    const uint4* go = reinterpret_cast<const uint4*>(t.w[NHH + 1]);
#pragma unroll
    for (int j = 0; j < WW::CPW; ++j) {
        const int c = wave + kWaves * j;
        W.wo[j] = (c < CHH) ? go[(size_t)c * 64 + lane] : uint4{0, 0, 0, 0};
    }
    if constexpr (P == kBF16 && NHH > 0) {
        // W_o[i][k], k = 16 nt + 4g + j, sits in 32-wide chunk k / 32 at lane
        // i + 16 ((k % 32) / 8), elements (k % 8): four consecutive BF16
        const uint8_t* gob = t.w[NHH + 1];
        const int g = lane >> 4, i = lane & 15;
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            const int nt = wave + kWaves * tt;
            const int src = i + 16 * (2 * (nt & 1) + (g >> 1));
            W.wo16[tt] = *reinterpret_cast<const uint2*>(gob + ((size_t)(nt >> 1) * 64 + src) * 16 + 8 * (g & 1));
        }
    }
    if constexpr (P == kFP8 && NHH > 0) {
        // W_o[i][k], k = 16 nt + 4g + j, sits in 64-wide chunk k / 64 at lane
        // i + 16 ((k % 64) / 16), byte k % 16 = 4g + j: one word per tile
        const uint8_t* gob = t.w[NHH + 1];
        const int g = lane >> 4, i = lane & 15;
#pragma unroll
        for (int q = 0; q < (T + 1) / 2; ++q) {
            uint32_t w2[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int tt = 2 * q + h, nt = wave + kWaves * tt;
                w2[h] = tt < T ? *reinterpret_cast<const uint32_t*>(
                                     gob + ((size_t)(nt >> 2) * 64 + (nt & 3) * 16 + i) * 16 + 4 * g)
                               : 0u;
            }
            W.wo8[q] = uint2{w2[0], w2[1]};
        }
    }
}

// acc = A * in for the wave's T neuron tiles over `art` row tiles (inputs
// from LDS, row stride sin bytes).
// One layer's MFMAs over NT live row tiles (chunks of 16/32 reduction
// values). The B fragments of a chunk are loaded D chunks ahead of its
// MFMAs, and scheduling barriers keep the loads ahead, so LDS latency hides
// behind the matrix core: one chunk ahead in FP32 (each load feeds four MFMAs
// per output tile), about four 16-byte loads ahead in BF16 (one MFMA per
// output tile).
// Fully unrolled, so only the D + 1 chunks in flight hold registers.
template <int P, int T, int NCH, int NT>
__device__ __forceinline__ void layer_acc_tiles(const uint4 (&A)[T][NCH], int nch, const uint8_t* bp, int sin,
                                                floatx4 (&acc)[T][Rows<P>::kRTT])
{
    constexpr int kc = Traits<P>::kChunk, es = Traits<P>::kEsize;
    constexpr int D = (P == kFP32 || NT >= 4) ? 1 : 4 / NT;
    uint4 b[NCH][NT];
#pragma unroll
    for (int c = 0; c < D && c < NCH; ++c) {
        if (c < nch) {
#pragma unroll
            for (int rt = 0; rt < NT; ++rt)
                b[c][rt] = *reinterpret_cast<const uint4*>(bp + rt * 16 * sin + c * kc * es);
        }
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        if (c < nch) {
            if (c + D < NCH && c + D < nch) {
#pragma unroll
                for (int rt = 0; rt < NT; ++rt)
                    b[c + D][rt] = *reinterpret_cast<const uint4*>(bp + rt * 16 * sin + (c + D) * kc * es);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int rt = 0; rt < NT; ++rt)
#pragma unroll
                for (int tt = 0; tt < T; ++tt)
                    mma_chunk<P>(A[tt][c], b[c][rt], acc[tt][rt]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Picks the instantiation for the number of live row tiles, art in [1, NT]
// (art = 0 does nothing).
template <int P, int T, int NCH, int NT>
__device__ __forceinline__ void layer_acc_dispatch(const uint4 (&A)[T][NCH], int nch, const uint8_t* bp, int sin,
                                                   int art, floatx4 (&acc)[T][Rows<P>::kRTT])
{
    if (art == NT)
        layer_acc_tiles<P, T, NCH, NT>(A, nch, bp, sin, acc);
    else if constexpr (NT > 1)
        layer_acc_dispatch<P, T, NCH, NT - 1>(A, nch, bp, sin, art, acc);
}

template <int P, int T, int NCH>
__device__ __forceinline__ void layer_acc(const uint4 (&A)[T][NCH], int nch, const uint8_t* in, int sin, int art,
                                          int g, int c16, floatx4 (&acc)[T][Rows<P>::kRTT])
{
    constexpr int kc = Traits<P>::kChunk, es = Traits<P>::kEsize, kRTT = Rows<P>::kRTT;
#pragma unroll
    for (int tt = 0; tt < T; ++tt)
#pragma unroll
        for (int rt = 0; rt < kRTT; ++rt)
            acc[tt][rt] = floatx4{0.f, 0.f, 0.f, 0.f};
    static_assert(P != kFP8, "FP8 layers go through layer_acc_fp8");
    const uint8_t* bp = in + c16 * sin + g * (kc / 4) * es;
    layer_acc_dispatch<P, T, NCH, kRTT>(A, nch, bp, sin, art, acc);
}

// FP8 layer body over NT live row tiles: a layer has at most two chunk
// pairs, so every B fragment of it is read before the first MFMA; acc holds
// the starting values, and the products enter scaled by 2^(sc - 127).
template <int T, int NCH, int NT>
__device__ __forceinline__ void layer_acc_fp8_tiles(const uint4 (&A)[T][NCH], const uint8_t* bp, int sin, int sc,
                                                    floatx4 (&acc)[T][Rows<kFP8>::kRTT])
{
    constexpr int kc = Traits<kFP8>::kChunk, NP = NCH / 2;
    static_assert(NCH % 2 == 0, "FP8 inputs are padded to chunk pairs");
    uint4 b0[NP][NT], b1[NP][NT];
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int rt = 0; rt < NT; ++rt) {
            b0[q][rt] = *reinterpret_cast<const uint4*>(bp + rt * 16 * sin + 2 * q * kc);
            b1[q][rt] = *reinterpret_cast<const uint4*>(bp + rt * 16 * sin + (2 * q + 1) * kc);
        }
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int rt = 0; rt < NT; ++rt)
#pragma unroll
            for (int tt = 0; tt < T; ++tt)
                mma_pair_scaled<kFP8>(A[tt][2 * q], A[tt][2 * q + 1], b0[q][rt], b1[q][rt], acc[tt][rt], sc);
}

template <int T, int NCH, int NT>
__device__ __forceinline__ void layer_acc_fp8(const uint4 (&A)[T][NCH], const uint8_t* bp, int sin, int art, int sc,
                                              floatx4 (&acc)[T][Rows<kFP8>::kRTT])
{
    if (art == NT)
        layer_acc_fp8_tiles<T, NCH, NT>(A, bp, sin, sc, acc);
    else if constexpr (NT > 1)
        layer_acc_fp8<T, NCH, NT - 1>(A, bp, sin, art, sc, acc);
}

// One layer with register-resident A fragments: out = act(A * in) for the
// wave's T neuron tiles over `art` row tiles. FP8: the output in the next
// layer's input scale is ReLU(deq A in + b) inv_next = ReLU(c1 A in +
// b inv_next) with c1 = deq inv_next a power of two, so the accumulators
// start at b inv_next, the products enter through the MFMA block scale c1,
// and the epilogue is the clamp and the conversion alone.
template <int P, int T, int NCH>
__device__ __forceinline__ void layer_regs(const uint4 (&A)[T][NCH], int nch, const uint8_t* in, int sin,
                                           uint8_t* out, int sout, const float* bias, float deq, float inv_next,
                                           int art, int wave, int g, int c16)
{
    constexpr int es = Traits<P>::kEsize, kRTT = Rows<P>::kRTT;
    floatx4 acc[T][kRTT];
    if constexpr (P == kFP8) {
        const int sc = e8m0_of(deq * inv_next);
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            const float* bb = bias + (wave + kWaves * tt) * 16 + g * 4;
            const floatx4 b4 = {bb[0] * inv_next, bb[1] * inv_next, bb[2] * inv_next, bb[3] * inv_next};
#pragma unroll
            for (int rt = 0; rt < kRTT; ++rt)
                acc[tt][rt] = b4;
        }
        layer_acc_fp8<T, NCH, kRTT>(A, in + c16 * sin + g * (Traits<P>::kChunk / 4) * es, sin, art, sc, acc);
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            const int nt = wave + kWaves * tt;
#pragma unroll
            for (int rt = 0; rt < kRTT; ++rt)
                if (rt < art)
                    store_act4<P>(out + (rt * 16 + c16) * sout + (nt * 16 + g * 4) * es, acc[tt][rt][0],
                                  acc[tt][rt][1], acc[tt][rt][2], acc[tt][rt][3]);
        }
    } else {
        layer_acc<P, T, NCH>(A, nch, in, sin, art, g, c16, acc);
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            const int nt = wave + kWaves * tt;
            const float* bb = bias + nt * 16 + g * 4;
            const float b0 = bb[0], b1 = bb[1], b2 = bb[2], b3 = bb[3];
#pragma unroll
            for (int rt = 0; rt < kRTT; ++rt) {
                if (rt < art) {
                    store4<P>(out + (rt * 16 + c16) * sout + (nt * 16 + g * 4) * es,
                              fmaxf(acc[tt][rt][0] * deq + b0, 0.f), fmaxf(acc[tt][rt][1] * deq + b1, 0.f),
                              fmaxf(acc[tt][rt][2] * deq + b2, 0.f), fmaxf(acc[tt][rt][3] * deq + b3, 0.f),
                              inv_next);
                }
            }
        }
    }
}

// Actor forward pass on the matrix cores over nrows <= 64 rows whose
// per-node inputs are in bufA. The output layer's reduction is split over the
// waves: it leaves one partial logit tile per wave, [wave][row][16] floats, in
// the buffer returned (the enforcer adds them up). bias: LDS copy of every
// layer's bias.
template <int P, int T, int CH1, int CHH, int NHH>
__device__ __forceinline__ float* mlp_mfma(const DevTree& t, const WaveWeights<P, T, CH1, CHH, NHH>& W, int nrows,
                                           uint8_t* bufA, uint8_t* bufB, const float* bias, const int* bias_off)
{
    using WW = WaveWeights<P, T, CH1, CHH, NHH>;
    constexpr int kc = Traits<P>::kChunk, es = Traits<P>::kEsize, kRTT = Rows<P>::kRTT, kRT = Rows<P>::kRT;
    const int lane = threadIdx.x & 63, wave = wave_id(), g = lane >> 4, c16 = lane & 15;
    const int art = (nrows + 15) >> 4;
    constexpr int s0 = CH1 * kc * es + 16, sh = CHH * kc * es + 16;
    layer_regs<P, T, CH1>(W.w1, CH1, bufA, s0, bufB, sh, bias + bias_off[0], t.deq[0], t.inv_in_scale[1], art, wave,
                          g, c16);
    lds_barrier();
    if constexpr ((P == kFP32 || P == kBF16) && NHH > 0) {
        // The last hidden layer feeds the output layer from registers. Lane
        // (g, c16)'s accumulator of tile tt holds neurons 16 nt + 4g ..
        // 16 nt + 4g + 3 of row rt*16 + c16: the B fragment of a 16-deep step
        // of the output layer over tile nt (FP32: the 16x16x4 chunk nt, this
        // wave's W.wo[tt]; BF16: one 16x16x16 MFMA with W.wo16[tt], the
        // activations rounded to BF16 as an LDS store would). Its activations
        // never go to LDS.
        static_assert(P != kFP32 || WW::CPW == T, "output-layer chunks are the wave's own tiles");
        floatx4 hacc[T][kRTT];
        layer_acc<P, T, CHH>(W.wh, CHH, bufB, sh, art, g, c16, hacc);
        floatx4 acc[kRTT];
#pragma unroll
        for (int rt = 0; rt < kRTT; ++rt)
            acc[rt] = floatx4{0.f, 0.f, 0.f, 0.f};
        const float deq = t.deq[1];
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            const float* bb = bias + bias_off[1] + (wave + kWaves * tt) * 16 + g * 4;
            const float b0 = bb[0], b1 = bb[1], b2 = bb[2], b3 = bb[3];
#pragma unroll
            for (int rt = 0; rt < kRTT; ++rt)
                if (rt < art) {
                    const float h0 = fmaxf(hacc[tt][rt][0] * deq + b0, 0.f);
                    const float h1 = fmaxf(hacc[tt][rt][1] * deq + b1, 0.f);
                    const float h2 = fmaxf(hacc[tt][rt][2] * deq + b2, 0.f);
                    const float h3 = fmaxf(hacc[tt][rt][3] * deq + b3, 0.f);
                    if constexpr (P == kFP32) {
                        const uint4 h = {__float_as_uint(h0), __float_as_uint(h1), __float_as_uint(h2),
                                         __float_as_uint(h3)};
                        mma_chunk<P>(W.wo[tt], h, acc[rt]);
                    } else {
                        const uint2 h = {bf16x2_bits(h0, h1), bf16x2_bits(h2, h3)};
                        acc[rt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                            __builtin_bit_cast(short4v, W.wo16[tt]), __builtin_bit_cast(short4v, h), acc[rt], 0, 0, 0);
                    }
                }
        }
        // bufA (the inputs, consumed before the last barrier) takes the partials
        float* part = reinterpret_cast<float*>(bufA);
#pragma unroll
        for (int rt = 0; rt < kRTT; ++rt)
            if (rt < art)
                *reinterpret_cast<floatx4*>(part + (size_t)(wave * kRT + rt * 16 + c16) * 16 + g * 4) = acc[rt];
        lds_barrier();
        return part;
    }
    if constexpr (P == kFP8 && NHH > 0) {
        // The last hidden layer feeds the output layer from registers, as
        // above: its accumulators start at b inv_next and take the products
        // through the block scale, so ReLU and the E4M3 rounding (what an LDS
        // store would keep) are the whole epilogue; lane (g, c16) then holds
        // the E4M3 activations of neurons 16 nt + 4g .. + 3 of its row for each
        // of its tiles, the B fragment of a 16x16x32 FP8 step over a pair of
        // tiles, with W.wo8 as the matching A fragment.
        const float inv_next = t.inv_in_scale[2];
        const int sc = e8m0_of(t.deq[1] * inv_next);
        floatx4 hacc[T][kRTT];
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            const float* bb = bias + bias_off[1] + (wave + kWaves * tt) * 16 + g * 4;
            const floatx4 b4 = {bb[0] * inv_next, bb[1] * inv_next, bb[2] * inv_next, bb[3] * inv_next};
#pragma unroll
            for (int rt = 0; rt < kRTT; ++rt)
                hacc[tt][rt] = b4;
        }
        layer_acc_fp8<T, CHH, kRTT>(W.wh, bufB + c16 * sh + g * (kc / 4) * es, sh, art, sc, hacc);
        floatx4 acc[kRTT];
#pragma unroll
        for (int rt = 0; rt < kRTT; ++rt)
            acc[rt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int rt = 0; rt < kRTT; ++rt)
            if (rt < art) {
#pragma unroll
                for (int q = 0; q < (T + 1) / 2; ++q) {
                    const uint32_t lo = act4_e4m3(hacc[2 * q][rt][0], hacc[2 * q][rt][1], hacc[2 * q][rt][2],
                                                  hacc[2 * q][rt][3]);
                    const uint32_t hi = 2 * q + 1 < T ? act4_e4m3(hacc[2 * q + 1][rt][0], hacc[2 * q + 1][rt][1],
                                                                  hacc[2 * q + 1][rt][2], hacc[2 * q + 1][rt][3])
                                                      : 0u;
                    const long a = (long)(((uint64_t)W.wo8[q].y << 32) | W.wo8[q].x);
                    const long b = (long)(((uint64_t)hi << 32) | lo);
                    acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, acc[rt], 0, 0, 0);
                }
            }
        float* part = reinterpret_cast<float*>(bufA);
#pragma unroll
        for (int rt = 0; rt < kRTT; ++rt)
            if (rt < art)
                *reinterpret_cast<floatx4*>(part + (size_t)(wave * kRT + rt * 16 + c16) * 16 + g * 4) = acc[rt];
        lds_barrier();
        return part;
    }
    uint8_t* in = bufB;
    uint8_t* out = bufA;
    if constexpr (NHH > 0) {
        layer_regs<P, T, CHH>(W.wh, CHH, bufB, sh, bufA, sh, bias + bias_off[1], t.deq[1], t.inv_in_scale[2], art,
                              wave, g, c16);
        lds_barrier();
        in = bufA;
        out = bufB;
    }
    // output layer: this wave's slice of the reduction, partial tile to LDS
    float* part = reinterpret_cast<float*>(out);
    floatx4 acc[kRTT];
#pragma unroll
    for (int rt = 0; rt < kRTT; ++rt)
        acc[rt] = floatx4{0.f, 0.f, 0.f, 0.f};
    const uint8_t* bp = in + c16 * sh + g * (kc / 4) * es;
#pragma unroll
    for (int j = 0; j < WW::CPW; ++j) {
        const int c = wave + kWaves * j;
        if (c < CHH) {
#pragma unroll
            for (int rt = 0; rt < kRTT; ++rt)
                if (rt < art) {
                    const uint4 b = *reinterpret_cast<const uint4*>(bp + rt * 16 * sh + c * kc * es);
                    mma_chunk<P>(W.wo[j], b, acc[rt]);
                }
        }
    }
#pragma unroll
    for (int rt = 0; rt < kRTT; ++rt)
        if (rt < art)
            *reinterpret_cast<floatx4*>(part + (size_t)(wave * kRT + rt * 16 + c16) * 16 + g * 4) = acc[rt];
    lds_barrier();
    return part;
}

}  // namespace

}  // namespace cyrus
