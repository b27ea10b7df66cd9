// The subtree algorithm of one codebook, as one workgroup runs it for the
// subtree below node r of level `split`: the `split` ancestors of that node
// from the root (one evaluation each, recomputed redundantly by the
// workgroups that share them; the first descendant writes them), then the
// subtree level by level with workgroup barriers only. Nodes below different
// level-`split` nodes never interact, so no synchronisation between
// workgroups is needed. Run by the subtree kernel (one workgroup per subtree
// root, the whole codebook in one launch) and by the resident serving worker
// (one claimed root at a time).
//
// Every wave loads its share of the actor into registers once (the MFMA A
// fragments of its output-neuron tiles, plus its slice of the output layer's
// reduction dimension); afterwards each level step only moves node
// activations through LDS. The first 3E inputs (R, MCS, SINR) are the same for
// every node of the tree, so their part of the first layer is computed once
// per workgroup and folded into that layer's bias; node rows then carry only
// their E + 2 own inputs (c, tau, k). Waves meet at LDS-only barriers: the
// body never reads back what it writes to global memory, so codebook stores
// (to HBM or, for host builds, to pinned host memory) stay in flight across
// steps.
//
// COH (the resident worker): the UE state is read, and the codebook written,
// with agent-scope relaxed atomics, which bypass the per-XCD caches: another
// workgroup of the same launch wrote the state and delivers the codebook.
#pragma once

#include "cyrus_device.h"
#include "cyrus_regmlp.h"

namespace cyrus {

namespace {

template <bool COH>
__device__ __forceinline__ void put_byte(uint8_t* base, int64_t i, uint8_t v)
{
    if constexpr (COH)
        __hip_atomic_store(base + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        base[i] = v;
}

template <bool COH>
__device__ __forceinline__ int32_t load_i32(const int32_t* base, int i)
{
    if constexpr (COH)
        return __hip_atomic_load(base + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        return base[i];
}

__device__ __forceinline__ int64_t sub_level_offset(int K, int tau)
{
    int64_t p = 1;
    for (int i = 0; i < tau; ++i)
        p *= (K + 1);
    return (p - 1) / K;
}

// Gaussian-head draw slots of one subtree workgroup: one row per ancestor
// level, then every evaluated row of the subtree levels, sum over d of
// K (K+1)^(d-1) = (K+1)^(M-split) - 1.
__host__ __device__ inline int eps_slots(int K, int M, int split)
{
    int w = 1;
    for (int i = 0; i < M - split; ++i)
        w *= K + 1;
    return split + w - 1;
}

__device__ __forceinline__ int ipow_dev(int b, int e)
{
    int r = 1;
    for (int i = 0; i < e; ++i)
        r *= b;
    return r;
}

// FP32, few rows: the same register-resident fragments used as a GEMV on
// the vector ALU. Lane (g, i) holds W[n0 + i][16c + 4g + j]; it multiplies its
// four weights of every chunk with the matching inputs, and the four lane
// groups are summed with two butterfly steps, so each lane ends with the
// whole dot product of neuron n0 + i (row swaps on the vector ALU, no LDS).
// Rows go one after the other: the weights already fill most of the register
// file.
template <int T>
__device__ __forceinline__ void valu_store(const float (&acc)[T], float* out, const float (&bias)[T], int wave,
                                           int g, int c16)
{
#pragma unroll
    for (int tt = 0; tt < T; ++tt) {
        const float v = row_sum4(acc[tt]);
        const int n = (wave + kWaves * tt) * 16 + c16;
        if (g == 0)
            out[n] = fmaxf(v + bias[tt], 0.f);
    }
}

// Biases of the first two layers for the neurons a lane sums in the
// vector-ALU steps (neuron 16 (wave + kWaves tt) + c16 of each of its tiles),
// read from LDS once per launch.
template <int T>
struct ValuBias {
    float b1[T];
    float b2[T];
};

template <int T, int NCH>
__device__ __forceinline__ void valu_fma4(const uint4 (&A)[T][NCH], int c, const float (&h)[4], float (&acc)[T])
{
#pragma unroll
    for (int tt = 0; tt < T; ++tt) {
        acc[tt] = fmaf(__uint_as_float(A[tt][c].x), h[0], acc[tt]);
        acc[tt] = fmaf(__uint_as_float(A[tt][c].y), h[1], acc[tt]);
        acc[tt] = fmaf(__uint_as_float(A[tt][c].z), h[2], acc[tt]);
        acc[tt] = fmaf(__uint_as_float(A[tt][c].w), h[3], acc[tt]);
    }
}

// FP32 actor pass over nrows <= 4 rows on the vector ALU. The first layer
// forms its inputs [c/64 | tau/8 | k/8] in registers from the state rows in
// LDS (state_of(row), k_of(row)), so no feature rows are written and no
// barrier precedes it. Returns the per-wave partial logit tiles, as mlp_mfma
// does.
template <int T, int CH1, int CHH, int NHH, class StateOf, class KOf>
__device__ __forceinline__ float* mlp_valu(const DevTree& t, const WaveWeights<kFP32, T, CH1, CHH, NHH>& W,
                                           int nrows, uint8_t* bufA, uint8_t* bufB, const ValuBias<T>& vb, int tau,
                                           StateOf state_of, KOf k_of)
{
    using WW = WaveWeights<kFP32, T, CH1, CHH, NHH>;
    constexpr int kRT = Rows<kFP32>::kRT;
    constexpr int sh = CHH * 16 + 4;  // hidden row stride in floats (16-byte pad)
    const int lane = threadIdx.x & 63, wave = wave_id(), g = lane >> 4, c16 = lane & 15;
    const int E = t.E;
    float* hA = reinterpret_cast<float*>(bufA);
    float* hB = reinterpret_cast<float*>(bufB);
    const float ftau = (float)tau * (1.f / 8.f);
#pragma unroll 1
    for (int r = 0; r < nrows; ++r) {
        float acc[T];
#pragma unroll
        for (int tt = 0; tt < T; ++tt)
            acc[tt] = 0.f;
        const uint8_t* st = state_of(r);
        const float fk = (float)k_of(r) * (1.f / 8.f);
#pragma unroll
        for (int c = 0; c < CH1; ++c) {
            // every lane reads four state bytes (clamped into the row, so the
            // reads need no branch) and keeps those that are inputs
            uint32_t sb[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                sb[j] = st[min(16 * c + 4 * g + j, E - 1)];
            float h[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int f = 16 * c + 4 * g + j;
                const float sv = (float)sb[j] * (1.f / 64.f);
                const float tv = f == E ? ftau : fk;
                const float ov = f <= E + 1 ? tv : 0.f;
                h[j] = f < E ? sv : ov;
            }
            valu_fma4<T, CH1>(W.w1, c, h, acc);
        }
        valu_store<T>(acc, hB + r * sh, vb.b1, wave, g, c16);
    }
    lds_barrier();
    float* in = hB;
    float* out = hA;
    if constexpr (NHH > 0) {
        // The hidden layer feeds the output layer without LDS: after the
        // row sums every lane holds neuron 16 nt + c16 of each of its tiles,
        // and lane (g, i) takes neurons 16 nt + 4g .. 16 nt + 4g + 3 (its
        // output weights W.wo[tt] of chunk nt) from lanes 4g .. 4g + 3 of its
        // own row. The partial logits go to bufA, which no wave reads now.
        static_assert(WW::CPW == T, "output-layer chunks are the wave's own tiles");
        float* part = hA;
        // The hidden row is read in batches of four chunks, each batch loaded
        // while the previous one's FMAs run; the scheduling barriers keep the
        // loads ahead (the compiler otherwise issues one 16-byte load per
        // chunk and waits for it, to save registers).
        constexpr int kBatch = 4;
        static_assert(CHH % kBatch == 0, "hidden chunks come in batches of four");
        const int src = (lane & 48) | (4 * g);
#pragma unroll 1
        for (int r = 0; r < nrows; ++r) {
            float acc[T];
#pragma unroll
            for (int tt = 0; tt < T; ++tt)
                acc[tt] = 0.f;
            const float* hr = hB + r * sh + 4 * g;
            floatx4 hv[kBatch], hn4[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; ++j)
                hv[j] = *reinterpret_cast<const floatx4*>(hr + 16 * j);
#pragma unroll
            for (int c0 = 0; c0 < CHH; c0 += kBatch) {
                if (c0 + kBatch < CHH) {
#pragma unroll
                    for (int j = 0; j < kBatch; ++j)
                        hn4[j] = *reinterpret_cast<const floatx4*>(hr + 16 * (c0 + kBatch + j));
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int j = 0; j < kBatch; ++j) {
                    const float h[4] = {hv[j][0], hv[j][1], hv[j][2], hv[j][3]};
                    valu_fma4<T, CHH>(W.wh, c0 + j, h, acc);
                }
                __builtin_amdgcn_sched_barrier(0);
                if (c0 + kBatch < CHH) {
#pragma unroll
                    for (int j = 0; j < kBatch; ++j)
                        hv[j] = hn4[j];
                }
            }
            // every tile's four permutes are issued before the first is used
            float hn[T][4];
#pragma unroll
            for (int tt = 0; tt < T; ++tt) {
                const float h = fmaxf(row_sum4(acc[tt]) + vb.b2[tt], 0.f);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    hn[tt][j] = __shfl(h, src + j);
            }
            __builtin_amdgcn_sched_barrier(0);
            float z = 0.f;
#pragma unroll
            for (int tt = 0; tt < T; ++tt) {
                z = fmaf(__uint_as_float(W.wo[tt].x), hn[tt][0], z);
                z = fmaf(__uint_as_float(W.wo[tt].y), hn[tt][1], z);
                z = fmaf(__uint_as_float(W.wo[tt].z), hn[tt][2], z);
                z = fmaf(__uint_as_float(W.wo[tt].w), hn[tt][3], z);
            }
            z = row_sum4(z);
            if (g == 0)
                part[(size_t)(wave * kRT + r) * 16 + c16] = z;
        }
        lds_barrier();
        return part;
    }
    // output layer: this wave's slice of the reduction, one partial tile
    float* part = out;
#pragma unroll 1
    for (int r = 0; r < nrows; ++r) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < WW::CPW; ++j) {
            const int c = wave + kWaves * j;
            if (c < CHH) {
                const floatx4 h = *reinterpret_cast<const floatx4*>(in + r * sh + 4 * g + 16 * c);
                acc = fmaf(__uint_as_float(W.wo[j].x), h[0], acc);
                acc = fmaf(__uint_as_float(W.wo[j].y), h[1], acc);
                acc = fmaf(__uint_as_float(W.wo[j].z), h[2], acc);
                acc = fmaf(__uint_as_float(W.wo[j].w), h[3], acc);
            }
        }
        acc = row_sum4(acc);
        if (g == 0)
            part[(size_t)(wave * kRT + r) * 16 + c16] = acc;
    }
    lds_barrier();
    return part;
}

struct SubtreeSmem {
    uint8_t* bufA;
    uint8_t* bufB;
    float* zl;
    int* R;         // kMaxUE
    int* misc;      // [0] = sum R, [1..kMaxLayers] = bias offsets
    float* statf;   // 3 * kMaxUE static features: R/32, MCS/32, SINR/32
    float* bias;    // every layer's bias, out_pad each
    uint8_t* st0;   // states of the previous level (local nodes), E bytes each
    uint8_t* st1;   // states of the current level
    float* eps;     // Gaussian head: the draws of every evaluated node, E each
};

// Per-node input rows for `nrows` nodes: [c/64 | tau/8 | k/8], zero padded
// to in_pad_d, with state c from state_of(row), level tau and arrival
// arrival_of(row). One thread per four consecutive inputs of a row (so a
// single row still spreads over many lanes); groups past the E + 2 values
// are zeros.
template <int P, int CH1, class StateOf, class ArrivalOf>
__device__ __forceinline__ void write_features(const DevTree& t, const SubtreeSmem& sm, int nrows, int tau,
                                               StateOf state_of, ArrivalOf arrival_of)
{
    constexpr int es = Traits<P>::kEsize, in0 = CH1 * Traits<P>::kChunk, s0 = in0 * es + 16;
    constexpr int ngr = in0 / 4;  // groups of four inputs per row
    static_assert(kThreads % ngr == 0, "whole rows per pass");
    const int E = t.E;
    // MFMA passes read whole 16-row tiles: rows past nrows are zeroed so they
    // stay finite (each output row depends on its own input row only)
    const int nrows_pad = ((nrows + 15) >> 4) << 4;
    const float inv0 = t.inv_in_scale[0], ftau = (float)tau * (1.f / 8.f);
    const int grp = threadIdx.x % ngr, fb = grp * 4;
    for (int row = threadIdx.x / ngr; row < nrows_pad; row += kThreads / ngr) {
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        if (row < nrows && fb <= E + 1) {
            const uint8_t* st = state_of(row);
            const float fk = (float)arrival_of(row) * (1.f / 8.f);
            // every state byte is read, and blended in by a multiply, so the
            // reads are issued together rather than each behind a branch
            uint32_t sb[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                sb[j] = st[min(fb + j, E - 1)];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int f = fb + j;
                v[j] = (float)sb[j] * (f < E ? 1.f / 64.f : 0.f) + (f == E ? ftau : 0.f) + (f == E + 1 ? fk : 0.f);
            }
        }
        store4<P>(sm.bufA + row * s0 + fb * es, v[0], v[1], v[2], v[3], inv0);
    }
}

// One actor pass over the nrows nodes of a step: the FP32 vector-ALU path for
// up to four rows, else the per-node input rows and the matrix-core path.
template <int P, int T, int CH1, int CHH, int NHH, class StateOf, class KOf>
__device__ __forceinline__ const float* eval_rows(const DevTree& t, const SubtreeSmem& sm,
                                                  const WaveWeights<P, T, CH1, CHH, NHH>& W,
                                                  const ValuBias<T>& vb, int nrows, int tau, const int* bias_off,
                                                  StateOf state_of, KOf k_of)
{
    if constexpr (P == kFP32) {
        if (nrows <= 4)
            return mlp_valu<T, CH1, CHH, NHH>(t, W, nrows, sm.bufA, sm.bufB, vb, tau, state_of, k_of);
    }
    write_features<P, CH1>(t, sm, nrows, tau, state_of, k_of);
    lds_barrier();
    return mlp_mfma<P, T, CH1, CHH, NHH>(t, W, nrows, sm.bufA, sm.bufB, sm.bias, bias_off);
}

// Enforcer over `nrows` rows, G lanes per row (lane e = UE e). Each lane first
// adds up its logit from the per-wave partial tiles (fixed wave order) plus
// the bias. Row r has arrival k_of(r), input state cin_of(r); it writes its
// state to sout_of(r) (LDS) and, when node_of(r) >= 0, the node's allocation
// (and logits) to global memory; when sib_of(r) >= 0 (the first child of a
// parent) it also writes that k = 0 sibling: nothing punctured, parent state
// passed on, into sib_st_of(r). Node states stay in LDS: no later launch
// reads them on this path (the level kernels keep their own state array).
template <int G, int RT, bool EXT, bool COH, class KOf, class CinOf, class SoutOf, class EpsOf, class NodeOf,
          class SibOf, class SibStOf>
__device__ __forceinline__ void finish_rows(const DevTree& t, const SubtreeSmem& sm, const float* part, float deq,
                                            const float* bo, int nrows, KOf k_of, CinOf cin_of, SoutOf sout_of,
                                            EpsOf eps_of, NodeOf node_of, SibOf sib_of, SibStOf sib_st_of)
{
    const int E = t.E;
    for (int base = 0; base < nrows; base += kThreads / G) {
        const int row = base + (int)threadIdx.x / G, e = (int)threadIdx.x % G;
        if (row < nrows) {
            // every LDS value of the row is requested before the first add:
            // the UE's caps and parent state, then the partial logits
            const int k = k_of(row);
            const int R = e < E ? sm.R[e] : 0;
            const int rsum = sm.misc[0];
            const uint8_t c = e < E ? cin_of(row)[e] : (uint8_t)0;
            float z = 0.f;
            if (e < E) {
                // (the adds keep the wave order)
                float pw[kWaves];
#pragma unroll
                for (int w = 0; w < kWaves; ++w)
                    pw[w] = part[(size_t)(w * RT + row) * 16 + e];
                const float be = bo[e];
                float acc = 0.f;
#pragma unroll
                for (int w = 0; w < kWaves; ++w)
                    acc += pw[w];
                z = acc * deq + be;
                if (EXT && t.head == kGaussianHead) {  // one output tile: mu (0..E-1), log sigma (E..2E-1)
                    float acc2 = 0.f;
#pragma unroll
                    for (int w = 0; w < kWaves; ++w)
                        acc2 += part[(size_t)(w * RT + row) * 16 + E + e];
                    z = gaussian_log_share_eps(z, acc2 * deq + bo[E + e], eps_of(row)[e]);
                }
            }
            const int a = enforce_dpp<G>(E, e, z, R, rsum, t.U * k, sm.zl + row * kLogitStride,
                                         EXT ? t.rounding : (int)kLargestRemainder);
            const uint8_t st = (uint8_t)(c + a);
            if (e < E) {
                sout_of(row)[e] = st;
                const int64_t node = node_of(row);
                if (node >= 0) {
                    put_byte<COH>(t.alloc, node * E + e, (uint8_t)a);
                    if (t.logits)
                        t.logits[node * E + e] = z;
                }
                const int64_t sib = sib_of(row);
                if (sib >= 0) {
                    sib_st_of(row)[e] = c;
                    put_byte<COH>(t.alloc, sib * E + e, 0);
                    if (t.logits)
                        t.logits[sib * E + e] = 0.f;
                }
            }
        }
    }
}

template <int P, int T, int CH1, int CHH, int NHH, int G, bool EXT, bool COH>
__device__ __forceinline__ void subtree_body(const DevTree& t, int split, int r, int bufsize, int stbytes,
                                             uint8_t* smem)
{
    SubtreeSmem sm;
    sm.bufA = smem;
    sm.bufB = smem + bufsize;
    sm.zl = reinterpret_cast<float*>(smem + 2 * bufsize);
    sm.R = reinterpret_cast<int*>(sm.zl + kRTmax * kLogitStride);
    sm.misc = sm.R + kMaxUE;
    sm.statf = reinterpret_cast<float*>(sm.misc + 8);
    sm.bias = sm.statf + 3 * kMaxUE;
    int nbias = 0;
    for (int l = 0; l < t.n_layers; ++l)
        nbias += t.out_pad[l];
    sm.st0 = reinterpret_cast<uint8_t*>(sm.bias + nbias);
    sm.st1 = sm.st0 + stbytes;
    sm.eps = reinterpret_cast<float*>(
        (reinterpret_cast<uintptr_t>(sm.st1 + stbytes) + 15) & ~static_cast<uintptr_t>(15));

    const int lane = threadIdx.x & 63, wave = wave_id();
    const int E = t.E, K = t.K, M = t.M, K1 = K + 1;

    // Global loads, issued in the order they are consumed and the register-
    // resident weights last, so that the set-up below waits for nothing
    // behind it: the UE state, every layer's bias (tid < out_pad), and the
    // static-input fragments of neuron tid of the first layer.
    constexpr int NL = NHH + 2;                                   // layers
    constexpr int kc = Traits<P>::kChunk, per = kc / 4;           // inputs per 16-byte fragment
    constexpr int NQ = 3 * 16 / per;                              // static fragments per neuron, E <= 16
    const int tid = threadIdx.x, n_stat = 3 * E;
    int32_t ue_rb = 0, ue_mcs = 0, ue_sinr = 0;
    if (tid < E) {
        ue_rb = load_i32<COH>(t.ue, tid);
        ue_mcs = load_i32<COH>(t.ue, E + tid);
        ue_sinr = load_i32<COH>(t.ue, 2 * E + tid);
    }
    float bl[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l)
        bl[l] = tid < t.out_pad[l] ? t.b[l][tid] : 0.f;
    // inputs q*per .. q*per + per - 1 of neuron n sit in chunk q / 4, lane
    // 16 * (q % 4) + n % 16 of n's tile in the full-width layout
    uint4 sw[NQ];
    {
        const int nch = t.in_pad[0] / kc;
        const uint4* g = reinterpret_cast<const uint4*>(t.w[0]);
        const bool mine = tid < t.out_pad[0];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            sw[q] = (mine && q * per < n_stat) ? g[((size_t)(tid >> 4) * nch + q / 4) * 64 + 16 * (q % 4) + (tid & 15)]
                                               : uint4{0, 0, 0, 0};
    }
    WaveWeights<P, T, CH1, CHH, NHH> W;
    load_weights(t, W, wave, lane);

    if (tid < E) {
        sm.R[tid] = ue_rb;
        sm.statf[tid] = (float)ue_rb * (1.f / 32.f);
        sm.statf[E + tid] = (float)ue_mcs * (1.f / 32.f);
        sm.statf[2 * E + tid] = __int_as_float(ue_sinr) * (1.f / 32.f);
        sm.st0[tid] = 0;  // root state
    }
    if (wave == 0) {
        // total RBs (E <= 16: lanes 0..15) and the bias offsets
        int v = lane < E ? ue_rb : 0;
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        if (lane == 0) {
            sm.misc[0] = v;
            int off = 0;
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                sm.misc[1 + l] = off;
                off += t.out_pad[l];
            }
        }
    }
    {
        int off = t.out_pad[0];
#pragma unroll
        for (int l = 1; l < NL; ++l) {
            if (tid < t.out_pad[l])
                sm.bias[off + tid] = bl[l];
            off += t.out_pad[l];
        }
    }
    if constexpr (EXT) {
        if (t.head == kGaussianHead) {
            // The draws depend on (node, UE, seed, TTI) only, so every node
            // this workgroup evaluates gets its E draws here, all threads at
            // once, while the register weights stream in. Slot tau - 1 holds
            // ancestor level tau; the subtree levels follow, row j of level
            // split + d at its level's offset + j.
            const int nsub = eps_slots(K, M, split) - split;
            for (int f = tid; f < (split + nsub) * E; f += kThreads) {
                const int slot = f / E, e = f - slot * E;
                int64_t node;
                if (slot < split) {
                    const int tau = slot + 1;
                    node = sub_level_offset(K, tau) + r / ipow_dev(K1, split - tau);
                } else {
                    int j = slot - split, d = 1, n = K;
                    while (j >= n) {
                        j -= n;
                        n *= K1;
                        ++d;
                    }
                    const int p = j / K, k = j - p * K + 1;
                    node = sub_level_offset(K, split + d) + (int64_t)r * ipow_dev(K1, d) + p * K1 + k;
                }
                sm.eps[f] = gaussian_eps(t.seed, t.tti, node, e);
            }
        }
    }
    lds_barrier();
    // first-layer bias with the static inputs folded in, from the values the
    // MFMA would read: the stored weights and the inputs in the storage type
    if (tid < t.out_pad[0]) {
        const float inv0 = t.inv_in_scale[0];
        float acc = 0.f;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (q * per < n_stat) {
#pragma unroll
                for (int j = 0; j < per; ++j) {
                    const int f = q * per + j;
                    if (f < n_stat)
                        acc = fmaf(frag_value<P>(sw[q], j), stored_value<P>(sm.statf[f], inv0), acc);
                }
            }
        }
        sm.bias[tid] = bl[0] + t.deq[0] * acc;
    }
    lds_barrier();
    const int* bias_off = sm.misc + 1;
    ValuBias<T> vb;
    if constexpr (P == kFP32) {
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            const int n = (wave + kWaves * tt) * 16 + (lane & 15);
            vb.b1[tt] = sm.bias[bias_off[0] + n];
            vb.b2[tt] = NHH > 0 ? sm.bias[bias_off[1] + n] : 0.f;
        }
    }
    const float deq_out = t.deq[NHH + 1];
    const float* bias_out = sm.bias + bias_off[NHH + 1];
    constexpr int kRT = Rows<P>::kRT;

    // ---- ancestors of subtree root r, levels 1..split. The current state is
    // sm.st0[0..E); a k = 0 ancestor punctures nothing and leaves it as is.
    for (int tau = 1; tau <= split; ++tau) {
        const int below = ipow_dev(K1, split - tau);
        const int idx = r / below;  // index of the ancestor within level tau
        const int k = idx % K1;
        const int64_t node = sub_level_offset(K, tau) + idx;
        const bool owner = (r % below) == 0;
        if (k > 0) {
            const float* part = eval_rows<P, T, CH1, CHH, NHH>(
                t, sm, W, vb, 1, tau, bias_off, [&](int) { return sm.st0; }, [&](int) { return k; });
            finish_rows<G, kRT, EXT, COH>(
                t, sm, part, deq_out, bias_out, 1, [&](int) { return k; }, [&](int) { return sm.st0; },
                [&](int) { return sm.st1; }, [&](int) { return sm.eps + (tau - 1) * E; },
                [&](int) { return owner ? node : (int64_t)-1; },
                [&](int) { return (int64_t)-1; }, [&](int) { return sm.st1; });
            lds_barrier();
            uint8_t* tmp = sm.st0;
            sm.st0 = sm.st1;
            sm.st1 = tmp;
        } else if (owner && threadIdx.x < E) {
            put_byte<COH>(t.alloc, node * E + threadIdx.x, 0);
            if (t.logits)
                t.logits[node * E + threadIdx.x] = 0.f;
        }
    }

    // ---- subtree levels split+1..M; st0 holds the previous level's states
    const float invK = 1.0f / (float)K;
    int eps_row = split;  // first slot of this level's draws
    for (int tau = split + 1; tau <= M; ++tau) {
        const int d = tau - split;
        const int width = ipow_dev(K1, d);
        const int n_eval = K * (width / K1);
        const int64_t base = sub_level_offset(K, tau) + (int64_t)r * width;
        uint8_t* prev = sm.st0;
        uint8_t* cur = sm.st1;
        for (int j0 = 0; j0 < n_eval; j0 += kRT) {
            const int nrows = min(kRT, n_eval - j0);
            // row j of the level: parent p = j / K, arrival k = j % K + 1
            auto parent_of = [&](int row) { return (int)(((float)(j0 + row) + 0.5f) * invK); };
            auto k_of = [&](int row) { return j0 + row - parent_of(row) * K + 1; };
            const float* part = eval_rows<P, T, CH1, CHH, NHH>(
                t, sm, W, vb, nrows, tau, bias_off, [&](int row) { return prev + parent_of(row) * E; }, k_of);
            finish_rows<G, kRT, EXT, COH>(
                t, sm, part, deq_out, bias_out, nrows, k_of, [&](int row) { return prev + parent_of(row) * E; },
                [&](int row) { return cur + (parent_of(row) * K1 + k_of(row)) * E; },
                [&](int row) { return sm.eps + (eps_row + j0 + row) * E; },
                [&](int row) { return base + parent_of(row) * K1 + k_of(row); },
                [&](int row) { return k_of(row) == 1 ? base + parent_of(row) * K1 : (int64_t)-1; },
                [&](int row) { return cur + parent_of(row) * K1 * E; });
            lds_barrier();
        }
        eps_row += n_eval;
        uint8_t* tmp = sm.st0;
        sm.st0 = sm.st1;
        sm.st1 = tmp;
    }
}

}  // namespace

}  // namespace cyrus
