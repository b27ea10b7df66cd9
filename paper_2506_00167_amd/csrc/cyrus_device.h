// Device-side building blocks of the codebook builder for gfx950 (CDNA4).
//
// Matrix layout used by every layer (the "transposed" form): a layer computes
// H_out^T = W * H_in^T with the weights as the MFMA A operand (M = output
// neurons, 16 per tile) and the node activations as the B operand (N = 16
// node rows per tile). The 16x16 FP32 accumulator then holds, in lane
// (g = lane/16, c = lane%16), the outputs of neurons 4g..4g+3 for node row c,
// which are written back as 4 consecutive values of that row.
//
// Both operands are fed with one 16-byte load per lane per "chunk" of the
// reduction dimension. Lane group g covers k in [g*kc/4, (g+1)*kc/4) of the
// chunk, contiguous, so a B fragment is 16 contiguous bytes of a row held in
// LDS and an A fragment is 16 contiguous bytes of a pre-packed weight block:
//   FP32  chunk = 16 k: 4 x v_mfma_f32_16x16x4_f32, element j of the lane's
//                       float4 feeds instruction j
//   BF16  chunk = 32 k: 1 x v_mfma_f32_16x16x32_bf16
//   FP8   chunk = 64 k: 2 x v_mfma_f32_16x16x32_fp8_fp8, bytes 0-7 and 8-15
// Packed weights: [n_tile][chunk][lane][16 bytes], 1 KiB per (tile, chunk),
// so one wave reads a fragment with a single coalesced 1 KiB load.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cyrus_internal.h"

namespace cyrus {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Weight fragments live in device global memory. Reading them through a
// global-address-space pointer makes the compiler emit global (not flat)
// loads: flat loads also count against the LDS wait counter, so every wait
// for an LDS read would otherwise drain the weight prefetch as well.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 guint4;
__device__ __forceinline__ const guint4* as_global(const void* p)
{
    return (const guint4*)(p);
}
typedef __attribute__((address_space(1))) uint8_t gu8;
typedef __attribute__((address_space(1))) float gf32;
__device__ __forceinline__ gu8* as_global_mut(uint8_t* p) { return (gu8*)(p); }
__device__ __forceinline__ gf32* as_global_mut(float* p) { return (gf32*)(p); }
// Read-only view of device data through a global-address-space pointer.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gptr(const T* p)
{
    return (const __attribute__((address_space(1))) T*)(p);
}
__device__ __forceinline__ uint4 gld(const guint4* p)
{
    const u32x4 v = *p;
    return uint4{v[0], v[1], v[2], v[3]};
}

template <int P>
struct Traits;
template <>
struct Traits<kFP32> {
    static constexpr int kEsize = 4;
    static constexpr int kChunk = 16;
};
template <>
struct Traits<kBF16> {
    static constexpr int kEsize = 2;
    static constexpr int kChunk = 32;
};
template <>
struct Traits<kFP8> {
    static constexpr int kEsize = 1;
    static constexpr int kChunk = 64;
};

// One reduction chunk: acc += A_chunk * B_chunk.
template <int P>
__device__ __forceinline__ void mma_chunk(const uint4& a, const uint4& b, floatx4& acc);

template <>
__device__ __forceinline__ void mma_chunk<kFP32>(const uint4& a, const uint4& b, floatx4& acc)
{
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), acc, 0, 0, 0);
}

template <>
__device__ __forceinline__ void mma_chunk<kBF16>(const uint4& a, const uint4& b, floatx4& acc)
{
    bf16x8 av, bv;
    __builtin_memcpy(&av, &a, 16);
    __builtin_memcpy(&bv, &b, 16);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
}

template <>
__device__ __forceinline__ void mma_chunk<kFP8>(const uint4& a, const uint4& b, floatx4& acc)
{
    long a0 = (long)(((uint64_t)a.y << 32) | a.x), a1 = (long)(((uint64_t)a.w << 32) | a.z);
    long b0 = (long)(((uint64_t)b.y << 32) | b.x), b1 = (long)(((uint64_t)b.w << 32) | b.z);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a0, b0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a1, b1, acc, 0, 0, 0);
}

// Two consecutive chunks at once. For FP8 this is one gfx950
// v_mfma_scale_f32_16x16x128_f8f6f4 (E4M3 operands, unit E8M0 scales) at twice
// the rate of the 16x16x32 form: each lane supplies its 16 bytes of chunk c
// followed by its 16 bytes of chunk c+1, for A and B alike, so whichever
// reduction index the instruction assigns to a (lane group, byte) position, A
// and B agree on it and the 128-term dot products are the same sums.
template <int P>
__device__ __forceinline__ void mma_pair(const uint4& a0, const uint4& a1, const uint4& b0, const uint4& b1,
                                         floatx4& acc)
{
    mma_chunk<P>(a0, b0, acc);
    mma_chunk<P>(a1, b1, acc);
}

typedef int intx8 __attribute__((ext_vector_type(8)));

template <>
__device__ __forceinline__ void mma_pair<kFP8>(const uint4& a0, const uint4& a1, const uint4& b0, const uint4& b1,
                                               floatx4& acc)
{
    const intx8 a = {(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w, (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
    const intx8 b = {(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w, (int)b1.x, (int)b1.y, (int)b1.z, (int)b1.w};
    acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc, 0, 0, 0, 127, 0, 127);
}

// acc += s (A B) for two consecutive chunks, s a power of two given as its
// E8M0 code (the biased FP32 exponent). FP8 applies s through the block
// scales of v_mfma_scale_f32_16x16x128_f8f6f4 (exact: a power of two);
// FP32 and BF16 carry no scales (s = 1), so the code is ignored.
template <int P>
__device__ __forceinline__ void mma_pair_scaled(const uint4& a0, const uint4& a1, const uint4& b0, const uint4& b1,
                                                floatx4& acc, int)
{
    mma_pair<P>(a0, a1, b0, b1, acc);
}
template <>
__device__ __forceinline__ void mma_pair_scaled<kFP8>(const uint4& a0, const uint4& a1, const uint4& b0,
                                                      const uint4& b1, floatx4& acc, int e8m0)
{
    const intx8 a = {(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w, (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
    const intx8 b = {(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w, (int)b1.x, (int)b1.y, (int)b1.z, (int)b1.w};
    acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc, 0, 0, 0, e8m0, 0, 127);
}
__device__ __forceinline__ int e8m0_of(float pow2) { return (int)((__float_as_uint(pow2) >> 23) & 0xffu); }

// ---------------------------------------------------------------------------
// Gaussian policy head (Sec. IV-B). Philox4x32-10 (Salmon, Moraes, Dror and
// Shaw, SC'11), from its definition: ten rounds of two 32x32->64 products of
// counter words 0 and 2 by the round constants, recombined as
// (hi(R1 c2) ^ c1 ^ k0, lo(R1 c2), hi(R0 c0) ^ c3 ^ k1, lo(R0 c0)), the key
// bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                              uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// The log-share log b_e of UE e at tree node `node`: eps ~ N(0, 1) from Philox
// (key = seed, counter = (node, e, tti)) by Box-Muller on the first two words
// mapped to (0, 1) as (w + 1/2) 2^-32, u = mu + sigma eps with sigma =
// exp(clamp(log sigma, -20, 2)), b = (1 + tanh u) / 2, evaluated as
// -log(1 + exp(-2u)). -ln(w-uniform) is taken from whichever end of (0, 1) is
// exact in FP32: ln(u1) for u1 < 1/2, log1p(-(1 - u1)) above, where 1 - u1 is
// formed from the complemented word.
__device__ __forceinline__ float gaussian_eps(uint64_t seed, uint64_t tti, int64_t node, int e)
{
    uint32_t w0 = (uint32_t)node, w1 = (uint32_t)e, w2 = (uint32_t)tti, w3 = (uint32_t)(tti >> 32);
    philox4x32_10(w0, w1, w2, w3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const float kTwoM32 = 2.3283064365386963e-10f;  // 2^-32
    const float nlog_u1 = w0 < 0x80000000u ? -logf(((float)w0 + 0.5f) * kTwoM32)
                                           : -log1pf(-((float)(~w0) + 0.5f) * kTwoM32);
    return sqrtf(2.f * nlog_u1) * cospif(2.f * (((float)w1 + 0.5f) * kTwoM32));
}

__device__ __forceinline__ float clamp_log_sigma(float ls) { return fminf(fmaxf(ls, -20.f), 2.f); }

// The log-share for a given draw eps (the same number as gaussian_log_share
// with that node's eps).
__device__ __forceinline__ float gaussian_log_share_eps(float mu, float log_sigma, float eps)
{
    const float u = mu + expf(clamp_log_sigma(log_sigma)) * eps;
    return u >= 0.f ? -log1pf(expf(-2.f * u)) : 2.f * u - log1pf(expf(2.f * u));
}

__device__ __forceinline__ float gaussian_log_share(float mu, float log_sigma, uint64_t seed, uint64_t tti,
                                                   int64_t node, int e)
{
    return gaussian_log_share_eps(mu, log_sigma, gaussian_eps(seed, tti, node, e));
}

// Index of the calling wave in its workgroup, as a wave-uniform (scalar)
// value, so that offsets derived from it live in SGPRs.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Workgroup barrier that orders LDS only: waits for this wave's LDS operations
// (lgkmcnt = 0) and meets the other waves, but leaves global loads and stores in
// flight (vmcnt and expcnt at their maximum in the gfx9 s_waitcnt encoding).
// For code whose waves exchange data through LDS only: global results are
// write-only and global loads are waited for by the compiler before use.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_s_barrier();
}

// float -> bfloat16 bits, round to nearest even (gfx950 hardware conversion).
__device__ __forceinline__ uint32_t bf16_bits(float v)
{
    return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v);
}

// Two floats -> two BF16 (low half = v0), one gfx950 v_cvt_pk_bf16_f32.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16x2_bits(float v0, float v1)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2{v0, v1}), bf16x2));
}

// Four floats -> four OCP E4M3 bytes (hardware round to nearest even), with
// explicit saturation at +-448.
__device__ __forceinline__ uint32_t e4m3x4(float v0, float v1, float v2, float v3)
{
    // saturate to E4M3's finite range (median of three: one instruction; the
    // inputs are finite)
    v0 = __builtin_amdgcn_fmed3f(v0, -448.f, 448.f);
    v1 = __builtin_amdgcn_fmed3f(v1, -448.f, 448.f);
    v2 = __builtin_amdgcn_fmed3f(v2, -448.f, 448.f);
    v3 = __builtin_amdgcn_fmed3f(v3, -448.f, 448.f);
    int lo = __builtin_amdgcn_cvt_pk_fp8_f32(v0, v1, 0, false);
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v2, v3, lo, true);
}

// Store four consecutive activations of one row in the storage type of P.
// `inv_scale` is the reciprocal of the next layer's FP8 input scale.
template <int P>
__device__ __forceinline__ void store4(uint8_t* dst, float v0, float v1, float v2, float v3, float inv_scale);

template <>
__device__ __forceinline__ void store4<kFP32>(uint8_t* dst, float v0, float v1, float v2, float v3, float)
{
    *reinterpret_cast<floatx4*>(dst) = floatx4{v0, v1, v2, v3};
}

template <>
__device__ __forceinline__ void store4<kBF16>(uint8_t* dst, float v0, float v1, float v2, float v3, float)
{
    uint2 w;
    w.x = bf16x2_bits(v0, v1);
    w.y = bf16x2_bits(v2, v3);
    *reinterpret_cast<uint2*>(dst) = w;
}

template <>
__device__ __forceinline__ void store4<kFP8>(uint8_t* dst, float v0, float v1, float v2, float v3, float inv_scale)
{
    *reinterpret_cast<uint32_t*>(dst) = e4m3x4(v0 * inv_scale, v1 * inv_scale, v2 * inv_scale, v3 * inv_scale);
}

// Store four consecutive hidden-layer outputs v = W x + b, already in the
// next layer's input scale, as ReLU(v) in the storage type of P (FP8: also
// saturated at E4M3's largest finite value, 448).
template <int P>
__device__ __forceinline__ void store_act4(uint8_t* dst, float v0, float v1, float v2, float v3);

template <>
__device__ __forceinline__ void store_act4<kFP32>(uint8_t* dst, float v0, float v1, float v2, float v3)
{
    *reinterpret_cast<floatx4*>(dst) = floatx4{fmaxf(v0, 0.f), fmaxf(v1, 0.f), fmaxf(v2, 0.f), fmaxf(v3, 0.f)};
}

template <>
__device__ __forceinline__ void store_act4<kBF16>(uint8_t* dst, float v0, float v1, float v2, float v3)
{
    store4<kBF16>(dst, fmaxf(v0, 0.f), fmaxf(v1, 0.f), fmaxf(v2, 0.f), fmaxf(v3, 0.f), 1.f);
}

// ReLU(v), saturated at 448, as four E4M3 bytes (v0 in the low byte).
__device__ __forceinline__ uint32_t act4_e4m3(float v0, float v1, float v2, float v3)
{
    v0 = __builtin_amdgcn_fmed3f(v0, 0.f, 448.f);
    v1 = __builtin_amdgcn_fmed3f(v1, 0.f, 448.f);
    v2 = __builtin_amdgcn_fmed3f(v2, 0.f, 448.f);
    v3 = __builtin_amdgcn_fmed3f(v3, 0.f, 448.f);
    const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(v0, v1, 0, false);
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v2, v3, lo, true);
}

template <>
__device__ __forceinline__ void store_act4<kFP8>(uint8_t* dst, float v0, float v1, float v2, float v3)
{
    *reinterpret_cast<uint32_t*>(dst) = act4_e4m3(v0, v1, v2, v3);
}

// Store one activation (feature assembly, padding).
template <int P>
__device__ __forceinline__ void store1(uint8_t* dst, float v, float inv_scale);
template <>
__device__ __forceinline__ void store1<kFP32>(uint8_t* dst, float v, float)
{
    *reinterpret_cast<float*>(dst) = v;
}
template <>
__device__ __forceinline__ void store1<kBF16>(uint8_t* dst, float v, float)
{
    *reinterpret_cast<uint16_t*>(dst) = (uint16_t)bf16_bits(v);
}
template <>
__device__ __forceinline__ void store1<kFP8>(uint8_t* dst, float v, float inv_scale)
{
    v = fminf(fmaxf(v * inv_scale, -448.f), 448.f);
    *dst = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.f, 0, false) & 0xff);
}

// The value store1<P> would store for v, as a float: what an MFMA of
// precision P reads for that input.
template <int P>
__device__ __forceinline__ float stored_value(float v, float inv_scale);
template <>
__device__ __forceinline__ float stored_value<kFP32>(float v, float)
{
    return v;
}
template <>
__device__ __forceinline__ float stored_value<kBF16>(float v, float)
{
    return __uint_as_float(bf16_bits(v) << 16);
}
template <>
__device__ __forceinline__ float stored_value<kFP8>(float v, float inv_scale)
{
    v = fminf(fmaxf(v * inv_scale, -448.f), 448.f);
    return __builtin_amdgcn_cvt_f32_fp8(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.f, 0, false), 0);
}

// Element j (0 <= j < 16 / esize) of a 16-byte fragment of precision P, as a
// float (exact: every storage type widens to FP32 without rounding). j is a
// constant once the caller's loop is unrolled.
template <int P>
__device__ __forceinline__ float frag_value(const uint4& f, int j)
{
    const uint32_t w[4] = {f.x, f.y, f.z, f.w};
    if constexpr (P == kFP32)
        return __uint_as_float(w[j]);
    else if constexpr (P == kBF16)
        return __uint_as_float((j & 1) ? (w[j / 2] & 0xffff0000u) : (w[j / 2] << 16));
    else
        return __builtin_amdgcn_cvt_f32_fp8((int)(w[j / 4] >> (8 * (j % 4))), 0);
}

// ---------------------------------------------------------------------------
// Groups of 8 or 16 lanes on the DPP fabric: butterfly all-reductions with
// quad permutations (xor 1, xor 2), the half-row mirror (lane i <-> 7-i) and
// the row mirror (lane i <-> 15-i). Every lane of the group ends with the same
// value (each step adds two partial sums in either order).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror
constexpr int kDppMirror = 0x140;      // row_mirror

// ---------------------------------------------------------------------------
// Lane-parallel enforcer: a group of G lanes (G a power of two >= E, G <= 64)
// handles one node, lane e of the group UE e. Softmax, the capped split and
// largest remainder use butterfly reductions inside the group; the extra unit
// goes to UE e if it is eligible and fewer than r eligible UEs rank above it
// (larger fraction, or equal fraction and lower index). Every lane of the group
// must call this with the same row. Returns a_e (0 for lanes e >= E).
template <int G>
__device__ __forceinline__ float group_sum(float v)
{
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1)
        v += __shfl_xor(v, m, G);
    return v;
}

// The exact group reductions (integer sums, minima, maxima) of 8- and
// 16-lane groups run on the DPP fabric, wider groups through lane shuffles.
template <int G>
__device__ __forceinline__ float group_max(float v)
{
    if constexpr (G == 8 || G == 16) {
        v = fmaxf(v, dpp_f<kDppXor1>(v));
        v = fmaxf(v, dpp_f<kDppXor2>(v));
        v = fmaxf(v, dpp_f<kDppHalfMirror>(v));
        if constexpr (G == 16)
            v = fmaxf(v, dpp_f<kDppMirror>(v));
        return v;
    }
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1)
        v = fmaxf(v, __shfl_xor(v, m, G));
    return v;
}

template <int G>
__device__ __forceinline__ int group_isum(int v)
{
    if constexpr (G == 8 || G == 16) {
        v += dpp_i<kDppXor1>(v);
        v += dpp_i<kDppXor2>(v);
        v += dpp_i<kDppHalfMirror>(v);
        if constexpr (G == 16)
            v += dpp_i<kDppMirror>(v);
        return v;
    }
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1)
        v += __shfl_xor(v, m, G);
    return v;
}

template <int G>
__device__ __forceinline__ float group_min(float v)
{
    if constexpr (G == 8 || G == 16) {
        v = fminf(v, dpp_f<kDppXor1>(v));
        v = fminf(v, dpp_f<kDppXor2>(v));
        v = fminf(v, dpp_f<kDppHalfMirror>(v));
        if constexpr (G == 16)
            v = fminf(v, dpp_f<kDppMirror>(v));
        return v;
    }
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1)
        v = fminf(v, __shfl_xor(v, m, G));
    return v;
}

template <int G>
__device__ __forceinline__ int group_imax(int v)
{
    if constexpr (G == 8 || G == 16) {
        v = max(v, dpp_i<kDppXor1>(v));
        v = max(v, dpp_i<kDppXor2>(v));
        v = max(v, dpp_i<kDppHalfMirror>(v));
        if constexpr (G == 16)
            v = max(v, dpp_i<kDppMirror>(v));
        return v;
    }
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1)
        v = max(v, __shfl_xor(v, m, G));
    return v;
}

template <int G>
__device__ __forceinline__ int group_imin(int v)
{
    if constexpr (G == 8 || G == 16) {
        v = min(v, dpp_i<kDppXor1>(v));
        v = min(v, dpp_i<kDppXor2>(v));
        v = min(v, dpp_i<kDppHalfMirror>(v));
        if constexpr (G == 16)
            v = min(v, dpp_i<kDppMirror>(v));
        return v;
    }
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1)
        v = min(v, __shfl_xor(v, m, G));
    return v;
}

// Huntington-Hill integer step (Sec. IV-B, after Balinski and Young) for the
// shares x of one node, lane e of a G-lane group holding UE e. A unit's
// priority is x_e / sqrt(n (n+1)) for the n units UE e already holds (the
// first unit: infinite); the allocation is the T units of highest priority
// within the caps, equal priorities going to the larger share and then the
// lower index, and a UE with no share receiving nothing. Computed from the
// rounding at divisor 1 (every unit of priority >= 1), then the units of
// highest priority are added one by one, or those of lowest priority removed
// (the reverse order: smaller share, then higher index), until the sum is T.
// Below one unit per positive share this gives one unit to each of the T
// largest shares. The loops are uniform over the group.
template <int G>
__device__ __forceinline__ int hh_round(int e, bool live, float x, int R, int T)
{
    const float kInf = __builtin_huge_valf();
    const bool pos = live && R > 0 && x > 0.f;
    int a = 0;
    if (pos) {
        const float f = floorf(x);
        a = min((int)f + (x >= sqrtf(f * (f + 1.f)) ? 1 : 0), R);
    }
    int S = group_isum<G>(a);
    while (S < T) {
        const bool cand = pos && a < R;
        const float pr = cand ? (a == 0 ? kInf : x / sqrtf((float)a * (float)(a + 1))) : -1.f;
        const float top = group_max<G>(pr);
        const bool at = cand && pr == top;
        const float xm = group_max<G>(at ? x : -1.f);
        const int w = group_imin<G>(at && x == xm ? e : G);
        a += e == w ? 1 : 0;
        ++S;
    }
    while (S > T) {
        const bool cand = pos && a > 0;
        const float pr = cand ? (a == 1 ? kInf : x / sqrtf((float)(a - 1) * (float)a)) : kInf;
        const float low = group_min<G>(pr);
        const bool at = cand && pr == low;
        const float xm = group_min<G>(at ? x : kInf);
        const int w = group_imax<G>(at && x == xm ? e : -1);
        a -= e == w ? 1 : 0;
        --S;
    }
    return a;
}

template <int G>
__device__ __forceinline__ int enforce_group(int E, int e, float z, int R, int rsum, int demand, int rounding)
{
    const bool live = e < E;
    const float zmax = group_max<G>(live ? z : -3.0e38f);
    float p = live ? expf(fmaxf(z - zmax, -80.f)) : 0.f;
    const float sum = group_sum<G>(p);
    p = p / sum;
    const int T = demand < rsum ? demand : rsum;
    if (T >= rsum)
        return live ? R : 0;
    bool capped = !live;
    float s = 0.f;
    for (int pass = 0; pass <= G; ++pass) {
        // pass 0 caps only the padding lanes, which add no R: rem is T
        const float rem = pass == 0 ? (float)T : (float)T - group_sum<G>((live && capped) ? (float)R : 0.f);
        const float psum = group_sum<G>(capped ? 0.f : p);
        s = rem / psum;
        const bool grow = !capped && s * p >= (float)R;
        // the loop ends when no lane of the wave grows: a group that has
        // settled repeats its last pass with the same result
        if (__ballot(grow) == 0)
            break;
        capped = capped || grow;
    }
    const float x = !live ? 0.f : (capped ? (float)R : s * p);
    if (rounding == kHuntingtonHill)
        return hh_round<G>(e, live, x, R, T);
    const float fl = floorf(x);
    const int f = (int)fl;
    const float frac = x - fl;
    const int r = T - group_isum<G>(f);
    const bool elig = live && f < R;
    // ineligible UEs carry -1 and never rank above an eligible one; q = e
    // counts for neither test, so the count needs no branch
    const float mine = elig ? frac : -1.f;
    float fq[G];
#pragma unroll
    for (int q = 0; q < G; ++q)
        fq[q] = __shfl(mine, q, G);
    int rank = 0;
#pragma unroll
    for (int q = 0; q < G; ++q)
        rank += (fq[q] > frac || (fq[q] == frac && q < e)) ? 1 : 0;
    return f + ((elig && rank < r) ? 1 : 0);
}

template <int G>
__device__ __forceinline__ float dsum(float v)
{
    static_assert(G == 8 || G == 16, "DPP groups are 8 or 16 lanes");
    v += dpp_f<kDppXor1>(v);
    v += dpp_f<kDppXor2>(v);
    v += dpp_f<kDppHalfMirror>(v);
    if constexpr (G == 16)
        v += dpp_f<kDppMirror>(v);
    return v;
}
template <int G>
__device__ __forceinline__ float dmax(float v)
{
    v = fmaxf(v, dpp_f<kDppXor1>(v));
    v = fmaxf(v, dpp_f<kDppXor2>(v));
    v = fmaxf(v, dpp_f<kDppHalfMirror>(v));
    if constexpr (G == 16)
        v = fmaxf(v, dpp_f<kDppMirror>(v));
    return v;
}
template <int G>
__device__ __forceinline__ int disum(int v)
{
    v += dpp_i<kDppXor1>(v);
    v += dpp_i<kDppXor2>(v);
    v += dpp_i<kDppHalfMirror>(v);
    if constexpr (G == 16)
        v += dpp_i<kDppMirror>(v);
    return v;
}

// Sum over the four 16-lane rows of a wave, column by column: lane i ends
// with (v[c] + v[c + 16]) + (v[c + 32] + v[c + 48]), c = i % 16, the same value
// in all four rows. gfx950's row swaps (v_permlane16_swap, v_permlane32_swap)
// exchange rows on the vector ALU, without a round trip through LDS: a
// 16-swap of v with itself leaves rows (0, 1) and (2, 3) with each other's
// values in its two results, a 32-swap likewise rows (0, 1) and (2, 3).
__device__ __forceinline__ float row_sum4(float v)
{
    const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    const float s = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(s), __float_as_uint(s), false, false);
    return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}

// Same enforcer as enforce_group for groups of 8 or 16 lanes aligned to
// 8/16-lane boundaries, with DPP reductions; the remainder ranks go through
// `rank_row` (G floats of LDS private to this group).
template <int G>
__device__ __forceinline__ int enforce_dpp(int E, int e, float z, int R, int rsum, int demand, float* rank_row,
                                           int rounding)
{
    const bool live = e < E;
    const int T = demand < rsum ? demand : rsum;
    if (T >= rsum)
        return live ? R : 0;
    // the split only needs the softmax up to its normalisation: with
    // w_e = exp(z_e - max z), x_e = min(R_e, s' w_e) where s' absorbs 1/sum w
    const float zmax = dmax<G>(live ? z : -3.0e38f);
    const float p = live ? expf(fmaxf(z - zmax, -80.f)) : 0.f;
    bool capped = !live;
    float s = 0.f;
    for (int pass = 0; pass <= G; ++pass) {
        // pass 0 caps only the padding lanes, which add no R: rem is T
        const float rem = pass == 0 ? (float)T : (float)T - dsum<G>((live && capped) ? (float)R : 0.f);
        const float psum = dsum<G>(capped ? 0.f : p);
        s = rem / psum;
        const bool grow = !capped && s * p >= (float)R;
        // the loop ends when no lane of the wave grows: a group that has
        // settled repeats its last pass with the same result
        if (__ballot(grow) == 0)
            break;
        capped = capped || grow;
    }
    const float x = !live ? 0.f : (capped ? (float)R : s * p);
    if (rounding == kHuntingtonHill)
        return hh_round<G>(e, live, x, R, T);
    const float fl = floorf(x);
    const int f = (int)fl;
    const float frac = x - fl;
    const int r = T - disum<G>(f);
    const bool elig = live && f < R;
    rank_row[e] = elig ? frac : -1.f;  // ineligible UEs never rank above an eligible one
    // rank = UEs ahead of e (larger remainder, or equal with a lower index);
    // q = e counts for neither, so the count needs no branch, and every read
    // is issued before the first comparison
    float fq[G];
#pragma unroll
    for (int q = 0; q < G; ++q)
        fq[q] = rank_row[q];
    int rank = 0;
#pragma unroll
    for (int q = 0; q < G; ++q)
        rank += (fq[q] > frac || (fq[q] == frac && q < e)) ? 1 : 0;
    return f + ((elig && rank < r) ? 1 : 0);
}

// enforce_dpp for N rows at once per G-lane group (row j: logit z[j],
// demand[j], ranks through rank_row[j], which is touched only for a live row
// that needs a split; rows with live_row[j] false give 0).
// Each row's arithmetic is enforce_dpp's, in the same order, so the
// allocations are the same; the N independent reduction chains interleave, so
// one pass over N rows takes little more than a pass over one. The capping
// loop runs until no row of the wave grows: a settled row repeats its last
// pass with the same result, as a settled group does in enforce_dpp.
template <int G, int N>
__device__ __forceinline__ void enforce_dpp_n(int E, int e, const float (&z)[N], int R, int rsum,
                                              const int (&demand)[N], const bool (&live_row)[N],
                                              float* const (&rank_row)[N], int rounding, int (&a)[N])
{
    const bool live = e < E;
    int T[N];
    bool done[N], capped[N];
    float p[N], s[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        T[j] = demand[j] < rsum ? demand[j] : rsum;
        done[j] = !live_row[j] || T[j] >= rsum;  // no split to compute
        const float zmax = dmax<G>(live ? z[j] : -3.0e38f);
        p[j] = live ? expf(fmaxf(z[j] - zmax, -80.f)) : 0.f;
        capped[j] = !live;
        s[j] = 0.f;
    }
    for (int pass = 0; pass <= G; ++pass) {
        bool grow[N], any = false;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const float rem = pass == 0 ? (float)T[j] : (float)T[j] - dsum<G>((live && capped[j]) ? (float)R : 0.f);
            const float psum = dsum<G>(capped[j] ? 0.f : p[j]);
            s[j] = rem / psum;
            grow[j] = !done[j] && !capped[j] && s[j] * p[j] >= (float)R;
            any = any || grow[j];
        }
        if (__ballot(any) == 0)
            break;
#pragma unroll
        for (int j = 0; j < N; ++j)
            capped[j] = capped[j] || grow[j];
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const float x = !live ? 0.f : (capped[j] ? (float)R : s[j] * p[j]);
        a[j] = (live_row[j] && live) ? R : 0;  // the rows without a split
        if (done[j])
            continue;  // uniform over the group (its lanes share the row)
        if (rounding == kHuntingtonHill) {
            a[j] = hh_round<G>(e, live, x, R, T[j]);
        } else {
            const float fl = floorf(x);
            const int f = (int)fl;
            const float frac = x - fl;
            const int r = T[j] - disum<G>(f);
            const bool elig = live && f < R;
            rank_row[j][e] = elig ? frac : -1.f;
            float fq[G];
#pragma unroll
            for (int q = 0; q < G; ++q)
                fq[q] = rank_row[j][q];
            int rank = 0;
#pragma unroll
            for (int q = 0; q < G; ++q)
                rank += (fq[q] > frac || (fq[q] == frac && q < e)) ? 1 : 0;
            a[j] = f + ((elig && rank < r) ? 1 : 0);
        }
    }
}

}  // namespace cyrus
