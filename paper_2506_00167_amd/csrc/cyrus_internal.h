// Internal types shared by the host library and the kernels.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace cyrus {

constexpr int kWaves = 8;                 // waves per workgroup
constexpr int kThreads = kWaves * 64;     // threads per workgroup
constexpr int kXcds = 8;                  // accelerator complex dies, each with its own L2
constexpr int kMaxLayers = 5;
constexpr int kMaxUE = 32;
constexpr int kLogitStride = kMaxUE + 1;  // LDS row stride of the logits (bank-conflict free)
constexpr int kMaxEntries = 128;          // (codebook, level) entries per batched level launch

enum Prec { kFP32 = 0, kBF16 = 1, kFP8 = 2 };
enum Rounding { kLargestRemainder = 0, kHuntingtonHill = 1 };  // integer step of the enforcer
enum Head { kSoftmaxHead = 0, kGaussianHead = 1 };              // policy head: E logits, or 2E (mu, log sigma)

inline constexpr int prec_esize(int p) { return p == kFP32 ? 4 : (p == kBF16 ? 2 : 1); }
inline constexpr int prec_chunk(int p) { return p == kFP32 ? 16 : (p == kBF16 ? 32 : 64); }

// Everything a kernel needs to build one codebook; passed by value or read
// from a device array in batched launches.
struct DevTree {
    int32_t E, K, M, U;
    int32_t rounding;                 // Rounding
    int32_t n_layers;                 // hidden layers + output layer
    int32_t in_dim0;                  // 4E + 2
    int32_t in_pad[kMaxLayers];       // layer input width padded to the k-chunk
    int32_t out_pad[kMaxLayers];      // layer output width padded to 16
    const uint8_t* w[kMaxLayers];     // packed weight fragments
    // Layer 1 split by input: the first 3E inputs (R, MCS, SINR) are the same
    // for every node of a tree, the last E + 2 (c, tau, k) are the node's own.
    // w1d holds the fragments of the per-node columns only, in_pad_d wide.
    int32_t in_pad_d;
    const uint8_t* w1d;
    const float* b[kMaxLayers];       // biases, out_pad entries (zero padded)
    float deq[kMaxLayers];            // FP8: weight scale * input scale; else 1
    float inv_in_scale[kMaxLayers];   // FP8: 1 / input scale of layer l; else 1
    const int32_t* ue;                // rb[E], mcs[E], sinr_db[E] (float bits)
    uint8_t* alloc;                   // [nodes][E]
    uint8_t* state;                   // [nodes][E] punctured RBs so far, after the node
    float* logits;                    // [nodes][E] or null
    int32_t head;                     // Head
    uint64_t seed, tti;               // Gaussian head: Philox key and TTI
};

inline int64_t ipow(int64_t b, int e)
{
    int64_t r = 1;
    for (int i = 0; i < e; ++i)
        r *= b;
    return r;
}

}  // namespace cyrus
