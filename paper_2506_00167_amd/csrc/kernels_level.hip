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

#include <hip/hip_ext.h>

#include "cyrus_device.h"
#include "cyrus_kernels.h"
#include "cyrus_mlp.h"
#include "cyrus_subtree.h"

namespace cyrus {

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
// Stores of the resident worker (COH): node states and codebook bytes with
// agent-scope relaxed atomic stores, which write through the non-coherent
// caches, so other workgroups (on any XCD) and the copy engine that later
// moves the codebook to the host read them without a cache flush.
template <bool COH>
__device__ __forceinline__ void put_state(gu8* p, uint8_t v)
{
    if constexpr (COH)
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}
template <bool COH>
__device__ __forceinline__ void put_alloc(gu8* p, uint8_t v)
{
    put_state<COH>(p, v);
}

// The enforcer and the stores of rows [0, nrows) of a tile. With G lanes per
// row, kThreads / G rows make one pass; N passes' rows run together in one
// call of enforce_dpp_n (G <= 16), so a tile of up to N passes of rows takes
// one interleaved pass.
template <int G, int N, bool COH>
__device__ __forceinline__ void finish_rows_level_n(const DevTree& t, const float* zl, const int* R, int rsum, int row0,
                                                    int nrows, int64_t off, const uint8_t* pst, int p_lo)
{
    // Every field of t is read once, before the first store: the output
    // pointers could alias the tree descriptor in global memory, so a field
    // read after a store would be fetched again from memory.
    const int E = t.E, K = t.K, U = t.U, rounding = t.rounding;
    gu8* const alloc = as_global_mut(t.alloc);
    gu8* const state = as_global_mut(t.state);
    gf32* const logits = as_global_mut(t.logits);
    const bool with_logits = t.logits != nullptr;
    constexpr int GR = kThreads / G;  // rows of one pass
    const int e = (int)threadIdx.x % G;
    const int Re = e < E ? R[e] : 0;
    for (int base = 0; base < nrows; base += GR * N) {
        int row[N], a[N], k[N], pq[N], demand[N];
        bool live_row[N];
        float z[N];
        float* zrow[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            row[j] = base + j * GR + (int)threadIdx.x / G;
            live_row[j] = row[j] < nrows;
            const int r = row0 + row[j];
            pq[j] = r / K;
            k[j] = r - pq[j] * K + 1;
            demand[j] = U * k[j];
            zrow[j] = const_cast<float*>(zl) + (live_row[j] ? row[j] : 0) * kLogitStride;
            z[j] = (live_row[j] && e < E) ? zrow[j][e] : 0.f;
        }
        if constexpr (G <= 16) {
            enforce_dpp_n<G, N>(E, e, z, Re, rsum, demand, live_row, zrow, rounding, a);  // rows reused for ranks
        } else {
            static_assert(N == 1, "groups wider than 16 lanes take one row per call");
            a[0] = live_row[0] ? enforce_group<G>(E, e, z[0], Re, rsum, demand[0], rounding) : 0;
        }
#pragma unroll
        for (int j = 0; j < N; ++j) {
            if (live_row[j] && e < E) {
                const int p = pq[j];
                const int64_t node = off + (int64_t)p * (K + 1) + k[j];
                const uint8_t c = pst[(p - p_lo) * E + e];
                put_alloc<COH>(alloc + node * E + e, (uint8_t)a[j]);
                put_state<COH>(state + node * E + e, (uint8_t)(c + a[j]));
                if (with_logits)
                    logits[node * E + e] = z[j];
                if (k[j] == 1) {
                    const int64_t sib = off + (int64_t)p * (K + 1);
                    put_alloc<COH>(alloc + sib * E + e, 0);
                    put_state<COH>(state + sib * E + e, c);
                    if (with_logits)
                        logits[sib * E + e] = 0.f;
                }
            }
        }
    }
}

template <int G, int RTT, bool COH = false>
__device__ __forceinline__ void finish_rows_level(const DevTree& t, const float* zl, const int* R, int rsum, int row0,
                                                  int nrows, int64_t off, const uint8_t* pst, int p_lo)
{
    constexpr int GR = kThreads / G;
    constexpr int kPasses = (16 * RTT + GR - 1) / GR;  // passes of a full tile
    if constexpr (G > 16 || kPasses == 1) {
        finish_rows_level_n<G, 1, COH>(t, zl, R, rsum, row0, nrows, off, pst, p_lo);
    } else {
        // at most three rows per group; in the serving worker, whose tile
        // body also holds its claim state, two, and one in 96-row tiles
        // (registers: the BF16 instantiation would spill)
        constexpr int kMaxN = COH ? (RTT >= 6 ? 1 : 2) : 3;
        constexpr int NM = kPasses < kMaxN ? kPasses : kMaxN;
        if (nrows <= GR)
            finish_rows_level_n<G, 1, COH>(t, zl, R, rsum, row0, nrows, off, pst, p_lo);
        else
            finish_rows_level_n<G, NM, COH>(t, zl, R, rsum, row0, nrows, off, pst, p_lo);
    }
}

// LDS of a level workgroup: two activation buffers of `bufsize` bytes, the
// FP32 logits of the tile, the UE radio state, the parent states of the
// tile's rows, the row-independent feature template, the entry tables of a
// batched launch and, last (its size depends on the tree), the biases of
// every layer.
constexpr int kMaxIn0 = 256;  // widest padded first-layer input (E = 32, FP8 chunk pairs)

__host__ __device__ constexpr int pst_bytes(int rtt) { return ((16 * rtt + 2) * kMaxUE + 15) & ~15; }
__host__ __device__ constexpr int tab_bytes() { return (3 * (kMaxEntries + 1) * 4 + 15) & ~15; }

struct LevelSmem {
    uint8_t* bufA;
    uint8_t* bufB;
    float* zl;      // [RT][kLogitStride]
    int* R;         // [kMaxUE]
    int* rsum;      // [4]
    float* tmpl;    // [kMaxIn0] features common to every row (UE radio state, tau), zero elsewhere
    uint8_t* tmplq; // [kMaxIn0 * 4] the same row in the storage type of the first layer's input
    uint8_t* pst;   // [(RT + 2) * kMaxUE] states of the parents of the tile's rows
    int* tab;       // [3 * (kMaxEntries + 1)] ent_tree, ent_tau, prefix
    float* bias;    // [sum of out_pad] biases of all layers
};

template <int RTT>
__device__ __forceinline__ LevelSmem level_smem(uint8_t* smem, int bufsize)
{
    LevelSmem m;
    m.bufA = smem;
    m.bufB = smem + bufsize;
    m.zl = reinterpret_cast<float*>(smem + 2 * bufsize);
    m.R = reinterpret_cast<int*>(m.zl + 16 * RTT * kLogitStride);
    m.rsum = m.R + kMaxUE;
    m.tmpl = reinterpret_cast<float*>(m.rsum + 4);
    m.tmplq = reinterpret_cast<uint8_t*>(m.tmpl + kMaxIn0);
    m.pst = m.tmplq + kMaxIn0 * 4;
    m.tab = reinterpret_cast<int*>(m.pst + pst_bytes(RTT));
    m.bias = reinterpret_cast<float*>(reinterpret_cast<uint8_t*>(m.tab) + tab_bytes());
    return m;
}

// One tile of evaluated rows [row0, row0 + nrows) of level tau. COH (the
// resident worker): the parent states and the UE state, which other
// workgroups of the same launch wrote, are read with agent-scope relaxed
// atomic loads (coherent across XCDs), and the stores are the coherent ones.
template <int P, int RTT, bool COH = false>
__device__ __forceinline__ void level_tile(const DevTree& t, int tau, int row0, int nrows, const LevelSmem& m)
{
    constexpr int es = Traits<P>::kEsize, F = 16 / es;  // features per 16-byte LDS segment
    constexpr int kPstIters = (pst_bytes(RTT) + kThreads - 1) / kThreads;
    constexpr int kBiasBatch = 4;  // float4 bias loads in flight per thread
    const int E = t.E, K = t.K, nl = t.n_layers;
    const int in0 = t.in_pad[0];
    const int64_t off = dev_level_offset(K, tau), poff = dev_level_offset(K, tau - 1);

    // Stage the tile's inputs in LDS, every global load issued before the
    // first LDS store: the states of the parents of rows row0..row0+nrows-1
    // (one contiguous range of the parent level), the UE radio state (as the
    // feature template and R), and the biases of all layers.
    const int p_lo = row0 / K;
    const int npb = ((row0 + nrows - 1) / K - p_lo + 1) * E;
    const auto* sp = gptr(t.state + (poff + p_lo) * E);
    uint8_t pv[kPstIters];
#pragma unroll
    for (int j = 0; j < kPstIters; ++j) {
        const int i = (int)threadIdx.x + j * kThreads;
        if constexpr (COH)
            pv[j] = i < npb ? __hip_atomic_load(t.state + (poff + p_lo) * E + i, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT)
                            : (uint8_t)0;
        else
            pv[j] = i < npb ? sp[i] : (uint8_t)0;
    }
    const int f = threadIdx.x;  // feature index of the template
    int uev = 0;
    if (f < 3 * E) {
        if constexpr (COH)
            uev = __hip_atomic_load(t.ue + f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            uev = gptr(t.ue)[f];
    }
    int nb4 = 0;
    for (int l = 0; l < nl; ++l)
        nb4 += t.out_pad[l] >> 2;
    for (int i0 = 0; i0 < nb4; i0 += kBiasBatch * kThreads) {
        floatx4 bv[kBiasBatch];
#pragma unroll
        for (int j = 0; j < kBiasBatch; ++j) {
            const int i = i0 + j * kThreads + (int)threadIdx.x;
            if (i < nb4) {
                int l = 0, st = 0;
                while (l + 1 < nl && i >= st + (t.out_pad[l] >> 2)) {
                    st += t.out_pad[l] >> 2;
                    ++l;
                }
                bv[j] = gptr(reinterpret_cast<const floatx4*>(t.b[l]))[i - st];
                if (l + 1 < nl) {  // hidden layer: in the next layer's input scale (a power of two)
                    const float sc = t.inv_in_scale[l + 1];
                    bv[j] = floatx4{bv[j][0] * sc, bv[j][1] * sc, bv[j][2] * sc, bv[j][3] * sc};
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kBiasBatch; ++j) {
            const int i = i0 + j * kThreads + (int)threadIdx.x;
            if (i < nb4)
                reinterpret_cast<floatx4*>(m.bias)[i] = bv[j];
        }
    }
    if (f < in0) {
        float v = 0.f;
        if (f < 2 * E)
            v = (float)uev * (1.f / 32.f);
        else if (f < 3 * E)
            v = __int_as_float(uev) * (1.f / 32.f);
        else if (f == 4 * E)
            v = (float)tau * (1.f / 8.f);
        m.tmpl[f] = v;  // parent state and k are filled in per row
        store1<P>(m.tmplq + f * es, v, t.inv_in_scale[0]);
    }
    if (threadIdx.x < 64) {  // wave 0 holds R (f < E <= 32): sum by shuffles
        int r = f < E ? uev : 0;
        if (f < E)
            m.R[f] = r;
#pragma unroll
        for (int o = 16; o > 0; o >>= 1)
            r += __shfl_xor(r, o, 32);
        if (f == 0)
            *m.rsum = r;
    }
#pragma unroll
    for (int j = 0; j < kPstIters; ++j) {
        const int i = (int)threadIdx.x + j * kThreads;
        if (i < npb)
            m.pst[i] = pv[j];
    }
    lds_barrier();

    // Features of every row, zero padded to the k-chunk and to whole row
    // tiles, one 16-byte segment (F features) per step: the template, with
    // the parent state (features 3E..4E-1) and k/8 (feature 4E+1) of the row.
    // Segments without row-dependent features are copied from the template
    // already in the storage type. Row and parent come from small quotients
    // taken in float, exact here (numerators below 2^12, distance to the
    // next integer at least 1/(2 divisor)).
    const int s0 = in0 * es + 16;
    const int nseg = in0 / F;
    const int nrows_pad = ((nrows + 15) >> 4) << 4;
    const float inv0 = t.inv_in_scale[0], inv_nseg = 1.f / (float)nseg, invK = 1.f / (float)K;
    const int rk0 = row0 - p_lo * K;  // row0's position among the children of parent p_lo
    const int d0 = 3 * E, d1 = 4 * E + 2;  // row-dependent features [d0, d1)
    // segments sg0..sg0+nsg-1 hold row-dependent features; the others are
    // copied from the template (or zeroed on the padding rows) in a first
    // pass, the row-dependent ones written in a second, so that neither
    // pass diverges inside a wave (the two write disjoint segments)
    const int sg0 = d0 / F, nsg = (d1 - 1) / F - sg0 + 1;
    const float inv_nsg = 1.f / (float)nsg;
    for (int idx = threadIdx.x; idx < nrows_pad * nseg; idx += kThreads) {
        const int row = (int)(((float)idx + 0.5f) * inv_nseg), sg = idx - row * nseg, f0 = sg * F;
        uint8_t* dst = m.bufA + row * s0 + f0 * es;
        if (row >= nrows)
            *reinterpret_cast<uint4*>(dst) = uint4{0, 0, 0, 0};
        else if (sg < sg0 || sg >= sg0 + nsg)
            *reinterpret_cast<uint4*>(dst) = *reinterpret_cast<const uint4*>(m.tmplq + f0 * es);
    }
    for (int idx = threadIdx.x; idx < nrows * nsg; idx += kThreads) {
        const int row = (int)(((float)idx + 0.5f) * inv_nsg), f0 = (sg0 + idx - row * nsg) * F;
        uint8_t* dst = m.bufA + row * s0 + f0 * es;
        {
            const int pq = (int)(((float)(rk0 + row) + 0.5f) * invK);  // parent - p_lo
            const int k = rk0 + row - pq * K + 1;
            const uint8_t* ps = m.pst + pq * E;
            const float kf = (float)k * (1.f / 8.f);
            float v[F];
#pragma unroll
            for (int j = 0; j < F; j += 4) {
                const floatx4 q = *reinterpret_cast<const floatx4*>(m.tmpl + f0 + j);
                v[j] = q[0];
                v[j + 1] = q[1];
                v[j + 2] = q[2];
                v[j + 3] = q[3];
            }
#pragma unroll
            for (int j = 0; j < F; ++j) {
                const int fj = f0 + j;
                const float sv = (float)ps[min(max(fj - d0, 0), E - 1)] * (1.f / 64.f);
                v[j] = (fj >= d0 && fj < 4 * E) ? sv : (fj == 4 * E + 1 ? kf : v[j]);
            }
#pragma unroll
            for (int j = 0; j < F; j += 4)
                store4<P>(dst + j * es, v[j], v[j + 1], v[j + 2], v[j + 3], inv0);
        }
    }
    lds_barrier();
    run_mlp<P, RTT>(t, nrows, m.bufA, m.bufB, m.zl, m.bias, off, row0);

    const int rsum = *m.rsum;
    if (E <= 8)
        finish_rows_level<8, RTT, COH>(t, m.zl, m.R, rsum, row0, nrows, off, m.pst, p_lo);
    else if (E <= 16)
        finish_rows_level<16, RTT, COH>(t, m.zl, m.R, rsum, row0, nrows, off, m.pst, p_lo);
    else
        finish_rows_level<32, RTT, COH>(t, m.zl, m.R, rsum, row0, nrows, off, m.pst, p_lo);
}

template <int P, int RTT>
__global__ __launch_bounds__(kThreads) void level_kernel(DevTree t, int tau, int n_eval, int bufsize)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const int row0 = blockIdx.x * 16 * RTT;
    const int nrows = min(16 * RTT, n_eval - row0);
    if (nrows <= 0)
        return;
    level_tile<P, RTT>(t, tau, row0, nrows, level_smem<RTT>(smem, bufsize));
}

// Batched level launch over several codebooks (cells), each at its own level:
// entry j of the launch is codebook ent_tree[j] at level ent_tau[j] and owns
// row tiles [prefix[j], prefix[j+1]) of the prefix[n] tiles of the launch.
// Persistent: a grid of at most one workgroup per CU strides over the tiles;
// the entry tables are copied to LDS once and searched there.
template <int P, int RTT>
__global__ __launch_bounds__(kThreads) void level_kernel_batch(const DevTree* __restrict__ trees,
                                                               const int* __restrict__ ent_tree,
                                                               const int* __restrict__ ent_tau,
                                                               const int* __restrict__ prefix, int n, int bufsize)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const LevelSmem m = level_smem<RTT>(smem, bufsize);
    int* s_tree = m.tab;
    int* s_tau = m.tab + kMaxEntries;
    int* s_prefix = m.tab + 2 * kMaxEntries;
    for (int i = threadIdx.x; i <= n; i += kThreads) {
        s_prefix[i] = prefix[i];
        if (i < n) {
            s_tree[i] = ent_tree[i];
            s_tau[i] = ent_tau[i];
        }
    }
    lds_barrier();
    // XCD-aware tile order. Workgroups are dispatched to the eight XCDs in
    // turn, so workgroup w runs on XCD w % 8; each XCD takes a contiguous
    // eighth of the launch's tiles, and since a cell's tiles are contiguous,
    // its L2 holds the weights of about an eighth of the cells rather than
    // streaming all of them.
    const int total = s_prefix[n];
    int b0 = blockIdx.x, bstep = gridDim.x, bend = total;
    if (gridDim.x % kXcds == 0) {
        const int x = blockIdx.x % kXcds;
        b0 = (int)((int64_t)total * x / kXcds) + blockIdx.x / kXcds;
        bstep = gridDim.x / kXcds;
        bend = (int)((int64_t)total * (x + 1) / kXcds);
    }
    for (int b = b0; b < bend; b += bstep) {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_prefix[mid] <= b)
                lo = mid;
            else
                hi = mid - 1;
        }
        const DevTree& t = trees[s_tree[lo]];
        const int tau = s_tau[lo];
        const int n_eval = (int)(t.K * (dev_level_offset(t.K, tau) - dev_level_offset(t.K, tau - 1)));
        const int row0 = (b - s_prefix[lo]) * 16 * RTT;
        const int nrows = min(16 * RTT, n_eval - row0);
        if (nrows > 0)
            level_tile<P, RTT>(t, tau, row0, nrows, m);
        lds_barrier();  // LDS is reused by the next tile
    }
}

// ----------------------------------------------------------------- serving
// Resident serving worker. Workgroup 0 is the control workgroup: it polls the
// ring in pinned host memory, copies each new request into the device slot
// table, clears the root state and opens level 1 of the request. Every other
// workgroup loops: claim one row tile of the oldest admitted request whose
// current level still has unclaimed tiles (one compare-and-swap on that
// slot's claim word, which also names the level, so a stale claim of a
// finished level cannot succeed), run it with the level kernel's tile body,
// count it done; the workgroup that completes a level's last tile opens the
// next level, or after level M flags the request finished in pinned memory.
// No workgroup ever waits for another: a level's work appears only once the
// previous level is complete.
//
// Coherence without cache flushes: every value one workgroup hands to another
// (slot records, counters, node states, UE state) or to the host (codebook
// bytes, flags) is written and read with relaxed atomic accesses of agent
// (device) or system scope, which bypass the non-coherent caches, and each
// workgroup waits for its stores to complete before the counter update that
// publishes them. An acquire fence would invalidate the whole L2 of the XCD
// and evict the actors' weights, which every tile reads through the caches; it
// is taken only when the host reports a weight refresh (wepoch).
//
// Idle tile workgroups poll one counter (opened), which the control workgroup
// bumps after admitting a request and a workgroup that opens a level of
// several tiles bumps after publishing it; they scan the claim words only
// when it has changed since their last fruitless scan, or right after a tile.
// (Scanning every slot on every poll, each a load past the per-XCD caches,
// kept the fabric busy enough to slow the loads of the workgroups at work.)
//
// Exits: the control workgroup leaves on the host's stop flag, which only it
// reads, when every record of the launch is used, after idle_ticks of
// wall-clock time with no request in flight and none in the ring, or after
// stall_ticks with requests in flight and none finishing, and then sets quit;
// the tile workgroups leave once quit is set and every admitted request has
// finished (they run the later levels of those requests at full width), or
// after stall_ticks without a tile.

__device__ __forceinline__ uint32_t sys_load_u32(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void sys_store_u32(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <class T>
__device__ __forceinline__ T dev_load(const T* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void dev_store(T* p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


// Control workgroup: admission from the ring.
__device__ void serve_control(const ServeArgs& a, int* sh)
{
    const int tid = threadIdx.x;
    uint32_t head = a.head0;
    int last_active = -1;
    uint64_t since = wall_clock64();  // start of the current idle or stalled stretch
    for (;;) {
        if (tid == 0) {
            sh[0] = (int)sys_load_u32(&a.host->stop);
            sh[1] = (int)sys_load_u32(&a.host->tail);
            sh[2] = dev_load(&a.ctl->active);
        }
        __syncthreads();
        const int stop = sh[0], active = sh[2];
        const uint32_t tail = (uint32_t)sh[1];
        __syncthreads();
        if (stop)
            break;
        if (head != tail) {
            // copy the entry word by word with system-scope loads into the
            // slot record with agent-scope stores
            const ServeRequest* src = &a.host->ring[head % kServeRing];
            const uint32_t* sw = reinterpret_cast<const uint32_t*>(src);
            constexpr int kWords = (int)(sizeof(ServeRequest) / 4);
            const int rec = (int)(head - a.head0);
            if (rec >= kServeRecords)
                break;  // every record of this launch is used: the host relaunches
            const int slot = (int)sys_load_u32(reinterpret_cast<const uint32_t*>(&src->slot));
            ServeRequest* dst = &a.recs[rec];
            uint32_t* dw = reinterpret_cast<uint32_t*>(dst);
            for (int i = tid; i < kWords; i += kThreads)
                dev_store(dw + i, sys_load_u32(sw + i));
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (tid == 0)  // the UE state is this record's own copy
                dev_store(reinterpret_cast<uint64_t*>(&dst->t.ue), (uint64_t)(uintptr_t)dst->ue);
            // the fields needed here are read from the ring as well
            const uint32_t gen = sys_load_u32(&src->gen);
            const uint32_t wepoch = sys_load_u32(&src->wepoch);
            const int E = (int)sys_load_u32(reinterpret_cast<const uint32_t*>(&src->t.E));
            const int nt1 = (int)sys_load_u32(reinterpret_cast<const uint32_t*>(&src->ntiles[1]));
            uint8_t* state = reinterpret_cast<uint8_t*>(__hip_atomic_load(
                reinterpret_cast<const uint64_t*>(&src->t.state), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
            uint8_t* alloc = reinterpret_cast<uint8_t*>(__hip_atomic_load(
                reinterpret_cast<const uint64_t*>(&src->t.alloc), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
            ServeSlotCtl& sc = a.ctl->slot[slot];
            if (tid < E) {  // the root punctures nothing
                dev_store(state + tid, (uint8_t)0);
                dev_store(alloc + tid, (uint8_t)0);
            }
            if (tid < 8)
                dev_store(&sc.ntiles[tid], (int32_t)sys_load_u32(reinterpret_cast<const uint32_t*>(&src->ntiles[tid])));
            if (tid == 0) {
                dev_store(&sc.M, (int32_t)sys_load_u32(reinterpret_cast<const uint32_t*>(&src->t.M)));
                dev_store(&sc.rec, rec);
                dev_store(&sc.lag, (int32_t)sys_load_u32(reinterpret_cast<const uint32_t*>(&src->lag)));
                dev_store(&sc.done, 0u);
                if (wepoch != dev_load(&a.ctl->wepoch))
                    dev_store(&a.ctl->wepoch, wepoch);
            }
            __builtin_amdgcn_s_waitcnt(0);  // every store above has completed
            __syncthreads();
            if (tid == 0) {
                __hip_atomic_fetch_add(&a.ctl->active, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_max(&a.ctl->hi, slot + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_s_waitcnt(0);
                dev_store(&sc.claim, serve_claim_word(gen, 1, nt1));
                __builtin_amdgcn_s_waitcnt(0);  // the claim word is visible before the bump
                __hip_atomic_fetch_add(&a.ctl->opened, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                sys_store_u32(&a.host->consumed, head + 1);
            }
            ++head;
            since = wall_clock64();
            continue;
        }
        const uint64_t now = wall_clock64();
        if (active != last_active)
            since = now;  // a request was admitted or finished
        last_active = active;
        if (now - since > (active == 0 ? a.idle_ticks : a.stall_ticks))
            break;
        __builtin_amdgcn_s_sleep(16);
    }
    if (tid == 0)
        dev_store(&a.ctl->quit, 1);
}

// Wave 0 of a tile workgroup: claim the next tile. Every lane reads the claim
// words of two slots; the oldest request (smallest generation plus the
// slot's lag) with tiles left gets one fetch-and-add, whose result is authoritative: if it names a
// live level and a count below that level's tiles, that tile is this
// workgroup's (whatever level the slot has reached meanwhile), else the
// increment is spent and the scan repeats. Returns in sh[0] the slot (-1:
// nothing claimed), sh[1] the level, sh[2] the tile.
__device__ void serve_claim(const ServeArgs& a, int* sh)
{
    const int lane = threadIdx.x & 63;
    for (int attempt = 0; attempt < 4; ++attempt) {
        uint64_t best = ~0ull;
#pragma unroll
        for (int j = 0; j < kServeSlots / 64; ++j) {
            const int s = lane + 64 * j;
            const uint64_t w = dev_load(&a.ctl->slot[s].claim);
            const int lag = dev_load(&a.ctl->slot[s].lag);
            const int lvl = (int)((w >> 41) & 7u), nt = (int)((w >> 24) & 0x1FFFFu), cnt = (int)(w & 0xFFFFFFu);
            const uint64_t key = (((w >> 44) + (uint64_t)lag) << 8) | (uint64_t)s;
            if (lvl != 0 && cnt < nt && key < best)
                best = key;
        }
        uint64_t m = best;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint64_t v = __shfl_xor(m, o);
            m = v < m ? v : m;
        }
        if (m == ~0ull)
            break;
        const int slot = (int)(m & 0xFF);
        int got = 0;
        if (lane == 0) {
            const uint64_t w = __hip_atomic_fetch_add(&a.ctl->slot[slot].claim, (uint64_t)1, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            const int lvl = (int)((w >> 41) & 7u), nt = (int)((w >> 24) & 0x1FFFFu), cnt = (int)(w & 0xFFFFFFu);
            if (lvl != 0 && cnt < nt) {
                got = 1;
                sh[0] = slot;
                sh[1] = lvl;
                sh[2] = cnt;
                sh[3] = (int)(uint32_t)(w >> 44);  // generation
            }
        }
        if (__shfl(got, 0))
            return;
    }
    if (lane == 0)
        sh[0] = -1;
}

template <int P, int RTT>
__global__ __launch_bounds__(kThreads) void serve_kernel(ServeArgs a, const ServeRequest* __restrict__ recs)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const LevelSmem m = level_smem<RTT>(smem, a.bufsize);
    int* sh = m.tab;  // scheduler words
    if (blockIdx.x == 0) {
        serve_control(a, sh);
        return;
    }
    const int tid = threadIdx.x;
    uint32_t wepoch = 0;  // weight-refresh epoch this workgroup's caches reflect
    uint64_t since = wall_clock64();
    int backoff = 1;      // idle sleep in units of about 64 cycles, doubled up to 64
    int cont = 0;         // the previous tile opened the next level and kept its tile 0
    int worked = 1;       // the last pass ran a tile: scan again whatever opened says
    uint32_t seen = 0;    // opened as read before the last fruitless scan
    int slot = 0, tau = 0, tile = 0, rec = 0, nt = 0, M = 0;
    uint32_t gen = 0;
    for (;;) {
        if (!cont) {
            if (tid == 0) {
                sh[8] = (int)dev_load(&a.ctl->opened);
                sh[9] = dev_load(&a.ctl->quit);
                sh[12] = dev_load(&a.ctl->active);
            }
            __syncthreads();
            const uint32_t op = (uint32_t)sh[8];
            // the control workgroup has left and no admitted request is
            // unfinished (leaving while some are would leave their later
            // levels to the few workgroups still at work)
            const int quit = sh[9] && sh[12] == 0;
            __syncthreads();
            if (worked || op != seen) {
                seen = op;  // read before the scan: a level opened after it changes opened
                if (tid < 64)
                    serve_claim(a, sh);
            } else if (tid == 0) {
                sh[0] = -1;
            }
            __syncthreads();
            slot = sh[0];
            tau = sh[1];
            tile = sh[2];
            gen = (uint32_t)sh[3];
            __syncthreads();
            worked = slot >= 0;
            if (slot < 0) {
                if (quit || wall_clock64() - since > a.stall_ticks)
                    break;
                for (int i = 0; i < backoff; ++i)
                    __builtin_amdgcn_s_sleep(1);
                backoff = backoff < 64 ? 2 * backoff : 64;
                continue;
            }
            backoff = 1;
            // the request's record and the level's tiles, and a cache
            // invalidation if the host refreshed some cell's weights
            if (tid == 0) {
                const ServeSlotCtl& sc = a.ctl->slot[slot];
                sh[4] = dev_load(&sc.rec);
                sh[5] = (int)dev_load(&a.ctl->wepoch);
                sh[6] = dev_load(&sc.ntiles[tau]);
            }
            __syncthreads();
            rec = __builtin_amdgcn_readfirstlane(sh[4]);
            nt = __builtin_amdgcn_readfirstlane(sh[6]);
            const uint32_t we = (uint32_t)sh[5];
            if (we != wepoch) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                wepoch = we;
            }
        }
        since = wall_clock64();
        const DevTree& t = recs[rec].t;
        const int split = recs[rec].sub_split;
        if (split > 0) {
            // subtree units: the request is one "level" whose tiles are the
            // subtree roots; the unit writes its nodes' allocations itself
            M = 1;
            if constexpr (P == kBF16) {
                const int bufsize = recs[rec].sub_bufsize, stbytes = recs[rec].sub_stbytes;
                if (t.E <= 8)
                    subtree_body<kBF16, 2, 1, 8, 1, 8, false, true>(t, split, tile, bufsize, stbytes, smem);
                else
                    subtree_body<kBF16, 2, 1, 8, 1, 16, false, true>(t, split, tile, bufsize, stbytes, smem);
            }
        } else {
            M = t.M;
            const int n_eval = (int)(t.K * (dev_level_offset(t.K, tau) - dev_level_offset(t.K, tau - 1)));
            const int row0 = tile * 16 * RTT;
            const int nrows = min(16 * RTT, n_eval - row0);
            if (nrows > 0)
                level_tile<P, RTT, true>(t, tau, row0, nrows, m);
        }
        // every store of the tile has completed before it is counted
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
            ServeSlotCtl& sc = a.ctl->slot[slot];
            int next = 0, last = 0;
            // the only tile of a level needs no count: its workgroup finishes it
            const bool finisher =
                nt == 1 ||
                __hip_atomic_fetch_add(&sc.done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 == (uint32_t)nt;
            if (finisher) {
                if (tau < M) {
                    // open the next level with its tile 0 already claimed by
                    // this workgroup, which goes on with it at once. A next
                    // level of one tile is not published: the claim word keeps
                    // showing an earlier level with every tile taken (levels
                    // only grow, so that level had one tile too).
                    const int nt_next = recs[rec].ntiles[tau + 1];
                    if (nt_next > 1) {
                        dev_store(&sc.done, 0u);
                        __builtin_amdgcn_s_waitcnt(0);
                        dev_store(&sc.claim, serve_claim_word(gen, tau + 1, nt_next) + 1);
                        __builtin_amdgcn_s_waitcnt(0);  // tiles for others: wake the idle workgroups
                        __hip_atomic_fetch_add(&a.ctl->opened, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    next = 1;
                    sh[6] = nt_next;
                } else {
                    last = 1;  // the request is complete: finished below
                }
            }
            sh[7] = next;
            sh[10] = last;
        }
        __syncthreads();
        if (sh[10]) {
            // Every tile's stores completed before its count, so the whole
            // codebook is in device memory. A small one is delivered here,
            // into the request's block of the pinned pool (coherent word
            // loads, system-scope stores), before the finished flag.
            const ServeRequest& q = recs[rec];
            const uint32_t words = q.cb_words;
            const uint32_t* src = reinterpret_cast<const uint32_t*>(q.t.alloc);
            uint32_t* dst = reinterpret_cast<uint32_t*>(q.cb_host);
            for (uint32_t i0 = 0; i0 < words; i0 += 8 * kThreads) {
                uint32_t v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const uint32_t i = i0 + j * kThreads + tid;
                    v[j] = i < words ? dev_load(src + i) : 0u;
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const uint32_t i = i0 + j * kThreads + tid;
                    if (i < words)
                        sys_store_u32(dst + i, v[j]);
                }
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (tid == 0) {
                ServeSlotCtl& sc = a.ctl->slot[slot];
                dev_store(&sc.claim, serve_claim_word(gen, 0, 0));
                __hip_atomic_fetch_add(&a.ctl->active, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_s_waitcnt(0);
                sys_store_u32(&a.host->finished[slot], gen);
            }
        }
        __syncthreads();  // LDS is reused by the next tile
        cont = sh[7];
        if (cont) {
            ++tau;
            tile = 0;
            nt = __builtin_amdgcn_readfirstlane(sh[6]);
        }
        __syncthreads();
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

size_t level_bias_bytes(const DevTree& t)
{
    size_t n = 0;
    for (int l = 0; l < t.n_layers; ++l)
        n += (size_t)t.out_pad[l] * 4;
    return n;
}

size_t level_lds_for_buf(size_t buf, size_t bias_bytes, int rtt)
{
    return 2 * buf + (size_t)16 * rtt * kLogitStride * 4 + (kMaxUE + 4) * 4 + 2 * kMaxIn0 * 4 + pst_bytes(rtt) +
           tab_bytes() + bias_bytes;
}

size_t level_lds_bytes(const DevTree& t, int prec, int rtt)
{
    return level_lds_for_buf(level_buf_bytes(t, prec, rtt), level_bias_bytes(t), rtt);
}

bool plan_level_batch(const DevTree* trees, int n, int prec, int* rtt, int* buf, size_t* lds)
{
    const int cands[] = {6, 4, 2, 1};  // row tiles per workgroup, largest first (FP32 stops at 4)
    for (int r : cands) {
        if (prec == kFP32 && r > 4)
            continue;
        size_t b = 0, bias = 0;
        for (int i = 0; i < n; ++i) {
            b = std::max(b, level_buf_bytes(trees[i], prec, r));
            bias = std::max(bias, level_bias_bytes(trees[i]));
        }
        const size_t need = level_lds_for_buf(b, bias, r);
        if (need <= 160 * 1024) {
            *rtt = r;
            *buf = (int)b;
            *lds = need;
            return true;
        }
    }
    return false;
}

template <int P, int RTT>
static hipError_t launch_level_t(const DevTree& t, int tau, hipStream_t s, hipEvent_t done)
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
    if (done)
        hipExtLaunchKernelGGL((level_kernel<P, RTT>), dim3(grid), dim3(kThreads), lds, s, nullptr, done, 0, t, tau,
                              n_eval, buf);
    else
        hipLaunchKernelGGL((level_kernel<P, RTT>), dim3(grid), dim3(kThreads), lds, s, t, tau, n_eval, buf);
    return hipGetLastError();
}

template <int P, int RTT>
static hipError_t launch_level_batch_t(const DevTree* trees, const int* ent_tree, const int* ent_tau,
                                       const int* prefix, int n, int nblocks, int buf, size_t lds, hipStream_t s,
                                       hipEvent_t done)
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
        return done ? hipEventRecord(done, s) : hipSuccess;
    if (done)
        hipExtLaunchKernelGGL((level_kernel_batch<P, RTT>), dim3(grid), dim3(kThreads), lds, s, nullptr, done, 0,
                              trees, ent_tree, ent_tau, prefix, n, buf);
    else
        hipLaunchKernelGGL((level_kernel_batch<P, RTT>), dim3(grid), dim3(kThreads), lds, s, trees, ent_tree, ent_tau,
                           prefix, n, buf);
    return hipGetLastError();
}

hipError_t launch_level(const DevTree& t, int prec, int rtt, int tau, hipStream_t s, hipEvent_t done)
{
#define CYRUS_LEVEL_CASE(P, R)                                                                                         \
    if (prec == P && rtt == R)                                                                                         \
        return launch_level_t<P, R>(t, tau, s, done);
    CYRUS_LEVEL_CASE(kFP32, 1) CYRUS_LEVEL_CASE(kFP32, 2) CYRUS_LEVEL_CASE(kFP32, 4)
    CYRUS_LEVEL_CASE(kBF16, 1) CYRUS_LEVEL_CASE(kBF16, 2) CYRUS_LEVEL_CASE(kBF16, 4) CYRUS_LEVEL_CASE(kBF16, 6)
    CYRUS_LEVEL_CASE(kFP8, 1) CYRUS_LEVEL_CASE(kFP8, 2) CYRUS_LEVEL_CASE(kFP8, 4) CYRUS_LEVEL_CASE(kFP8, 6)
#undef CYRUS_LEVEL_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_level_batch(const DevTree* trees, const int* ent_tree, const int* ent_tau, const int* prefix, int n,
                              int nblocks, int prec, int rtt, int buf, size_t lds, hipStream_t s, hipEvent_t done)
{
#define CYRUS_LEVEL_CASE(P, R)                                                                                         \
    if (prec == P && rtt == R)                                                                                         \
        return launch_level_batch_t<P, R>(trees, ent_tree, ent_tau, prefix, n, nblocks, buf, lds, s, done);
    CYRUS_LEVEL_CASE(kFP32, 1) CYRUS_LEVEL_CASE(kFP32, 2) CYRUS_LEVEL_CASE(kFP32, 4)
    CYRUS_LEVEL_CASE(kBF16, 1) CYRUS_LEVEL_CASE(kBF16, 2) CYRUS_LEVEL_CASE(kBF16, 4) CYRUS_LEVEL_CASE(kBF16, 6)
    CYRUS_LEVEL_CASE(kFP8, 1) CYRUS_LEVEL_CASE(kFP8, 2) CYRUS_LEVEL_CASE(kFP8, 4) CYRUS_LEVEL_CASE(kFP8, 6)
#undef CYRUS_LEVEL_CASE
    return hipErrorInvalidValue;
}

template <int P, int RTT>
static hipError_t launch_serve_t(const ServeArgs& a, int grid, size_t lds, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&serve_kernel<P, RTT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL((serve_kernel<P, RTT>), dim3(grid), dim3(kThreads), lds, s, a,
                       static_cast<const ServeRequest*>(a.recs));
    return hipGetLastError();
}

hipError_t launch_serve(const ServeArgs& a, int prec, int rtt, int grid, size_t lds, hipStream_t s)
{
    if (grid < 2 || lds < level_lds_for_buf(0, 0, rtt))
        return hipErrorInvalidValue;
#define CYRUS_SERVE_CASE(P, R)                                                                                         \
    if (prec == P && rtt == R)                                                                                         \
        return launch_serve_t<P, R>(a, grid, lds, s);
    CYRUS_SERVE_CASE(kFP32, 1) CYRUS_SERVE_CASE(kFP32, 2) CYRUS_SERVE_CASE(kFP32, 4)
    CYRUS_SERVE_CASE(kBF16, 1) CYRUS_SERVE_CASE(kBF16, 2) CYRUS_SERVE_CASE(kBF16, 4) CYRUS_SERVE_CASE(kBF16, 6)
    CYRUS_SERVE_CASE(kFP8, 1) CYRUS_SERVE_CASE(kFP8, 2) CYRUS_SERVE_CASE(kFP8, 4) CYRUS_SERVE_CASE(kFP8, 6)
#undef CYRUS_SERVE_CASE
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
