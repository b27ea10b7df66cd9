// The Near-RT RIC's critic pass (Sec. IV-B, Eqs. (3) and (4)) on MFMA. Each
// tile of 16*RTT rows (sample h, step tau) gets four workgroups, one per role,
// running FP32 MLPs with the activations in LDS and the weight fragments read
// from L2:
//   role 0, 1: critic Q1 or Q2 on [state, y];
//   role 2, 3: the actor at step tau+1, whose Gaussian draws give a fresh
//              action y~ and its log density, then target critic 1 or 2 on
//              [state at tau+1, y~].
// Roles 2 and 3 draw the same y~ (the draws are a function of the row, not of
// the thread), so no workgroup waits for another and the longest chain is two
// networks. A second, one-workgroup kernel forms the target of Eq. (4) and the
// mean squared errors of Eq. (3) in a fixed summation order.
#include "cyrus_device.h"
#include "cyrus_kernels.h"
#include "cyrus_mlp.h"
#include "cyrus_regmlp.h"

namespace cyrus {

namespace {

constexpr float kHalfLog2Pi = 0.91893853320467274f;
constexpr float kLog2 = 0.69314718055994531f;

// The tile's inputs, staged in LDS once: the UE state of the samples it
// touches, and k, c, y of its rows plus the row after the last (for step
// tau+1 of the last row).
struct CriticStage {
    int32_t* ue;  // [(RT / M + 2) samples][3E]
    int32_t* k;   // [RT + 1]
    int32_t* c;   // [(RT + 1) E]
    float* y;     // [RT E]
    int h0;
};

// Input value f of a network for row `row`, whose step is `tau` (1-based) and
// whose stored inputs sit at staged row `srow`: R/32, MCS/32, SINR/32, c/64
// per UE, tau/8, k/8, then the action (critic only: y_row, else zero), zero
// padded.
__device__ __forceinline__ float critic_feature(const CriticArgs& a, const CriticStage& st, int f, int h, int tau,
                                                int srow, const float* y_row)
{
    const int E = a.E;
    const int32_t* ue = st.ue + (h - st.h0) * 3 * E;
    if (f < 2 * E)
        return (float)ue[f] * (1.f / 32.f);
    if (f < 3 * E)
        return __int_as_float(ue[f]) * (1.f / 32.f);
    if (f < 4 * E)
        return (float)st.c[srow * E + f - 3 * E] * (1.f / 64.f);
    if (f == 4 * E)
        return (float)tau * (1.f / 8.f);
    if (f == 4 * E + 1)
        return (float)st.k[srow] * (1.f / 8.f);
    if (y_row && f < 5 * E + 2)
        return y_row[f - 4 * E - 2];
    return 0.f;
}

// One workgroup's share of a tile: staging, then the networks of its role.
// run_net(n, nrows, bufA, bufB, zl, bias) evaluates network n over the
// tile's rows, whose inputs are in bufA (row stride in_pad[0] + 4 floats),
// and leaves its outputs, bias included, in zl[row * kLogitStride + e].
template <int RT, class RunNet>
__device__ __forceinline__ void critic_tile(const CriticArgs& a, uint8_t* smem, RunNet run_net)
{
    uint8_t* bufA = smem;
    uint8_t* bufB = smem + a.bufsize;
    float* zl = reinterpret_cast<float*>(smem + 2 * a.bufsize);
    float* bias = zl + RT * kLogitStride;        // every network's biases
    float* lp = bias + a.bias_total;             // [RT] log pi of y~
    float* yt = lp + RT;                         // [RT][16] y~
    float* lpe = yt + RT * 16;                   // [RT][16] per-UE log-density terms
    CriticStage st;
    st.ue = reinterpret_cast<int32_t*>(lpe + RT * 16);
    st.k = st.ue + (RT + 2) * 3 * kMaxUE / 2;  // room for RT + 2 samples of E <= 16
    st.c = st.k + RT + 4;
    st.y = reinterpret_cast<float*>(st.c + (RT + 1) * 16);

    const int E = a.E, M = a.M;
    const int rows = a.H * M;
    const int role = (int)(blockIdx.x & 3u);
    const int j0 = (int)(blockIdx.x >> 2) * RT;
    const int nrows = min(RT, rows - j0);
    if (nrows <= 0)
        return;
    const int nin = min(nrows + 1, rows - j0);  // staged rows: the tile's, and the next one if it exists
    st.h0 = j0 / M;
    const int nsamp = (j0 + nin - 1) / M - st.h0 + 1;
    // stage the biases of all five networks and the tile's inputs: every
    // thread issues all its global loads (fixed, unrolled counts) before its
    // first LDS store, so the staging costs one memory latency. A layer has at
    // most kThreads outputs, so a thread copies at most one bias per layer.
    const int tid = threadIdx.x;
    float bv[5][kMaxLayers];
#pragma unroll
    for (int n = 0; n < 5; ++n)
#pragma unroll
        for (int l = 0; l < kMaxLayers; ++l) {
            const DevTree& t = a.nets[n];
            bv[n][l] = (l < t.n_layers && tid < t.out_pad[l]) ? gptr(t.b[l])[tid] : 0.f;
        }
    constexpr int nUe = ((RT + 2) * 3 * 16 + kThreads - 1) / kThreads;  // samples touched <= RT + 2, E <= 16
    constexpr int nC = ((RT + 1) * 16 + kThreads - 1) / kThreads;
    constexpr int nY = (RT * 16 + kThreads - 1) / kThreads;
    int32_t uev[nUe], cv[nC];
    float yv[nY];
#pragma unroll
    for (int q = 0; q < nUe; ++q) {
        const int i = tid + q * kThreads;
        uev[q] = i < nsamp * 3 * E ? gptr(a.ue)[(int64_t)st.h0 * 3 * E + i] : 0;
    }
    const int32_t kv = tid < nin ? gptr(a.k)[j0 + tid] : 0;
#pragma unroll
    for (int q = 0; q < nC; ++q) {
        const int i = tid + q * kThreads;
        cv[q] = i < nin * E ? (int32_t)gptr(a.c)[(int64_t)j0 * E + i] : 0;
    }
#pragma unroll
    for (int q = 0; q < nY; ++q) {
        const int i = tid + q * kThreads;
        yv[q] = i < nrows * E ? gptr(a.y)[(int64_t)j0 * E + i] : 0.f;
    }
#pragma unroll
    for (int n = 0; n < 5; ++n) {
        const DevTree& t = a.nets[n];
        int off = a.bias_off[n];
#pragma unroll
        for (int l = 0; l < kMaxLayers; ++l) {
            if (l < t.n_layers) {
                if (tid < t.out_pad[l])
                    bias[off + tid] = bv[n][l];
                off += t.out_pad[l];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < nUe; ++q) {
        const int i = tid + q * kThreads;
        if (i < nsamp * 3 * E)
            st.ue[i] = uev[q];
    }
    if (tid < nin)
        st.k[tid] = kv;
#pragma unroll
    for (int q = 0; q < nC; ++q) {
        const int i = tid + q * kThreads;
        if (i < nin * E)
            st.c[i] = cv[q];
    }
#pragma unroll
    for (int q = 0; q < nY; ++q) {
        const int i = tid + q * kThreads;
        if (i < nrows * E)
            st.y[i] = yv[q];
    }
    lds_barrier();

    // network input rows: critic (5E+2, stride sc) or actor (4E+2, stride sa)
    // floats, for the row's own step (next = false) or step tau+1 (next =
    // true; rows whose step is the last are zero)
    auto fill = [&](int width, int stride, bool next, bool with_y, const float* ysrc) {
        for (int idx = threadIdx.x; idx < RT * width; idx += kThreads) {
            const int row = idx / width, f = idx - row * width;
            const int j = j0 + row;
            float v = 0.f;
            if (row < nrows && (!next || (j % M) + 1 < M)) {
                const int srow = row + (next ? 1 : 0);
                const float* yr = !with_y ? nullptr : (ysrc ? ysrc + row * 16 : st.y + row * E);
                v = critic_feature(a, st, f, j / M, j % M + 1 + (next ? 1 : 0), srow, yr);
            }
            reinterpret_cast<float*>(bufA)[row * stride + f] = v;
        }
        lds_barrier();
    };
    const int wc = a.nets[1].in_pad[0], sc = wc + 4;
    const int wa = a.nets[0].in_pad[0], sa = wa + 4;
    auto net = [&](int n) { run_net(n, nrows, bufA, bufB, zl, bias); };

    if (role < 2) {
        // Q1 or Q2 on the stored action
        fill(wc, sc, false, true, nullptr);
        net(1 + role);
        for (int row = threadIdx.x; row < nrows; row += kThreads)
            a.q[(int64_t)role * rows + j0 + row] = zl[row * kLogitStride];
        return;
    }

    // the actor at step tau+1
    fill(wa, sa, true, false, nullptr);
    net(0);
    // y~ = (1 + tanh u) / 2 with u = mu + sigma eps, and the terms of log pi:
    // -eps^2/2 - log sigma - log(2 pi)/2 - log|dy/du|, where
    // log|dy/du| = log 2 - 2|u| - 2 log(1 + e^-2|u|)
    for (int idx = threadIdx.x; idx < nrows * 16; idx += kThreads) {
        const int row = idx >> 4, e = idx & 15;
        const int j = j0 + row;
        float y = 0.f, term = 0.f;
        if (e < E && (j % M) + 1 < M && st.k[row + 1] > 0) {
            const float mu = zl[row * kLogitStride + e];
            const float ls = clamp_log_sigma(zl[row * kLogitStride + E + e]);
            const float eps = gaussian_eps(a.seed, a.episode, (int64_t)(j + 1), e);
            const float u = mu + expf(ls) * eps;
            y = 0.5f * (1.f + tanhf(u));
            const float au = fabsf(u);
            const float log_jac = kLog2 - 2.f * au - 2.f * log1pf(expf(-2.f * au));
            term = -0.5f * eps * eps - ls - kHalfLog2Pi - log_jac;
        }
        yt[row * 16 + e] = y;
        lpe[row * 16 + e] = term;
    }
    lds_barrier();
    if (role == 2)
        for (int row = threadIdx.x; row < nrows; row += kThreads) {
            float s = 0.f;
            for (int e = 0; e < E; ++e)
                s += lpe[row * 16 + e];
            a.tlp[j0 + row] = s;
        }
    // target critic 1 or 2 on [state at tau+1, y~]
    fill(wc, sc, true, true, yt);
    net(1 + role);
    for (int row = threadIdx.x; row < nrows; row += kThreads)
        a.tq[(int64_t)(role - 2) * rows + j0 + row] = zl[row * kLogitStride];
}

template <int RTT>
__global__ __launch_bounds__(kThreads) void critic_kernel(CriticArgs a)
{
    extern __shared__ __align__(16) uint8_t smem[];
    critic_tile<16 * RTT>(a, smem, [&](int n, int nrows, uint8_t* bufA, uint8_t* bufB, float* zl, const float* bias) {
        run_mlp<kFP32, RTT>(a.nets[n], nrows, bufA, bufB, zl, bias + a.bias_off[n], 0, 0);
    });
}

// Register-resident variant for networks of two hidden layers of 128 T
// neurons, CH1 first-layer chunks (all five networks padded alike) and at
// most 16 outputs. For each network a workgroup runs, every wave loads its
// fragments into registers in one burst (the target critic of roles 2 and 3
// reuses the registers of the actor), and the layers run from registers as in
// the subtree kernel. The waves' partial outputs are added in wave order.
template <int T, int CH1, int RTT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 2))) void critic_regs_kernel(
    CriticArgs a)
{
    constexpr int CHH = 8 * T, kRT = Rows<kFP32>::kRT;
    static_assert(16 * RTT <= kRT, "row tiles of one pass");
    extern __shared__ __align__(16) uint8_t smem[];
    WaveWeights<kFP32, T, CH1, CHH, 1> W;
    const int lane = threadIdx.x & 63, wave = wave_id();
    critic_tile<16 * RTT>(a, smem, [&](int n, int nrows, uint8_t* bufA, uint8_t* bufB, float* zl, const float* bias) {
        const DevTree& t = a.nets[n];
        load_weights(t, W, wave, lane);
        const int boff[3] = {0, t.out_pad[0], t.out_pad[0] + t.out_pad[1]};
        const float* b = bias + a.bias_off[n];
        const float* part = mlp_mfma<kFP32, T, CH1, CHH, 1>(t, W, nrows, bufA, bufB, b, boff);
        for (int idx = threadIdx.x; idx < nrows * 16; idx += kThreads) {
            const int row = idx >> 4, e = idx & 15;
            float s = 0.f;
#pragma unroll
            for (int w = 0; w < kWaves; ++w)
                s += part[(size_t)(w * kRT + row) * 16 + e];
            zl[row * kLogitStride + e] = s + b[boff[2] + e];
        }
        lds_barrier();
    });
}

// The target of Eq. (4) per row, then loss[i] = mean over rows of
// (q[i][row] - qhat[row])^2. Thread t takes rows t, t + 512, ... in batches of
// four per thread whose loads are all issued before the arithmetic; the
// thread sums then meet in a fixed-order tree in LDS.
__global__ __launch_bounds__(kThreads) void critic_loss_kernel(CriticArgs a)
{
    constexpr int kB = 4;
    __shared__ float part[2][kThreads];
    const int rows = a.H * a.M, tid = threadIdx.x;
    float s0 = 0.f, s1 = 0.f;
    for (int base = 0; base < rows; base += kB * kThreads) {
        float q0[kB], q1[kB], t1[kB], t2[kB], lp[kB], rw[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            const int j = base + b * kThreads + tid;
            const bool in = j < rows;
            const int jj = in ? j : 0;
            q0[b] = a.q[jj];
            q1[b] = a.q[rows + jj];
            t1[b] = a.tq[jj];
            t2[b] = a.tq[rows + jj];
            lp[b] = a.tlp[jj];
            rw[b] = a.reward[jj / a.M];
        }
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            const int j = base + b * kThreads + tid;
            if (j < rows) {
                const float target = (j % a.M) + 1 == a.M
                                         ? rw[b]
                                         : a.discount * (fminf(t1[b], t2[b]) - a.entropy_coef * lp[b]);
                a.qhat[j] = target;
                const float d0 = q0[b] - target, d1 = q1[b] - target;
                s0 += d0 * d0;
                s1 += d1 * d1;
            }
        }
    }
    part[0][tid] = s0;
    part[1][tid] = s1;
    __syncthreads();
    for (int w = kThreads / 2; w >= 1; w >>= 1) {
        if (tid < w) {
            part[0][tid] += part[0][tid + w];
            part[1][tid] += part[1][tid + w];
        }
        __syncthreads();
    }
    if (tid < 2)
        a.loss[tid] = part[tid][0] / (float)rows;
}

}  // namespace

size_t critic_lds_bytes(int bufsize, int bias_total, int rtt)
{
    const size_t RT = 16 * (size_t)rtt;
    const size_t stage = ((RT + 2) * 3 * kMaxUE / 2 + RT + 4 + (RT + 1) * 16) * 4 + RT * 16 * 4;
    return 2 * (size_t)bufsize + RT * kLogitStride * 4 + (size_t)bias_total * 4 + RT * 4 + RT * 16 * 4 * 2 + stage;
}

template <void (*K)(CriticArgs)>
static hipError_t launch_critic_k(int tile_rows, const CriticArgs& a, size_t lds, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(K), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        attr = true;
    }
    const int rows = a.H * a.M;
    const int grid = 4 * ((rows + tile_rows - 1) / tile_rows);  // four roles per row tile
    hipLaunchKernelGGL(K, dim3(grid), dim3(kThreads), lds, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(critic_loss_kernel, dim3(1), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_critic(const CriticArgs& a, int rtt, int regs_t, int regs_ch1, size_t lds, hipStream_t s)
{
    if (regs_t == 2) {
        if (regs_ch1 == 1)
            return launch_critic_k<critic_regs_kernel<2, 1, 2>>(32, a, lds, s);
        if (regs_ch1 == 2)
            return launch_critic_k<critic_regs_kernel<2, 2, 2>>(32, a, lds, s);
        return launch_critic_k<critic_regs_kernel<2, 3, 2>>(32, a, lds, s);
    }
    if (regs_t == 1) {
        if (regs_ch1 == 1)
            return launch_critic_k<critic_regs_kernel<1, 1, 2>>(32, a, lds, s);
        if (regs_ch1 == 2)
            return launch_critic_k<critic_regs_kernel<1, 2, 2>>(32, a, lds, s);
        return launch_critic_k<critic_regs_kernel<1, 3, 2>>(32, a, lds, s);
    }
    switch (rtt) {
    case 4:
        return launch_critic_k<critic_kernel<4>>(64, a, lds, s);
    case 2:
        return launch_critic_k<critic_kernel<2>>(32, a, lds, s);
    default:
        return launch_critic_k<critic_kernel<1>>(16, a, lds, s);
    }
}

}  // namespace cyrus
