/*
 * FP64 reference ("oracle") for the Cyrus+ real-time O-DU puncturing-codebook
 * builder (arXiv 2506.00167).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline of the benchmark load this file. The product path never calls it and
 * shares no code with it: the HIP library has its own kernels, headers and
 * helpers. The oracle is plain, slow and written to be checked against the
 * paper by eye: every loop follows the definition it cites, in float64.
 *
 * What it computes (the O-DU side of Sec. IV-C, Sec. V-B and Alg. 2, extended
 * from one mini-slot to the tree of all arrival sequences over a slot):
 *
 *   For every prefix (k_1..k_tau) of URLLC arrival counts, tau = 1..M,
 *   k_t in {0..K} with K = floor(N/L) (Sec. III-A, Sec. IV-A):
 *     c_in   = sum of the puncturing vectors chosen on the path so far
 *     if k_tau == 0: no URLLC packet, nothing is punctured (the no-arrival
 *                    branch is not considered by the O-DU, Sec. IV-C footnote)
 *     else:          x = features(s(t), c_in, tau, k_tau)
 *                    z = f_a(x)                      actor forward, Sec. VI-B
 *                    p = softmax(z)                  policy split
 *                    xq = KL projection of T*p onto {0 <= m_e <= R_e,
 *                         sum m_e = T}               Eqs. (6)-(7)
 *                    a = integer rounding of xq keeping sum = T
 *     node state passed to the children = c_in + a
 *
 * Readings of points the paper leaves open (each is listed with its reason in
 * the design notes of the repository):
 *   - f_a outputs E logits; the split is softmax(z) instead of a Gaussian
 *     sample passed through tanh. The KL projection of Eq. (7) only rescales
 *     its input, so any positive vector proportional to the policy output
 *     gives the same projection.
 *   - softmax arguments z_e - max(z) are clamped below at -80, so every p_e is
 *     positive and the capped split stays well defined.
 *   - T = min(U*k, sum_e R_e): demand is capped by the RBs scheduled in the
 *     TTI (Eq. (7) has no solution above that). Caps are per mini-slot.
 *   - The integer step is largest remainder (Hamilton) rounding with ties
 *     broken towards the lower UE index by default; the paper names
 *     Huntington-Hill, which cannot place fewer units than there are positive
 *     quotas. Huntington-Hill is the other rounding mode (priority form, ties
 *     to the larger share then the lower index; below one unit per positive
 *     share the T largest shares get one unit each).
 *   - Features (dim 4E+2, blocks of E): R_e/32, MCS_e/32, SINR_e/32, c_e/64,
 *     then tau/8 and k/8. All scales are powers of two.
 *   - BFS node order, level by level; within a level k_1 is the most
 *     significant digit, so the children of node i of level tau-1 are nodes
 *     (K+1)i + k of level tau.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

#define ORACLE_EXACT 0
#define ORACLE_BF16 1
#define ORACLE_FP8_E4M3 2

#define SOFTMAX_FLOOR (-80.0)
#define MAX_UE 64
#define MAX_WIDTH 4096

typedef struct {
    int32_t num_ue;        /* E */
    int32_t max_arrival;   /* K */
    int32_t num_minislots; /* M */
    int32_t rb_per_unit;   /* U */
    int32_t rounding;      /* ORACLE_LARGEST_REMAINDER or ORACLE_HUNTINGTON_HILL */
    int32_t head;          /* ORACLE_SOFTMAX_HEAD (E logits) or ORACLE_GAUSSIAN_HEAD (2E: mu, log sigma) */
    uint64_t seed;         /* Gaussian head: Philox key */
    uint64_t tti;          /* Gaussian head: TTI number, part of the Philox counter */
} oracle_tree;

#define ORACLE_LARGEST_REMAINDER 0
#define ORACLE_HUNTINGTON_HILL 1
#define ORACLE_SOFTMAX_HEAD 0
#define ORACLE_GAUSSIAN_HEAD 1

typedef struct {
    int32_t num_layers;      /* weight layers: hidden layers + output layer */
    const int32_t* dims;     /* num_layers + 1 widths: d_in, hidden..., E */
    const float* const* w;   /* w[l]: row-major [dims[l+1]][dims[l]] */
    const float* const* b;   /* b[l]: [dims[l+1]] */
    int32_t precision;       /* ORACLE_EXACT, ORACLE_BF16, ORACLE_FP8_E4M3 */
    const double* act_scale; /* FP8: scale of each layer input (num_layers) */
    const double* const* wq; /* optional: w[l] already rounded to `precision`
                                (oracle_quantize_weights); NULL rounds on use */
} oracle_actor;

/* ---------------------------------------------------------------- tree size */

static int64_t ipow64(int64_t base, int32_t e)
{
    int64_t r = 1;
    for (int32_t i = 0; i < e; ++i)
        r *= base;
    return r;
}

/* First node index of level tau in BFS order: ((K+1)^tau - 1) / K. */
int64_t oracle_level_offset(int32_t K, int32_t tau)
{
    return (ipow64(K + 1, tau) - 1) / K;
}

/* Nodes in levels 0..M, the root included. */
int64_t oracle_num_nodes(int32_t K, int32_t M)
{
    return oracle_level_offset(K, M + 1);
}

/* ------------------------------------------------------- number formats */

/* Round v to the nearest value with `bits` significant bits (ties to even),
 * with the exponent of the quantum floored at min_exp (gradual underflow). */
static double round_sig(double v, int bits, int min_exp)
{
    if (v == 0.0 || !isfinite(v))
        return v;
    int e;
    frexp(fabs(v), &e);              /* |v| = f * 2^e, f in [0.5, 1) */
    int q_exp = (e - 1) - (bits - 1); /* exponent of one unit in the last place */
    if (q_exp < min_exp)
        q_exp = min_exp;
    double q = ldexp(1.0, q_exp);
    return nearbyint(v / q) * q; /* default rounding mode: nearest, ties even */
}

/* bfloat16: 8 significant bits, exponent range of float32. */
double oracle_round_bf16(double v)
{
    return round_sig(v, 8, -126 - 7);
}

/* OCP FP8 E4M3 (no infinities): 4 significant bits, smallest normal 2^-6,
 * subnormal quantum 2^-9, largest finite 448. Out-of-range values saturate. */
double oracle_round_e4m3(double v)
{
    double r = round_sig(v, 4, -9);
    if (r > 448.0)
        r = 448.0;
    if (r < -448.0)
        r = -448.0;
    return r;
}

/* ------------------------------------------------------------- features */

/* State vector of one node: s(t) per UE (RBs, MCS, SINR), the RBs punctured
 * so far on this path, the mini-slot index and the arrival count. The paper
 * feeds [s(t), j] (Sec. VI-B); the extra per-UE channel features and the
 * carried state follow the tree extension. */
void oracle_features(int32_t E, const int32_t* rb, const int32_t* mcs, const float* sinr_db,
                     const int32_t* c, int32_t tau, int32_t k, double* x)
{
    for (int32_t e = 0; e < E; ++e) {
        x[e] = rb[e] / 32.0;
        x[E + e] = mcs[e] / 32.0;
        x[2 * E + e] = (double)sinr_db[e] / 32.0;
        x[3 * E + e] = c[e] / 64.0;
    }
    x[4 * E] = tau / 8.0;
    x[4 * E + 1] = k / 8.0;
}

/* -------------------------------------------------------------- actor */

static double quantize(double v, int32_t precision, double scale)
{
    if (precision == ORACLE_BF16)
        return oracle_round_bf16(v);
    if (precision == ORACLE_FP8_E4M3)
        return oracle_round_e4m3(v / scale) * scale;
    return v;
}

/* Power-of-two per-tensor scale for E4M3 weights: the smallest 2^n with
 * max|w| / 2^n <= 448. */
double oracle_e4m3_weight_scale(const float* w, int64_t n)
{
    double amax = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (fabs((double)w[i]) > amax)
            amax = fabs((double)w[i]);
    if (amax == 0.0)
        return 1.0;
    double s = 1.0;
    while (amax / s > 448.0)
        s *= 2.0;
    while (amax / (s * 0.5) <= 448.0)
        s *= 0.5;
    return s;
}

/* Round a whole weight tensor to `precision`, scale included, into doubles
 * (the values the reduced-precision forward pass multiplies with). */
void oracle_quantize_weights(const float* w, int64_t n, int32_t precision, double* out)
{
    double s = (precision == ORACLE_FP8_E4M3) ? oracle_e4m3_weight_scale(w, n) : 1.0;
    for (int64_t i = 0; i < n; ++i)
        out[i] = quantize((double)w[i], precision, s);
}

/* Forward pass of the actor f_a: h_{l+1} = ReLU(W_l h_l + b_l) for the hidden
 * layers and z = W_L h_L + b_L for the output (Sec. VI-B: each layer is the
 * product with the weight matrix plus the bias, then the activation, layer
 * after layer). The three-layer actor of the case study is num_layers = 2.
 *
 * With a reduced precision the layer inputs and weights are first rounded to
 * that format (per-tensor power-of-two scales for E4M3), the products and
 * sums stay exact in float64, and the bias is added unrounded. amax, if not
 * NULL, receives the running maximum |input| of every layer. */
int oracle_mlp(const oracle_actor* f, const double* x, double* z, double* amax)
{
    if (!f || f->num_layers < 1)
        return ORACLE_EINVAL;
    double* h = (double*)malloc(sizeof(double) * MAX_WIDTH);
    double* g = (double*)malloc(sizeof(double) * MAX_WIDTH);
    if (!h || !g) {
        free(h);
        free(g);
        return ORACLE_ENOMEM;
    }
    int32_t n_in = f->dims[0];
    for (int32_t i = 0; i < n_in; ++i)
        h[i] = x[i];
    for (int32_t l = 0; l < f->num_layers; ++l) {
        int32_t in = f->dims[l], out = f->dims[l + 1];
        if (in > MAX_WIDTH || out > MAX_WIDTH) {
            free(h);
            free(g);
            return ORACLE_EINVAL;
        }
        double s_act = (f->act_scale ? f->act_scale[l] : 1.0);
        double s_w = 1.0;
        if (f->precision == ORACLE_FP8_E4M3 && !f->wq)
            s_w = oracle_e4m3_weight_scale(f->w[l], (int64_t)in * out);
        if (amax)
            for (int32_t i = 0; i < in; ++i)
                if (fabs(h[i]) > amax[l])
                    amax[l] = fabs(h[i]);
        for (int32_t i = 0; i < in; ++i)
            h[i] = quantize(h[i], f->precision, s_act);
        for (int32_t o = 0; o < out; ++o) {
            double acc = 0.0;
            if (f->wq) {
                const double* wrow = f->wq[l] + (int64_t)o * in;
                for (int32_t i = 0; i < in; ++i)
                    acc += wrow[i] * h[i];
            } else {
                const float* wrow = f->w[l] + (int64_t)o * in;
                for (int32_t i = 0; i < in; ++i)
                    acc += quantize((double)wrow[i], f->precision, s_w) * h[i];
            }
            acc += (double)f->b[l][o];
            g[o] = (l + 1 < f->num_layers && acc < 0.0) ? 0.0 : acc;
        }
        memcpy(h, g, sizeof(double) * out);
    }
    memcpy(z, h, sizeof(double) * f->dims[f->num_layers]);
    free(h);
    free(g);
    return ORACLE_OK;
}

/* ------------------------------------------- feasibility enforcer, Sec. V-B */

/* p_e = exp(z_e - max z) / sum_j exp(z_j - max z), arguments clamped at -80. */
void oracle_softmax(int32_t E, const double* z, double* p)
{
    double zmax = z[0];
    for (int32_t e = 1; e < E; ++e)
        if (z[e] > zmax)
            zmax = z[e];
    double sum = 0.0;
    for (int32_t e = 0; e < E; ++e) {
        double d = z[e] - zmax;
        if (d < SOFTMAX_FLOOR)
            d = SOFTMAX_FLOOR;
        p[e] = exp(d);
        sum += p[e];
    }
    for (int32_t e = 0; e < E; ++e)
        p[e] /= sum;
}

/* Infeasibility (i): the nearest vector in KL divergence, Eqs. (6)-(7),
 *     min  sum_e b_e log(b_e / bhat_e)   s.t.  0 <= bhat_e <= R_e,
 *                                              sum_e bhat_e = T,
 * for b proportional to p. Stationarity of the Lagrangian gives
 * bhat_e = min(R_e, s * p_e) with one multiplier s fixed by the sum: UEs whose
 * proportional share reaches their cap are pinned to it and the rest of the
 * demand is split in proportion to p among the others ("water-filling").
 * The capped set only grows and s only increases, so at most E passes.
 * Returns the final s; x receives bhat. */
double oracle_capped_scale(int32_t E, const double* p, const int32_t* R, int64_t T, double* x)
{
    int capped[MAX_UE];
    int64_t rsum = 0;
    for (int32_t e = 0; e < E; ++e) {
        capped[e] = 0;
        rsum += R[e];
    }
    if (T <= 0) {
        for (int32_t e = 0; e < E; ++e)
            x[e] = 0.0;
        return 0.0;
    }
    if (T >= rsum) { /* all capacity is used: bhat = R */
        for (int32_t e = 0; e < E; ++e)
            x[e] = R[e];
        return INFINITY;
    }
    double s = 0.0;
    for (;;) {
        double rem = (double)T, psum = 0.0;
        for (int32_t e = 0; e < E; ++e) {
            if (capped[e])
                rem -= R[e];
            else
                psum += p[e];
        }
        s = rem / psum;
        int added = 0;
        for (int32_t e = 0; e < E; ++e)
            if (!capped[e] && s * p[e] >= (double)R[e]) {
                capped[e] = 1;
                added = 1;
            }
        if (!added)
            break;
    }
    for (int32_t e = 0; e < E; ++e)
        x[e] = capped[e] ? (double)R[e] : s * p[e];
    return s;
}

/* ------------------------------------------------------- Gaussian head */

/* Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and Shaw
 * (SC'11), written from its definition: ten rounds, each multiplying counter
 * words 0 and 2 by the two round constants into 64-bit products, then
 * recombining (hi(R1 c2) ^ c1 ^ k0, lo(R1 c2), hi(R0 c0) ^ c3 ^ k1, lo(R0 c0));
 * the key is bumped by the two Weyl constants between rounds. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n1 = (uint32_t)p1;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        const uint32_t n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* The standard normal draw of UE e at tree node `node` in TTI `tti`: Philox
 * with key = seed and counter = (node, e, tti low, tti high), then Box-Muller
 * on the first two words, each mapped to (0, 1) as (w + 1/2) / 2^32. */
double oracle_normal(uint64_t seed, uint64_t tti, int64_t node, int32_t e)
{
    const uint32_t ctr[4] = {(uint32_t)node, (uint32_t)e, (uint32_t)tti, (uint32_t)(tti >> 32)};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    const double u1 = ((double)w[0] + 0.5) / 4294967296.0;
    const double u2 = ((double)w[1] + 0.5) / 4294967296.0;
    const double two_pi = 6.283185307179586476925286766559;
    return sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
}

/* Log standard deviations are clamped to [-20, 2] (the usual SAC bounds). */
static double clamp_log_sigma(double ls)
{
    return ls < -20.0 ? -20.0 : (ls > 2.0 ? 2.0 : ls);
}

/* The paper's stochastic policy head (Sec. IV-B and its GPU implementation):
 * the actor's 2E outputs are means mu_e and, in the usual SAC form, log
 * standard deviations clamped to [-20, 2]; u_e = mu_e + sigma_e eps_e with the
 * reparameterisation trick; tanh maps the sample to b_e = (1 + tanh u_e) / 2 in
 * (0, 1). The KL projection only needs b up to its scale, so the node's
 * logits are z_e = log b_e, evaluated as -log(1 + exp(-2 u_e)) (the same
 * number: (1 + tanh u) / 2 is the logistic function of 2u), and softmax(z) =
 * b / sum b. */
void oracle_gaussian_head(int32_t E, const double* out, uint64_t seed, uint64_t tti, int64_t node, double* z)
{
    for (int32_t e = 0; e < E; ++e) {
        const double ls = clamp_log_sigma(out[E + e]);
        const double u = out[e] + exp(ls) * oracle_normal(seed, tti, node, e);
        z[e] = u >= 0.0 ? -log1p(exp(-2.0 * u)) : 2.0 * u - log1p(exp(2.0 * u));
    }
}

/* log of the density of the policy's action y = (1 + tanh u) / 2 at the
 * pre-tanh point u, for the actor outputs (mu, log sigma): the Gaussian log
 * density of u minus the log of |dy/du| = (1 - tanh(u)^2) / 2 (change of
 * variables), summed over the E independent UEs. log((1 - tanh^2 u) / 2) is
 * log(2 y (1 - y)), evaluated as log 2 - log(1 + e^-2u) - log(1 + e^2u). */
double oracle_log_prob_tanh_gaussian(int32_t E, const double* out, const double* u)
{
    const double half_log_two_pi = 0.91893853320467274178032973640562;
    double lp = 0.0;
    for (int32_t e = 0; e < E; ++e) {
        const double ls = clamp_log_sigma(out[E + e]);
        const double d = (u[e] - out[e]) / exp(ls);
        const double log_jac = log(2.0) - log1p(exp(-2.0 * u[e])) - log1p(exp(2.0 * u[e]));
        lp += -0.5 * d * d - ls - half_log_two_pi - log_jac;
    }
    return lp;
}

/* One action of the policy for the critic's target (Eq. (4)): the same draws
 * as the Gaussian head, y_e = (1 + tanh u_e) / 2 with u = mu + sigma eps; returns
 * log pi(y). */
double oracle_sample_tanh_gaussian(int32_t E, const double* out, uint64_t seed, uint64_t tti, int64_t node, double* y)
{
    double u[MAX_UE];
    for (int32_t e = 0; e < E; ++e) {
        const double ls = clamp_log_sigma(out[E + e]);
        u[e] = out[e] + exp(ls) * oracle_normal(seed, tti, node, e);
        y[e] = (1.0 + tanh(u[e])) / 2.0;
    }
    return oracle_log_prob_tanh_gaussian(E, out, u);
}

/* Infeasibility (ii): integer rounding that keeps sum = T. Largest remainder:
 * floor every share, then give one more unit to each of the r = T - sum floor
 * UEs with the largest fractional parts among those still below their cap,
 * ties to the lower UE index. Among integer vectors with the same sum and
 * bounds this minimises sum (a_e - x_e)^2. */
void oracle_largest_remainder(int32_t E, const double* x, const int32_t* R, int64_t T, int32_t* a)
{
    int64_t fsum = 0;
    for (int32_t e = 0; e < E; ++e) {
        a[e] = (int32_t)floor(x[e]);
        fsum += a[e];
    }
    int64_t r = T - fsum;
    int picked[MAX_UE];
    for (int32_t e = 0; e < E; ++e)
        picked[e] = 0;
    for (int64_t n = 0; n < r; ++n) {
        int32_t best = -1;
        double best_frac = -1.0;
        for (int32_t e = 0; e < E; ++e) {
            if (picked[e] || a[e] >= R[e])
                continue;
            double frac = x[e] - floor(x[e]);
            if (frac > best_frac) { /* strict: equal fractions keep the lower index */
                best = e;
                best_frac = frac;
            }
        }
        if (best < 0)
            break;
        picked[best] = 1;
        a[best] += 1;
    }
}

/* Huntington-Hill apportionment of T units (the paper's rounding, Sec. IV-B,
 * after Balinski and Young), in its priority form: units are handed out one at
 * a time, each to the UE with the largest priority x_e / sqrt(n_e (n_e + 1)),
 * n_e being the units it already holds; a UE's first unit has infinite
 * priority, a UE at its cap R_e takes no more, and a UE with x_e = 0 takes
 * none. Equal priorities go to the larger share, then to the lower index. When
 * T is smaller than the number of positive shares (no Huntington-Hill
 * allocation exists then, as every positive share is owed a unit), the same
 * rule gives one unit to each of the T largest shares. */
void oracle_huntington_hill(int32_t E, const double* x, const int32_t* R, int64_t T, int32_t* a)
{
    for (int32_t e = 0; e < E; ++e)
        a[e] = 0;
    for (int64_t n = 0; n < T; ++n) {
        int32_t best = -1;
        double best_pr = 0.0;
        for (int32_t e = 0; e < E; ++e) {
            if (!(x[e] > 0.0) || a[e] >= R[e])
                continue;
            const double pr = a[e] == 0 ? INFINITY : x[e] / sqrt((double)a[e] * (double)(a[e] + 1));
            /* strict comparisons keep the lower index among full ties */
            if (best < 0 || pr > best_pr || (pr == best_pr && x[e] > x[best])) {
                best = e;
                best_pr = pr;
            }
        }
        if (best < 0)
            break;
        a[best] += 1;
    }
}

/* Float64 decision margin of Huntington-Hill, in the max norm over the shares
 * (each kept in [0, R_e], the range of the capped split): no share vector
 * closer to x than this in every component yields another allocation, and
 * some move of two shares by a little more does. Every decision compares unit
 * priorities x_e / g(n) with g(n) = sqrt(n (n+1)); they move with x
 * continuously, and a UE at its cap is excluded whatever the shares, so the
 * capped split switching a UE between capped and uncapped changes nothing.
 * What can flip:
 * - a held unit (the a_i-th of UE i) and a withheld one (the (a_j+1)-th of
 *   UE j) swapping priority. Moving x_i down and x_j up by d, the priorities
 *   meet at d = (pr_i - pr_j) / (1/g_i + 1/g_j); if x_j would pass its cap
 *   first, x_j stops at R_j and x_i alone closes the rest, d = x_i - g_i R_j / g_j;
 * - two first units (infinite priorities, ordered by the shares), the same
 *   with g = 1 on both sides;
 * - a held unit lost when its share reaches zero (a positive share is owed
 *   its first unit, a zero share none). */
double oracle_margin_hh(int32_t E, const double* x, const int32_t* R, int64_t T, const int32_t* a)
{
    int64_t rsum = 0;
    for (int32_t e = 0; e < E; ++e)
        rsum += R[e];
    if (T <= 0 || T >= rsum)
        return INFINITY;
    double m = INFINITY;
    for (int32_t i = 0; i < E; ++i) {
        if (a[i] < 1)
            continue;
        if (x[i] < m) /* a first unit is owed only to a positive share */
            m = x[i];
        const double gi = sqrt((double)(a[i] - 1) * (double)a[i]); /* last held unit */
        for (int32_t j = 0; j < E; ++j) {
            if (j == i || !(x[j] > 0.0) || a[j] >= R[j])
                continue;
            const double gj = sqrt((double)a[j] * (double)(a[j] + 1)); /* next withheld unit */
            double hi = gi, hj = gj;
            if (gi == 0.0 && gj == 0.0) {
                hi = hj = 1.0; /* two first units: ordered by the shares */
            } else if (gi == 0.0) {
                continue; /* an infinite priority never loses to a finite one */
            } else if (gj == 0.0) {
                m = 0.0; /* a withheld first unit behind a held later one: not a Huntington-Hill result */
                continue;
            }
            double d = (x[i] / hi - x[j] / hj) / (1.0 / hi + 1.0 / hj);
            if (x[j] + d > (double)R[j])
                d = x[i] - hi * (double)R[j] / hj;
            if (d < m)
                m = d;
        }
    }
    return m < 0.0 ? 0.0 : m;
}

/* Float64 decision margin of largest remainder, in the max norm over the
 * shares: no share vector (each share kept in [0, R_e]) closer to x than this
 * in every component rounds to another allocation.
 * Largest remainder gives floor(x_e) plus one unit to the r = T - sum floor(x)
 * eligible UEs (floor below the cap) with the largest remainders. That is
 * the same as rounding every x_e - theta up (and capping at R_e) for any
 * threshold theta strictly between the r-th and (r+1)-th largest eligible
 * remainders, at which the rounded values sum to T. At the midpoint threshold
 * every x_e - theta, including a capped R_e - theta, lies at least half that
 * gap from an integer, so a shift of each share by less than half the gap
 * rounds the same way; moving the r-th UE down and the (r+1)-th up by a
 * little more swaps them. A share crossing an integer or reaching its cap
 * flips nothing by itself: its remainder wraps between the top and the bottom
 * of the order while r changes by one, and the same units are handed out.
 * With r = 0 every share is an integer and any threshold in [0, 1) works: the
 * margin is 1/2, exact when one share can give up a unit and another can take
 * one (a lower bound otherwise). INFINITY when nothing can flip (T = 0, or T >= sum R: every
 * UE at its cap). */
double oracle_margin(int32_t E, const double* x, const int32_t* R, int64_t T)
{
    int64_t rsum = 0;
    for (int32_t e = 0; e < E; ++e)
        rsum += R[e];
    if (T <= 0 || T >= rsum)
        return INFINITY;
    double rem[MAX_UE];
    int64_t fsum = 0;
    int32_t n = 0;
    for (int32_t e = 0; e < E; ++e) {
        const double f = floor(x[e]);
        fsum += (int64_t)f;
        if (f < (double)R[e]) /* eligible for one more unit */
            rem[n++] = x[e] - f;
    }
    const int64_t r = T - fsum;
    if (r == 0)
        return 0.5;
    if (r < 0 || r >= n)
        return 0.0; /* cannot happen for shares that sum to T within their caps */
    for (int32_t i = 1; i < n; ++i) { /* insertion sort, descending */
        const double v = rem[i];
        int32_t j = i - 1;
        while (j >= 0 && rem[j] < v) {
            rem[j + 1] = rem[j];
            --j;
        }
        rem[j + 1] = v;
    }
    return 0.5 * (rem[r - 1] - rem[r]);
}

/* From logits to the integer puncturing vector of one node with largest
 * remainder rounding (see oracle_allocate_rounding). Returns the margin. */
double oracle_allocate_rounding(int32_t E, const double* z, const int32_t* R, int32_t U, int32_t k, int32_t rounding,
                                int32_t* a, double* x_out);

double oracle_allocate(int32_t E, const double* z, const int32_t* R, int32_t U, int32_t k, int32_t* a,
                       double* x_out)
{
    return oracle_allocate_rounding(E, z, R, U, k, ORACLE_LARGEST_REMAINDER, a, x_out);
}

/* The enforcer of one node (Sec. IV-B): softmax, the capped proportional split
 * of T = min(U k, sum R) (Eq. (7)), then the integer step (largest remainder,
 * or Huntington-Hill). Returns the decision margin. */
double oracle_allocate_rounding(int32_t E, const double* z, const int32_t* R, int32_t U, int32_t k, int32_t rounding,
                                int32_t* a, double* x_out)
{
    double p[MAX_UE], x[MAX_UE];
    int64_t rsum = 0;
    for (int32_t e = 0; e < E; ++e)
        rsum += R[e];
    int64_t demand = (int64_t)U * k;
    int64_t T = demand < rsum ? demand : rsum;
    oracle_softmax(E, z, p);
    oracle_capped_scale(E, p, R, T, x);
    if (rounding == ORACLE_HUNTINGTON_HILL)
        oracle_huntington_hill(E, x, R, T, a);
    else
        oracle_largest_remainder(E, x, R, T, a);
    if (x_out)
        for (int32_t e = 0; e < E; ++e)
            x_out[e] = x[e];
    if (rounding == ORACLE_HUNTINGTON_HILL)
        return oracle_margin_hh(E, x, R, T, a);
    return oracle_margin(E, x, R, T);
}

/* ----------------------------------------------------------- tree / Alg. 2 */

static int check_inputs(const oracle_tree* t, const oracle_actor* f)
{
    if (!t || !f)
        return ORACLE_EINVAL;
    if (t->num_ue < 1 || t->num_ue > MAX_UE / 2 || t->max_arrival < 1 || t->num_minislots < 1 ||
        t->rb_per_unit < 0 || t->rounding < ORACLE_LARGEST_REMAINDER || t->rounding > ORACLE_HUNTINGTON_HILL ||
        t->head < ORACLE_SOFTMAX_HEAD || t->head > ORACLE_GAUSSIAN_HEAD)
        return ORACLE_EINVAL;
    const int32_t n_out = t->head == ORACLE_GAUSSIAN_HEAD ? 2 * t->num_ue : t->num_ue;
    if (f->dims[0] != 4 * t->num_ue + 2 || f->dims[f->num_layers] != n_out)
        return ORACLE_EINVAL;
    return ORACLE_OK;
}

/* One evaluated node: features, actor, enforcer. */
static int eval_node(const oracle_tree* t, const oracle_actor* f, const int32_t* rb, const int32_t* mcs,
                     const float* sinr, const int32_t* c_in, int64_t node, int32_t tau, int32_t k, int32_t* a,
                     double* z, double* margin, double* amax)
{
    double x[4 * MAX_UE + 2], out[MAX_UE];
    oracle_features(t->num_ue, rb, mcs, sinr, c_in, tau, k, x);
    int rc = oracle_mlp(f, x, out, amax);
    if (rc)
        return rc;
    if (t->head == ORACLE_GAUSSIAN_HEAD)
        oracle_gaussian_head(t->num_ue, out, t->seed, t->tti, node, z);
    else
        for (int32_t e = 0; e < t->num_ue; ++e)
            z[e] = out[e];
    double m = oracle_allocate_rounding(t->num_ue, z, rb, t->rb_per_unit, k, t->rounding, a, NULL);
    if (margin)
        *margin = m;
    return ORACLE_OK;
}

/* Free-running build of the whole codebook tree (Alg. 2 for every arrival
 * prefix). alloc: [nodes][E] bytes. logits: [nodes][E] or NULL. margin:
 * [nodes] or NULL. The root and k = 0 nodes hold a zero allocation, zero
 * logits and an infinite margin. */
int oracle_build_tree(const oracle_tree* t, const oracle_actor* f, const int32_t* rb, const int32_t* mcs,
                      const float* sinr, uint8_t* alloc, double* logits, double* margin)
{
    int rc = check_inputs(t, f);
    if (rc)
        return rc;
    const int32_t E = t->num_ue, K = t->max_arrival;
    const int64_t nodes = oracle_num_nodes(K, t->num_minislots);
    int32_t* state = (int32_t*)calloc((size_t)nodes * E, sizeof(int32_t)); /* c_in + a per node */
    if (!state)
        return ORACLE_ENOMEM;
    memset(alloc, 0, (size_t)nodes * E);
    if (logits)
        memset(logits, 0, sizeof(double) * (size_t)nodes * E);
    if (margin)
        margin[0] = INFINITY;
    for (int32_t tau = 1; tau <= t->num_minislots && rc == ORACLE_OK; ++tau) {
        const int64_t off = oracle_level_offset(K, tau), poff = oracle_level_offset(K, tau - 1);
        const int64_t width = ipow64(K + 1, tau);
        for (int64_t i = 0; i < width; ++i) {
            const int64_t node = off + i, parent = poff + i / (K + 1);
            const int32_t k = (int32_t)(i % (K + 1));
            const int32_t* c_in = state + parent * E;
            int32_t a[MAX_UE] = {0};
            double z[MAX_UE] = {0}, m = INFINITY;
            if (k > 0) {
                rc = eval_node(t, f, rb, mcs, sinr, c_in, node, tau, k, a, z, &m, NULL);
                if (rc)
                    break;
            }
            for (int32_t e = 0; e < E; ++e) {
                alloc[node * E + e] = (uint8_t)a[e];
                state[node * E + e] = c_in[e] + a[e];
                if (logits)
                    logits[node * E + e] = z[e];
            }
            if (margin)
                margin[node] = m;
        }
    }
    free(state);
    return rc;
}

/* Conditioned evaluation: each listed node is recomputed from the state its
 * ancestors reach under a GIVEN codebook (for instance one produced
 * elsewhere), so a disagreement in a parent cannot spread to its children.
 * given: [nodes][E]. out_alloc: [n][E]. out_logits: [n][E] or NULL.
 * out_margin: [n] or NULL. */
int oracle_eval_conditioned(const oracle_tree* t, const oracle_actor* f, const int32_t* rb,
                            const int32_t* mcs, const float* sinr, const uint8_t* given,
                            const int64_t* node_ids, int64_t n, int32_t* out_alloc, double* out_logits,
                            double* out_margin)
{
    int rc = check_inputs(t, f);
    if (rc)
        return rc;
    const int32_t E = t->num_ue, K = t->max_arrival;
    const int64_t nodes = oracle_num_nodes(K, t->num_minislots);
    for (int64_t j = 0; j < n; ++j) {
        int64_t node = node_ids[j];
        if (node < 0 || node >= nodes)
            return ORACLE_EINVAL;
        int32_t tau = 0;
        while (oracle_level_offset(K, tau + 1) <= node)
            ++tau;
        int32_t a[MAX_UE] = {0}, c_in[MAX_UE] = {0};
        double z[MAX_UE] = {0}, m = INFINITY;
        if (tau > 0) {
            int64_t i = node - oracle_level_offset(K, tau);
            int32_t k = (int32_t)(i % (K + 1));
            /* walk up: c_in is the sum of the given allocations of the
             * strict ancestors */
            int64_t anc_i = i / (K + 1);
            for (int32_t lev = tau - 1; lev >= 1; --lev) {
                const uint8_t* g = given + (oracle_level_offset(K, lev) + anc_i) * E;
                for (int32_t e = 0; e < E; ++e)
                    c_in[e] += g[e];
                anc_i /= (K + 1);
            }
            if (k > 0) {
                rc = eval_node(t, f, rb, mcs, sinr, c_in, node, tau, k, a, z, &m, NULL);
                if (rc)
                    return rc;
            }
        }
        for (int32_t e = 0; e < E; ++e) {
            out_alloc[j * E + e] = a[e];
            if (out_logits)
                out_logits[j * E + e] = z[e];
        }
        if (out_margin)
            out_margin[j] = m;
    }
    return ORACLE_OK;
}

/* Sequential roll-out of one arrival sequence k_1..k_len, as the O-RU would
 * experience it mini-slot by mini-slot (Alg. 3): the state starts at zero and
 * accumulates the chosen vector after every mini-slot. out: [len][E]. amax, if
 * not NULL, collects the largest |input| seen by each actor layer. */
int oracle_rollout(const oracle_tree* t, const oracle_actor* f, const int32_t* rb, const int32_t* mcs,
                   const float* sinr, const int32_t* seq, int32_t len, int32_t* out, double* amax)
{
    int rc = check_inputs(t, f);
    if (rc)
        return rc;
    const int32_t E = t->num_ue, K = t->max_arrival;
    int32_t c[MAX_UE] = {0};
    int64_t i = 0; /* index of the current node within its level */
    for (int32_t tau = 1; tau <= len; ++tau) {
        int32_t k = seq[tau - 1];
        if (k < 0 || k > K)
            return ORACLE_EINVAL;
        i = i * (K + 1) + k;
        int32_t a[MAX_UE] = {0};
        if (k > 0) {
            double z[MAX_UE];
            rc = eval_node(t, f, rb, mcs, sinr, c, oracle_level_offset(K, tau) + i, tau, k, a, z, NULL, amax);
            if (rc)
                return rc;
        }
        for (int32_t e = 0; e < E; ++e) {
            out[(tau - 1) * E + e] = a[e];
            c[e] += a[e];
        }
    }
    return ORACLE_OK;
}

/* O-RU side of one slot (the controller of the simulator, Sec. III-A and
 * Sec. VI-A, then Alg. 3): at most K packets are punctured in a mini-slot and
 * the rest wait for the next one, so the served count is
 * k_tau = min(K, a_tau + q_{tau-1}) with backlog q_tau = a_tau + q_{tau-1} - k_tau
 * (q_0 = carry_in). The puncturing vector of mini-slot tau is the codebook
 * entry of the served prefix, here obtained by a sequential roll-out.
 * raw: [len] arrivals; served: [len]; y: [len][E]; *carry_out = q_len. */
int oracle_oru_assemble(const oracle_tree* t, const oracle_actor* f, const int32_t* rb, const int32_t* mcs,
                        const float* sinr, const int32_t* raw, int32_t len, int32_t carry_in, int32_t* served,
                        int32_t* y, int32_t* carry_out)
{
    if (!t || len < 0 || len > t->num_minislots || carry_in < 0)
        return ORACLE_EINVAL;
    int32_t q = carry_in;
    for (int32_t tau = 0; tau < len; ++tau) {
        if (raw[tau] < 0)
            return ORACLE_EINVAL;
        int32_t want = raw[tau] + q;
        served[tau] = want < t->max_arrival ? want : t->max_arrival;
        q = want - served[tau];
    }
    *carry_out = q;
    return oracle_rollout(t, f, rb, mcs, sinr, served, len, y, NULL);
}

/* ------------------------------------------------------------ critic (RIC) */

typedef struct {
    int32_t num_ue;        /* E */
    int32_t num_minislots; /* M, steps per sample */
    int32_t num_samples;   /* H */
    double discount;       /* lambda of Eq. (4) */
    double entropy_coef;   /* zeta of Eq. (4) */
} oracle_critic_cfg;

/* Critic input at step tau of sample h: the actor's state features
 * (oracle_features with the carried state c and arrivals k of that step)
 * followed by the action y, dimension 5E+2. */
static void critic_input(int32_t E, const int32_t* ue_h, const uint8_t* c_step, int32_t tau, int32_t k,
                         const double* y, double* x)
{
    int32_t rb[MAX_UE] = {0}, mcs[MAX_UE] = {0}, c[MAX_UE] = {0};
    float sinr[MAX_UE] = {0};
    for (int32_t e = 0; e < E; ++e) {
        rb[e] = ue_h[e];
        mcs[e] = ue_h[E + e];
        memcpy(&sinr[e], &ue_h[2 * E + e], 4);
        c[e] = c_step[e];
    }
    oracle_features(E, rb, mcs, sinr, c, tau, k, x);
    for (int32_t e = 0; e < E; ++e)
        x[4 * E + 2 + e] = y[e];
}

/* The Near-RT RIC's critic pass over H buffer samples of M steps (Sec. IV-B):
 *   q[i][h][tau]  = Q_i([s, c, tau, k], y) for the stored action y (Eq. (3));
 *   qhat[h][tau]  = Eq. (4): for tau < M, lambda (min_i Qtarg_i(state of step
 *                   tau+1, y~) - zeta log pi(y~)), y~ a fresh action of the
 *                   actor at step tau+1 (the Gaussian head's draws, counter
 *                   node = h M + tau, TTI = episode); when no packet arrives
 *                   at tau+1 the policy does not act (y~ = 0, log pi = 0);
 *                   at tau = M the slot's reward r_h;
 *   loss[i]       = (1 / (H M)) sum_h sum_tau (q[i][h][tau] - qhat[h][tau])^2.
 * Layouts: ue [H][3E] (rb, mcs, sinr bits), k [H][M], c [H][M][E] (punctured
 * RBs carried into the step), y [H][M][E], r [H]; q [2][H][M]; qhat and
 * logpi (optional) [H][M]. */
int oracle_critic_evaluate(const oracle_critic_cfg* cfg, const oracle_actor* actor, const oracle_actor* q1,
                           const oracle_actor* q2, const oracle_actor* qt1, const oracle_actor* qt2,
                           const int32_t* ue, const int32_t* k, const uint8_t* c, const float* y, const float* r,
                           uint64_t seed, uint64_t episode, double* q, double* qhat, double* logpi, double* loss)
{
    if (!cfg || cfg->num_ue < 1 || cfg->num_ue > MAX_UE / 2 || cfg->num_minislots < 1 || cfg->num_samples < 1)
        return ORACLE_EINVAL;
    const int32_t E = cfg->num_ue, M = cfg->num_minislots, H = cfg->num_samples;
    const oracle_actor* crit[2] = {q1, q2};
    const oracle_actor* targ[2] = {qt1, qt2};
    for (int i = 0; i < 2; ++i)
        if (crit[i]->dims[0] != 5 * E + 2 || crit[i]->dims[crit[i]->num_layers] != 1 ||
            targ[i]->dims[0] != 5 * E + 2 || targ[i]->dims[targ[i]->num_layers] != 1)
            return ORACLE_EINVAL;
    if (actor->dims[0] != 4 * E + 2 || actor->dims[actor->num_layers] != 2 * E)
        return ORACLE_EINVAL;
    double sq[2] = {0.0, 0.0};
    for (int32_t h = 0; h < H; ++h) {
        const int32_t* ue_h = ue + (int64_t)h * 3 * E;
        for (int32_t tau = 1; tau <= M; ++tau) {
            const int64_t row = (int64_t)h * M + (tau - 1);
            double x[5 * MAX_UE + 2], yv[MAX_UE], out[MAX_UE], qv;
            for (int32_t e = 0; e < E; ++e)
                yv[e] = y[row * E + e];
            critic_input(E, ue_h, c + row * E, tau, k[row], yv, x);
            for (int i = 0; i < 2; ++i) {
                int rc = oracle_mlp(crit[i], x, &qv, NULL);
                if (rc)
                    return rc;
                q[(int64_t)i * H * M + row] = qv;
            }
            double target, lp = 0.0;
            if (tau == M) {
                target = r[h];
            } else {
                const int64_t nrow = row + 1; /* step tau + 1 of the same sample */
                const int32_t kn = k[nrow];
                double yt[MAX_UE];
                for (int32_t e = 0; e < E; ++e)
                    yt[e] = 0.0;
                if (kn > 0) {
                    double xa[4 * MAX_UE + 2];
                    critic_input(E, ue_h, c + nrow * E, tau + 1, kn, yt, x); /* features only, y unused */
                    for (int32_t j = 0; j < 4 * E + 2; ++j)
                        xa[j] = x[j];
                    int rc = oracle_mlp(actor, xa, out, NULL);
                    if (rc)
                        return rc;
                    lp = oracle_sample_tanh_gaussian(E, out, seed, episode, nrow, yt);
                }
                critic_input(E, ue_h, c + nrow * E, tau + 1, kn, yt, x);
                double qt[2];
                for (int i = 0; i < 2; ++i) {
                    int rc = oracle_mlp(targ[i], x, &qt[i], NULL);
                    if (rc)
                        return rc;
                }
                target = cfg->discount * ((qt[0] < qt[1] ? qt[0] : qt[1]) - cfg->entropy_coef * lp);
            }
            qhat[row] = target;
            if (logpi)
                logpi[row] = lp;
            for (int i = 0; i < 2; ++i) {
                const double d = q[(int64_t)i * H * M + row] - target;
                sq[i] += d * d;
            }
        }
    }
    for (int i = 0; i < 2; ++i)
        loss[i] = sq[i] / ((double)H * M);
    return ORACLE_OK;
}
