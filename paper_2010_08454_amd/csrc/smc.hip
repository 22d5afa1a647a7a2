// smc.hip -- sequential Monte Carlo in one persistent cooperative launch.
//
// The paper suspends a model at each factor with a delimited continuation
// (Sec. 3.4, 4.3) and names particle-based inference on the GPU as future work
// (Sec. 6).  Here a suspended particle is its resume point (the factor index s,
// shared by all particles) plus fixed-size state held in registers across the
// whole run; only resampling moves state through device memory.
//
// One workgroup of 512 threads per CU, P particles per thread (slots
// j = block * 512 P + thread * P + p; a block's slots form one "tile").
// 512 threads leave each wave 256 registers, so the particle state, the
// resampling variables and the FP64 normaliser calls fit without spilling
// (spilled registers would be written back and refetched through HBM at
// every grid barrier).
// Per factor s:
//   1. every particle advances to factor s and adds its log-factor (FP32,
//      compensated summation);
//   2. block partial {max lw, sum e, sum e^2}, e = exp(lw - max) -> memory;
//      grid barrier; every block merges the partials in the same order, so
//      every block takes the same ESS decision;
//   3. if ESS < ess_frac N (and s is not the last factor): FP64 weights
//      e = exp(lw - max) give the epoch normaliser and the quantised integer
//      weights q; each block scans its q and publishes its tile total, its
//      tile-local exclusive prefix sums and its particles' state; grid barrier; each
//      block finds the contiguous ancestor range of its slots, stages those
//      prefix sums in LDS, and every slot binary-searches its ancestor there
//      and gathers the ancestor's state; lw = 0.
// Blocks meet at a record barrier: each block stores its record (the partial
// of step 2, the tile total of step 3, the final sums) on its own cache line
// and thread t of every block polls line t, so every block holds every record
// when it leaves, with no shared counter.  Every word a block publishes for
// others (record words, the prefix sums and state of step 3) carries the tag
// of its epoch or event, so a reader knows it has the current value without
// any release or acquire, and a reader that is early polls again.  The spin
// is bounded: if a wait exceeds the limit, the block raises the abort flag
// and every block leaves its loop at its next barrier, so the grid always
// drains.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "device.h"
#include "host.h"
#include "smc.h"
#include "timing.h"

namespace ppl {

constexpr int kSmcThreads = 512;
constexpr int kSmcWaves = kSmcThreads / 64;
constexpr int kSmcMaxBlocks = 1024;
constexpr int kBarLine = 32;                  // unsigned per 128-byte line
constexpr int kBarWords = kBarLine;           // word 1: abort flag
constexpr int kRecWords = 16;                 // 64-bit words per 128-byte record line
constexpr uint32_t kSpinLimit = 1u << 24;     // polls before a wait is declared hung (seconds)
constexpr int kYChunk = 2048;                 // observations staged in LDS at a time
constexpr int kStage = 8192;                  // most prefix sums staged in LDS for the ancestor search

struct SmcDev {
    const float *y;
    int64_t T, N;
    int K;
    Key key;
    uint32_t inst;
    float ess_frac;
    float hyp[5];            // model constants (FP32)
    double lconst;           // LGSSM: -1/2 log(2 pi r^2) ; GMM: -1/2 log(2 pi) - log(sd)
    int kbits;               // quantisation exponent
    int stage_cap;           // prefix sums that fit in the LDS stage
    // outputs (may be null)
    double *scalars;
    float *lw_out, *lat_out;
    double *ess_trace;
    uint8_t *resampled;
    int32_t *anc_out;
    float *elw_out;          // [max_events][N] log-weights each event resampled from
    double *logz_tr;         // [T] normaliser increment added after factor s
    double *alpha_out;       // [max_events][move_steps][N] log acceptance ratios of the moves
    int64_t max_events;
    int64_t t0, t1;          // factors of this launch [t0, t1)
    char *ckpt;              // checkpoint: header then [NF][N] state, [N] lw, [N] compensation
    int move_steps;          // resample-move steps per particle after each resampling
    double move_lam;         // random-walk scale factor
    double hyp64[2];         // GMM {mu_sd, comp_sd} in FP64 (move scales)
    int poll_all;            // 1: every tagged read takes the polling path (a checking aid)
    // workspace
    unsigned *bar;           // [1] abort flag
    uint64_t *rec;           // [2][nb][16] record lines: word 0 the epoch, words 1..3 the record
    uint64_t *qtag;          // [N] tagged tile-local exclusive prefix sums of q
    uint64_t *xtag;          // [NF][N] tagged particle state
    float *xbuf2;            // [NF][N] gathered particles while they move (resample-move)
};

// Checkpoint header (the first 256 bytes of a checkpoint).
struct SmcCkpt {
    int64_t t;               // next factor
    int64_t N;
    int64_t nres;
    int32_t nf;
    int32_t status;
    double logz;
    float mlast;
};
constexpr size_t kCkptHeader = 256;

// ------------------------------------------------------------- barrier --
// Record exchange for epoch e (a grid barrier that also hands every block
// every block's record): thread 0 stores NW words on its line of buffer
// e mod 2 with relaxed device-scope stores, each word holding e in its high
// half and 32 bits of the record in its low half; thread t < nb polls line t
// (its last word first) until every word of the line holds e.  Each word
// validates itself, so the exchange needs no release and no acquire (a
// device-scope release writes back the L2 of the issuing XCD, which at 256
// workgroups costs more than the exchange itself).  Two buffers suffice: a
// block cannot store record e + 2 before every block has stored record e + 1,
// which each does only after reading all records e.  Returns false
// (uniformly in the block) once any block has aborted.
template <int NW>
__device__ __forceinline__ bool tagged_barrier(uint64_t *rec, unsigned *bar, unsigned epoch, int nb,
                                               const uint32_t (&w)[NW], uint32_t (&r)[NW]) {
    static_assert(NW <= kRecWords, "record line overflow");
    __shared__ int s_bad;
    unsigned *abort_flag = bar + 1;
    uint64_t *buf = rec + (size_t)(epoch & 1u) * nb * kRecWords;
    const uint64_t tag = (uint64_t)epoch << 32;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t *mine = buf + (size_t)blockIdx.x * kRecWords;
#pragma unroll
        for (int k = 0; k < NW; ++k) __hip_atomic_store(mine + k, tag | w[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int k = 0; k < NW; ++k) r[k] = 0;
    if (threadIdx.x < nb) {          // nb <= kSmcThreads
        uint64_t *line = buf + (size_t)threadIdx.x * kRecWords;
        uint32_t spins = 0;
        while (true) {
            const uint64_t last = __hip_atomic_load(line + NW - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((last >> 32) == (uint64_t)epoch) {
                uint64_t v[NW];
                bool all = true;
#pragma unroll
                for (int k = 0; k < NW - 1; ++k) {
                    v[k] = __hip_atomic_load(line + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    all = all && (v[k] >> 32) == (uint64_t)epoch;
                }
                v[NW - 1] = last;
                if (all) {
#pragma unroll
                    for (int k = 0; k < NW; ++k) r[k] = (uint32_t)v[k];
                    break;
                }
            }
            __builtin_amdgcn_s_sleep(1);
            if ((++spins & 63) == 0) {
                if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { s_bad = 1; break; }
                if (spins > kSpinLimit) {
                    __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_bad = 1;
                    break;
                }
            }
        }
    }
    __syncthreads();
    return s_bad == 0;
}

__device__ __forceinline__ uint32_t hi32(double v) { return (uint32_t)((uint64_t)__double_as_longlong(v) >> 32); }
__device__ __forceinline__ uint32_t lo32(double v) { return (uint32_t)(uint64_t)__double_as_longlong(v); }
__device__ __forceinline__ double from32(uint32_t hi, uint32_t lo) {
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}


// --------------------------------------------------------------- models --
struct Lgssm {
    static constexpr int NF = 1;
    // hyp = {a, q_sd, r_sd, m0, p0_sd}
    __device__ static void init(const SmcDev &a, uint32_t j, float st[NF]) {
        float x = a.hyp[3];
        if (a.hyp[4] != 0.0f) {
            float z[4];
            normals4(philox(j, 1, 0, (a.inst << 8) | kTagPrior, a.key), z);
            x = fmaf(a.hyp[4], z[0], x);
        }
        st[0] = x;
    }
    // Noise of slot j at factor s is normal (s mod 4) of block (j, 0, s div 4):
    // the first or second Box-Muller pair of the block, recomputed at every
    // factor (keeping the block's four normals across factors costs four
    // registers per particle, and the kernel would spill).
    __device__ static float step(const SmcDev &a, int64_t s, uint32_t j, float st[NF], float ys) {
        const uint4 w = philox(j, 0, (uint32_t)(s >> 2), (a.inst << 8) | kTagPrior, a.key);
        float z0, z1;
        if (s & 2) box_muller(unit_f32(w.z), unit_f32(w.w), z0, z1);
        else box_muller(unit_f32(w.x), unit_f32(w.y), z0, z1);
        const float x = fmaf(a.hyp[0], st[0], a.hyp[1] * ((s & 1) ? z1 : z0));
        st[0] = x;
        const float r = (ys - x) / a.hyp[2];
        return (float)a.lconst - 0.5f * r * r;
    }
};

template <int K>
struct Gmm {
    static constexpr int NF = 2 * K;
    // hyp = {mu_sd, comp_sd}; state = {log pi_0..K-1, mu_0..K-1}
    __device__ static void init(const SmcDev &a, uint32_t j, float st[NF]) {
        const uint32_t c3 = (a.inst << 8) | kTagPrior;
        const uint4 w0 = philox(j, 0, 0, c3, a.key), w1 = philox(j, 1, 0, c3, a.key);
        const uint32_t w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
        float E[K], tot = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            E[k] = -logf(unit_f32(w[k]));
            tot += E[k];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) st[k] = logf(E[k] / tot);
        float z[8];
        normals4(philox(j, 2, 0, c3, a.key), z);
        normals4(philox(j, 3, 0, c3, a.key), z + 4);
#pragma unroll
        for (int k = 0; k < K; ++k) st[K + k] = a.hyp[0] * z[k];
    }
    __device__ static float step(const SmcDev &a, int64_t, uint32_t, float st[NF], float ys) {
        const float inv = 1.0f / a.hyp[1];
        float t[K], mx = -INFINITY;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float r = (ys - st[K + k]) * inv;
            t[k] = fmaf(-0.5f * r, r, st[k]);
            mx = fmaxf(mx, t[k]);
        }
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) s += expf(t[k] - mx);
        return (float)a.lconst + mx + logf(s);
    }
};

// ------------------------------------------------------- resample-move --
// After each resampling at factor s a mixture particle takes move_steps
// Metropolis-Hastings steps whose target is the posterior given y_0..y_s
// (particle inference of Sec. 6 with the acceptance rule of the paper's
// Metropolis-Hastings method, Sec. 3.6.3).  Coordinates u = (log pi_k -
// log pi_K for k < K, mu_k); prior density Dirichlet(1) (the softmax
// Jacobian sum_k log pi_k) times Normal(0, mu_sd) per mean; symmetric Gaussian
// random walk u' = u + h z with
//   h_mu = lam / sqrt(1/mu_sd^2 + (s+1)/(K comp_sd^2)),
//   h_b  = lam / sqrt(3/pi^2 + (s+1)/(2K)),
// accepted when log v < log alpha (FP64).  Move m of slot j draws sixteen
// normals from Philox blocks (j, 8m + b, s, inst << 8 | 7), b < 4, and v
// from word 0 of block 8m + 4.  The log-likelihood of y_0..y_s sums the
// model's FP32 factor within blocks of 16 data and in FP64 across blocks.
template <int K>
__device__ double gmm_loglik_upto(const SmcDev &a, int64_t s, const float st[2 * K]) {
    double tot = 0.0;
    float blk = 0.0f;
    int c = 0;
    for (int64_t d = 0; d <= s; ++d) {
        blk += Gmm<K>::step(a, d, 0, const_cast<float *>(st), a.y[d]);
        if (++c == 16) {
            tot += (double)blk;
            blk = 0.0f;
            c = 0;
        }
    }
    return tot + (double)blk;
}

template <int K>
__device__ __forceinline__ double gmm_log_prior(const float st[2 * K], float inv_mu_sd) {
    double l = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float r = st[K + k] * inv_mu_sd;
        l += (double)st[k] - 0.5 * (double)(r * r);
    }
    return l;
}

// One particle's moves; its state is read from and written back to g[f * stride].
template <int K>
__device__ void gmm_move(const SmcDev &a, int64_t s, uint32_t j, float *g, size_t stride,
                                      double *alpha_row, int64_t N) {
    float st[2 * K];
#pragma unroll
    for (int f = 0; f < 2 * K; ++f) st[f] = g[f * stride];
    const double n = (double)(s + 1);
    const float h_mu = (float)(a.move_lam / sqrt(1.0 / (a.hyp64[0] * a.hyp64[0]) +
                                                n / ((double)K * a.hyp64[1] * a.hyp64[1])));
    const float h_b = (float)(a.move_lam / sqrt(3.0 / (M_PI * M_PI) + n / (2.0 * K)));
    const float inv_mu_sd = 1.0f / a.hyp[0];
    const uint32_t c3 = (a.inst << 8) | kTagMove;
    double ll = gmm_loglik_upto<K>(a, s, st);
    double lp = gmm_log_prior<K>(st, inv_mu_sd);
    for (int m = 0; m < a.move_steps; ++m) {
        float z[16];
#pragma unroll
        for (int b = 0; b < 4; ++b) normals4(philox(j, (uint32_t)(8 * m + b), (uint32_t)s, c3, a.key), z + 4 * b);
        const float v = unit_f32(philox(j, (uint32_t)(8 * m + 4), (uint32_t)s, c3, a.key).x);
        float st2[2 * K];
        float mx = 0.0f;
#pragma unroll
        for (int k = 0; k < K - 1; ++k) {
            st2[k] = fmaf(h_b, z[k], st[k] - st[K - 1]);
            mx = fmaxf(mx, st2[k]);
        }
        float se = expf(-mx);
#pragma unroll
        for (int k = 0; k < K - 1; ++k) se += expf(st2[k] - mx);
        const float lse = mx + logf(se);
#pragma unroll
        for (int k = 0; k < K - 1; ++k) st2[k] -= lse;
        st2[K - 1] = -lse;
#pragma unroll
        for (int k = 0; k < K; ++k) st2[K + k] = fmaf(h_mu, z[K - 1 + k], st[K + k]);
        const double ll2 = gmm_loglik_upto<K>(a, s, st2);
        const double lp2 = gmm_log_prior<K>(st2, inv_mu_sd);
        const double la = (ll2 + lp2) - (ll + lp);
        if (alpha_row) alpha_row[(size_t)m * N + j] = la;
        if (log((double)v) < la) {
#pragma unroll
            for (int k = 0; k < 2 * K; ++k) st[k] = st2[k];
            ll = ll2;
            lp = lp2;
        }
    }
#pragma unroll
    for (int f = 0; f < 2 * K; ++f) g[f * stride] = st[f];
}

template <class M>
struct MoveOf {
    __device__ static void run(const SmcDev &, int64_t, uint32_t, float *, size_t, double *, int64_t) {}
};
template <int K>
struct MoveOf<Gmm<K>> {
    __device__ static void run(const SmcDev &a, int64_t s, uint32_t j, float *g, size_t stride, double *alpha_row,
                               int64_t N) {
        gmm_move<K>(a, s, j, g, stride, alpha_row, N);
    }
};

// FP64 log/exp kept out of line: inlined, their polynomial constants get hoisted
// out of the factor loop and occupy registers for the whole run.
__device__ __noinline__ double log_f64(double v) { return log(v); }
__device__ __noinline__ double exp_f64(double v) { return exp(v); }

// ------------------------------------------------------ block helpers --
__device__ __forceinline__ float block_max_f32(float v, float *lds) {
    v = wave_max_dpp(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    float m = lds[0];
#pragma unroll
    for (int w = 1; w < kSmcWaves; ++w) m = fmaxf(m, lds[w]);
    __syncthreads();
    return m;
}

__device__ __forceinline__ double block_sum_f64(double v, double *lds) {
    v = wave_sum_dpp(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kSmcWaves; ++w) s += lds[w];
    __syncthreads();
    return s;
}

// Two sums in one pass (lds holds 2 * kSmcWaves doubles).
__device__ __forceinline__ void block_sum2_f64(double &u, double &v, double *lds) {
    u = wave_sum_dpp(u);
    v = wave_sum_dpp(v);
    if ((threadIdx.x & 63) == 0) {
        lds[threadIdx.x >> 6] = u;
        lds[kSmcWaves + (threadIdx.x >> 6)] = v;
    }
    __syncthreads();
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int w = 0; w < kSmcWaves; ++w) {
        a += lds[w];
        b += lds[kSmcWaves + w];
    }
    __syncthreads();
    u = a;
    v = b;
}

// Exclusive scan of one u64 per thread across the block; returns the prefix,
// writes the block total.
__device__ __forceinline__ uint64_t block_exclusive_scan_u64(uint64_t v, uint64_t *lds, uint64_t &total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint64_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) lds[wv] = incl;
    __syncthreads();
    uint64_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kSmcWaves; ++w) {
        const uint64_t x = lds[w];
        if (w < wv) off += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return off + incl - v;
}

// Merge of the per-block partials {m, s1, s2} (identical in every block):
// fixed order, FP32 rescale factors (this feeds the resampling trigger only).
// Merges the per-block partials {max, s1, s2} that thread t < nb holds for
// block t, in the same order in every block.
__device__ __forceinline__ void merge_partials(float mb, double p1, double p2, float *ldsf, double *ldsd, float &M,
                                               double &S1, double &S2) {
    M = block_max_f32(mb, ldsf);
    double s1 = 0.0, s2 = 0.0;
    if (M > -INFINITY && mb > -INFINITY) {
        const float c = expf(mb - M);
        s1 = p1 * (double)c;
        s2 = p2 * (double)(c * c);
    }
    block_sum2_f64(s1, s2, ldsd);
    S1 = s1;
    S2 = s2;
}

// Slot thresholds.  For integers, N Q_a > j S + U  <=>  Q_a > floor((j S + U) / N),
// and with S = N Sq + Sr (Sr < N < 2^31):
//   tau_j = floor((j S + U) / N) = j Sq + floor((j Sr + U) / N),
// where j Sr + U < 2^63, so tau_j needs only 64-bit arithmetic.  Consecutive
// slots update the quotient and remainder incrementally.
struct SlotThreshold {
    uint64_t quo, rem;   // of (j Sr + U) / N
};

__device__ __forceinline__ SlotThreshold slot_threshold(uint32_t j, uint64_t Sr, uint64_t U, uint64_t N) {
    const uint64_t num = (uint64_t)j * Sr + U;
    return SlotThreshold{num / N, num % N};
}

__device__ __forceinline__ void slot_threshold_next(SlotThreshold &t, uint64_t Sr, uint64_t N) {
    t.rem += Sr;
    if (t.rem >= N) {
        t.rem -= N;
        t.quo += 1;
    }
}

// Resampling data carry their event's tag, so the readers need no acquire
// (and the writers no release).  A prefix word holds the tag in its top two
// bits (1 + r mod 3 for the (r + 1)-th event of the call: never 0, the value
// the words are cleared to before the launch, and never the previous
// event's) and the tile-local exclusive prefix (< 2^62) below; a state word
// holds r + 1 in its high half and the FP32 bits in its low half.  A reader
// that finds another tag (the store has not reached it yet) polls the word
// again; after kSpinLimit polls, or once another block has aborted, it sets
// `bad` and returns 0 (an in-range value, so every index derived from it
// stays in bounds).
constexpr int kQTagShift = 62;
constexpr uint64_t kQMask = (1ull << kQTagShift) - 1;

__device__ __forceinline__ uint64_t qtag_of(int64_t r) { return (uint64_t)(1 + r % 3) << kQTagShift; }

__device__ __forceinline__ uint64_t read_q(const uint64_t *w, uint64_t tag, unsigned *abort_flag, bool &bad) {
    uint64_t v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t spins = 0;
    while ((v & ~kQMask) != tag) {
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 63) == 0 &&
            (spins > kSpinLimit || __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
            __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bad = true;
            return 0;
        }
        v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return v & kQMask;
}

__device__ __forceinline__ float read_x(const uint64_t *w, uint32_t tag, unsigned *abort_flag, bool &bad) {
    uint64_t v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t spins = 0;
    while ((uint32_t)(v >> 32) != tag) {
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 63) == 0 &&
            (spins > kSpinLimit || __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
            __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bad = true;
            return 0.0f;
        }
        v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return __uint_as_float((uint32_t)v);
}

// Ancestor of the slot with threshold tau over the whole population: the
// last a with X_a <= tau, where X_a = tile_pre[b] + x_a is the exclusive
// prefix of q before a (x_a tile-local, tagged in device memory; tile ends
// and exclusive tile prefixes are in LDS).  This is min{a : Q_a > tau} for the
// inclusive prefix Q: a particle of zero weight shares its prefix with the
// next one.  lo_bound (the previous slot's ancestor, or -1) has X <= tau.
__device__ __forceinline__ int find_ancestor_global(uint64_t tau, int64_t N, int nb, int tile, const uint64_t *tile_end,
                                                    const uint64_t *tile_pre, const uint64_t *qt, uint64_t tag,
                                                    int lo_bound, unsigned *abort_flag, bool &bad) {
    int lo = lo_bound < 0 ? 0 : lo_bound / tile, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (tile_end[mid] > tau) hi = mid; else lo = mid + 1;
    }
    const uint64_t pre = tile_pre[lo];
    // X of the tile's first particle is tile_pre[lo] <= tau (tile lo is the first
    // whose end exceeds tau), so the answer is in [a0, a1): search for the first
    // index after a0 whose prefix exceeds tau
    int a0 = lo * tile;
    const int a1 = (int)min((int64_t)a0 + tile, N);
    if (lo_bound > a0) a0 = lo_bound;
    int l = a0 + 1, h = a1;
    while (l < h) {
        const int mid = (l + h) >> 1;
        if (pre + read_q(qt + mid, tag, abort_flag, bad) > tau) h = mid; else l = mid + 1;
    }
    return l - 1;
}

// ---------------------------------------------------------------- kernel --
// MOVES: the resample-move instantiation (a separate kernel, so the moves'
// registers never add to the plain filter's).
template <class M, int P, bool MOVES>
__global__ __launch_bounds__(kSmcThreads) void smc_persistent_kernel(SmcDev a) {
    __shared__ float ldsf[kSmcWaves];
    __shared__ double ldsd[2 * kSmcWaves];
    __shared__ uint64_t ldsu[kSmcWaves];
    __shared__ float ybuf[kYChunk];
    __shared__ int s_rng[2];
    __shared__ int s_cnt[kSmcWaves];
    // dynamic LDS: tile_end[nb] | tile_pre[nb] | stage[stage_cap] | own_q[kTile] (u64) |
    // s_anc[kTile] (i32) | own_x[kTile] (FP32, one-field models only)
    constexpr int kTile = kSmcThreads * P;
    constexpr bool kOwnX = M::NF == 1;
    extern __shared__ uint64_t dyn[];
    const int nb = gridDim.x;
    uint64_t *tile_end = dyn;
    uint64_t *tile_pre = dyn + nb;
    uint64_t *stage = dyn + 2 * nb;
    uint64_t *own_q = dyn + 2 * nb + a.stage_cap;
    int32_t *s_anc = (int32_t *)(own_q + kTile);
    float *own_x = (float *)(s_anc + kTile);

    const int64_t N = a.N;
    const int64_t tile0 = (int64_t)blockIdx.x * kTile;                 // this block's first slot
    const int tlen = (int)min((int64_t)kTile, N - tile0);               // and its slot count
    // tagged prefix words loaded per round: all of them for the one-field model,
    // fewer beside a larger particle state
    constexpr int kLoadBatch = M::NF > 2 ? 4 : 16;
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * P;

    float st[P][M::NF];
    float lw[P], lwc[P];     // log-weight and its compensation term
    bool valid[P];
    unsigned epoch = 0;
    double logz = 0.0;
    int64_t nres = 0;
    int status = 0;
    float Mlast = 0.0f;
    bool alive = true;
    const double logN = log_f64((double)N);
    if (a.t0 > 0) {
        // resume: the run's scalars from the header, each particle from the checkpoint
        const SmcCkpt *h = (const SmcCkpt *)a.ckpt;
        const float *cs = (const float *)(a.ckpt + kCkptHeader);
        if (h->t != a.t0 || h->N != N || h->nf != M::NF) {
            status = PPL_E_ARG;
        } else {
            logz = h->logz;
            nres = h->nres;
            Mlast = h->mlast;
            status = h->status;
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            valid[p] = base + p < N;
#pragma unroll
            for (int f = 0; f < M::NF; ++f) st[p][f] = valid[p] ? cs[(size_t)f * N + base + p] : 0.0f;
            lw[p] = valid[p] ? cs[(size_t)M::NF * N + base + p] : -INFINITY;
            lwc[p] = valid[p] ? cs[(size_t)(M::NF + 1) * N + base + p] : 0.0f;
        }
    } else {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            valid[p] = base + p < N;
            M::init(a, (uint32_t)(base + p), st[p]);
            lw[p] = valid[p] ? 0.0f : -INFINITY;
            lwc[p] = 0.0f;
        }
    }

    for (int64_t s = a.t0; status == 0 && s < a.t1; ++s) {
        if (s == a.t0 || (s % kYChunk) == 0) {     // stage the chunk of observations holding factor s
            const int64_t c0 = s - s % kYChunk;
            __syncthreads();
            for (int i = threadIdx.x; i < kYChunk; i += kSmcThreads)
                ybuf[i] = (c0 + i < a.T) ? a.y[c0 + i] : 0.0f;
            __syncthreads();
        }
        const float ys = ybuf[s % kYChunk];
        // The slot index is re-materialised every factor: otherwise the compiler
        // hoists every per-slot address out of the factor loop and runs out of VGPRs.
        int jb = (int)base;
        asm volatile("" : "+v"(jb));
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const float f = M::step(a, s, (uint32_t)(jb + p), st[p], ys);
            if (valid[p]) kahan_add(lw[p], lwc[p], f);
        }
        // block partial for the ESS trigger
        float ml = -INFINITY;
#pragma unroll
        for (int p = 0; p < P; ++p) ml = fmaxf(ml, lw[p]);
        const float mb = block_max_f32(ml, ldsf);
        float s1l = 0.0f, s2l = 0.0f;
        if (mb > -INFINITY) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const float e = expf(lw[p] - mb);
                s1l += e;
                s2l = fmaf(e, e, s2l);
            }
        }
        double s1b = s1l, s2b = s2l;
        block_sum2_f64(s1b, s2b, ldsd);
        uint32_t rt[5];
        if (!tagged_barrier<5>(a.rec, a.bar, ++epoch, nb,
                               {__float_as_uint(mb), hi32(s1b), lo32(s1b), hi32(s2b), lo32(s2b)}, rt)) {
            alive = false;
            break;
        }
        float Mg;
        double S1, S2;
        merge_partials(threadIdx.x < nb ? __uint_as_float(rt[0]) : -INFINITY, from32(rt[1], rt[2]),
                       from32(rt[3], rt[4]), ldsf, ldsd, Mg, S1, S2);
        Mlast = Mg;
        if (!(Mg > -INFINITY)) { status = PPL_E_ZERO_WEIGHT; break; }
        if (!(S1 > 0.0) || isnan(S1) || isnan(S2)) { status = PPL_E_NONFINITE; break; }
        const double ess = S1 * S1 / S2;
        const bool res = (s < a.T - 1) && (ess < (double)a.ess_frac * (double)N);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (a.ess_trace) a.ess_trace[s] = ess;
            if (a.resampled) a.resampled[s] = res ? 1 : 0;
            if (a.logz_tr && !res) a.logz_tr[s] = 0.0;
        }
        if (!res) continue;
        if (a.elw_out && nres < a.max_events) {
#pragma unroll
            for (int p = 0; p < P; ++p)
                if (valid[p]) a.elw_out[(size_t)nres * N + jb + p] = lw[p];
        }

        // ---- resampling: FP64 weights, normaliser, integer quantisation, tile scan
        uint64_t qx[P];          // exclusive prefixes within the thread
        uint64_t run = 0;
        double esl = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const double e = valid[p] ? exp_f64((double)lw[p] - (double)Mg) : 0.0;
            esl += e;
            qx[p] = run;
            run += (uint64_t)floor(ldexp(e, a.kbits));
        }
        uint64_t btot;
        const uint64_t off = block_exclusive_scan_u64(run, ldsu, btot);
        const double eb = block_sum_f64(esl, ldsd);
        const uint64_t qtag = qtag_of(nres);
        const uint32_t xtag = (uint32_t)(nres + 1);
        // The tile's prefix sums (and a one-field state) go to LDS, where this
        // block reads its own ancestors, and from there to memory with
        // coalesced stores (whole lines; the particle-major layout of the
        // registers would scatter each store over a wave's 64 particles).
#pragma unroll
        for (int p = 0; p < P; ++p) {
            own_q[threadIdx.x * P + p] = off + qx[p];
            if constexpr (kOwnX) own_x[threadIdx.x * P + p] = st[p][0];
        }
        if constexpr (!kOwnX) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (valid[p]) {
#pragma unroll
                    for (int f = 0; f < M::NF; ++f)
                        __hip_atomic_store(a.xtag + (size_t)f * N + jb + p,
                                           ((uint64_t)xtag << 32) | __float_as_uint(st[p][f]), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < tlen; i += kSmcThreads) {
            __hip_atomic_store(a.qtag + tile0 + i, qtag | own_q[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if constexpr (kOwnX)
                __hip_atomic_store(a.xtag + tile0 + i, ((uint64_t)xtag << 32) | __float_as_uint(own_x[i]),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        uint32_t rq[4];
        if (!tagged_barrier<4>(a.rec, a.bar, ++epoch, nb,
                               {(uint32_t)(btot >> 32), (uint32_t)btot, hi32(eb), lo32(eb)}, rq)) {
            alive = false;
            break;
        }
        unsigned *abort_flag = a.bar + 1;
        bool bad = false;

        // tile prefixes (LDS) and the normaliser sum, in the same order in every block
        {
            const uint64_t v = threadIdx.x < nb ? ((uint64_t)rq[0] << 32) | rq[1] : 0;
            const double ev0 = threadIdx.x < nb ? from32(rq[2], rq[3]) : 0.0;
            uint64_t S;
            const uint64_t ex = block_exclusive_scan_u64(v, ldsu, S);
            if (threadIdx.x < nb) {
                tile_pre[threadIdx.x] = ex;
                tile_end[threadIdx.x] = ex + v;
            }
            const double ev = block_sum_f64(ev0, ldsd);     // contains the barrier for tile_*
            const uint4 rw = philox(0, 0, (uint32_t)s, (a.inst << 8) | kTagResample, a.key);
            const uint64_t U = __umul64hi(((uint64_t)rw.y << 32) | rw.x, S);
            const double inc = (double)Mg + log_f64(ev) - logN;
            logz += inc;
            if (a.logz_tr && blockIdx.x == 0 && threadIdx.x == 0) a.logz_tr[s] = inc;
            ++nres;
            const uint64_t NN = (uint64_t)N;
            const uint64_t Sq = S / NN, Sr = S - Sq * NN;

            // ancestor range of this block's slots: the first and last slot's
            // ancestors, each found by half of the block.  The ancestor's tile
            // is the first with tile_end > tau (LDS); within it the exclusive
            // prefix sums are non-decreasing and the first is <= tau, so the
            // ancestor's offset is the number of entries <= tau, less one,
            // counted with one round of independent loads.
            const int js0 = blockIdx.x * kTile;
            const int js1 = (int)min((int64_t)js0 + kTile, N) - 1;
            {
                constexpr int kHalf = kSmcThreads / 2;
                const int half = threadIdx.x / kHalf, hl = threadIdx.x % kHalf;
                const uint32_t jsx = (uint32_t)(half ? js1 : js0);
                const SlotThreshold t = slot_threshold(jsx, Sr, U, NN);
                const uint64_t tau = (uint64_t)jsx * Sq + t.quo;
                int lo = 0, hi = nb - 1;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (tile_end[mid] > tau) hi = mid; else lo = mid + 1;
                }
                const int64_t tb = (int64_t)lo * kTile;
                const int len = (int)min((int64_t)kTile, N - tb);
                const uint64_t pre = tile_pre[lo];
                // all loads first (clamped in range), then the count; a word that
                // is not yet current sends the thread through the polling reads
                constexpr int kPer = kTile / kHalf;
                int cnt = 0;
                bool fresh = !a.poll_all;
                if (lo == (int)blockIdx.x) {       // this block's own tile: its prefix sums are in LDS
                    for (int i = hl; i < len; i += kHalf) cnt += (pre + own_q[i] <= tau) ? 1 : 0;
                } else {
#pragma unroll
                for (int k0 = 0; k0 < kPer; k0 += kLoadBatch) {
                    uint64_t v[kLoadBatch];
#pragma unroll
                    for (int k = 0; k < kLoadBatch; ++k)
                        v[k] = __hip_atomic_load(a.qtag + tb + min(hl + (k0 + k) * kHalf, len - 1), __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                    for (int k = 0; k < kLoadBatch; ++k) {
                        if (k0 + k < kPer && hl + (k0 + k) * kHalf < len) {
                            fresh = fresh && (v[k] & ~kQMask) == qtag;
                            cnt += (pre + (v[k] & kQMask) <= tau) ? 1 : 0;
                        }
                    }
                }
                }
                if (!fresh) {
                    cnt = 0;
                    for (int i = hl; i < len; i += kHalf)
                        cnt += (pre + read_q(a.qtag + tb + i, qtag, abort_flag, bad) <= tau) ? 1 : 0;
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
                if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = cnt;
                __syncthreads();
                if (hl == 0) {
                    int c = 0;
                    for (int w = 0; w < kSmcWaves / 2; ++w) c += s_cnt[half * (kSmcWaves / 2) + w];
                    s_rng[half] = (int)(tb + c - 1);
                }
            }
            __syncthreads();
            const int a_lo = s_rng[0], a_hi = s_rng[1];
            const int span = a_hi - a_lo + 1;
            const bool staged = span >= 1 && span <= a.stage_cap;
            if (staged) {
                constexpr int kPer = kStage / kSmcThreads;
                bool fresh = !a.poll_all;
#pragma unroll
                for (int k0 = 0; k0 < kPer; k0 += kLoadBatch) {
                    uint64_t v[kLoadBatch];
#pragma unroll
                    for (int k = 0; k < kLoadBatch; ++k) {
                        const int aa = a_lo + min((int)threadIdx.x + (k0 + k) * kSmcThreads, span - 1);
                        v[k] = (uint64_t)(aa - tile0) < (uint64_t)tlen
                                   ? qtag | own_q[aa - tile0]
                                   : __hip_atomic_load(a.qtag + aa, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
#pragma unroll
                    for (int k = 0; k < kLoadBatch; ++k) {
                        const int i = threadIdx.x + (k0 + k) * kSmcThreads;
                        if (k0 + k < kPer && i < span) {
                            fresh = fresh && (v[k] & ~kQMask) == qtag;
                            stage[i] = tile_pre[(a_lo + i) / kTile] + (v[k] & kQMask);
                        }
                    }
                }
                if (!fresh) {
                    for (int i = threadIdx.x; i < span; i += kSmcThreads) {
                        const int aa = a_lo + i;
                        const uint64_t x = (uint64_t)(aa - tile0) < (uint64_t)tlen
                                               ? own_q[aa - tile0]
                                               : read_q(a.qtag + aa, qtag, abort_flag, bad);
                        stage[i] = tile_pre[aa / kTile] + x;
                    }
                }
            }
            __syncthreads();

            int32_t *anc_row = (a.anc_out && nres - 1 < a.max_events) ? a.anc_out + (size_t)(nres - 1) * N : nullptr;
            if (jb < N) {
                SlotThreshold th = slot_threshold((uint32_t)jb, Sr, U, NN);
                if (staged) {
                    // Each ancestor is the last staged entry <= its slot's tau:
                    // one before the first entry > tau (span if none).  The
                    // thread's first slot binary-searches the stage (entry 0, the
                    // block's first ancestor, is <= tau); later slots count the
                    // entries <= tau among the kWin after the first slot's
                    // ancestor, held in registers (one round of LDS loads for all
                    // slots), and past that window gallop from the previous slot's
                    // ancestor (whose entry is <= tau) and finish with a binary
                    // search.
                    constexpr int kWin = 16;
                    int lo = 1, hi = span;
                    {
                        const uint64_t tau0 = (uint64_t)jb * Sq + th.quo;
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (stage[mid] > tau0) hi = mid; else lo = mid + 1;
                        }
                    }
                    const int pos0 = lo - 1;
                    uint64_t win[kWin];
#pragma unroll
                    for (int k = 0; k < kWin; ++k) win[k] = pos0 + 1 + k < span ? stage[pos0 + 1 + k] : ~0ull;
                    int prev = pos0;
#pragma unroll 1
                    for (int p = 0; p < P; ++p) {
                        const int j = jb + p;
                        if (j >= N) break;
                        if (p) slot_threshold_next(th, Sr, NN);
                        const uint64_t tau = (uint64_t)j * Sq + th.quo;
                        int c = 0;
#pragma unroll
                        for (int k = 0; k < kWin; ++k) c += win[k] <= tau ? 1 : 0;
                        int idx;
                        if (c < kWin) {
                            idx = pos0 + c;
                        } else {
                            int l = prev + 1, h = span;
                            if (l < h) {
                                if (stage[l] > tau) {
                                    h = l;
                                } else {
                                    int step = 1;
                                    while (l + step < h && !(stage[l + step] > tau)) {
                                        l += step;
                                        step <<= 1;
                                    }
                                    h = min(l + step, h);
                                    ++l;
                                }
                            }
                            while (l < h) {
                                const int mid = (l + h) >> 1;
                                if (stage[mid] > tau) h = mid; else l = mid + 1;
                            }
                            idx = l - 1;
                        }
                        s_anc[threadIdx.x * P + p] = a_lo + idx;
                        if (anc_row) anc_row[j] = a_lo + idx;
                        prev = idx;
                    }
                } else {
                    int prev = a_lo;
#pragma unroll 1
                    for (int p = 0; p < P; ++p) {
                        const int j = jb + p;
                        if (j >= N) break;
                        if (p) slot_threshold_next(th, Sr, NN);
                        const uint64_t tau = (uint64_t)j * Sq + th.quo;
                        const int anc = find_ancestor_global(tau, N, nb, kTile, tile_end, tile_pre, a.qtag, qtag, prev,
                                                             abort_flag, bad);
                        s_anc[threadIdx.x * P + p] = anc;
                        if (anc_row) anc_row[j] = anc;
                        prev = anc;
                    }
                }
            }
        }
        if constexpr (!MOVES) {
            // gather the ancestors' state: all loads first, then the tags; a word
            // that is not yet current sends the thread through the polling reads
            bool fresh = !a.poll_all;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (!valid[p]) continue;
                const int anc = s_anc[threadIdx.x * P + p];
                if (kOwnX && (uint64_t)(anc - tile0) < (uint64_t)tlen) {
                    st[p][0] = own_x[anc - tile0];      // an ancestor of this block's own tile
                } else {
#pragma unroll
                    for (int f = 0; f < M::NF; ++f) {
                        const uint64_t v = __hip_atomic_load(a.xtag + (size_t)f * N + anc, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                        fresh = fresh && (uint32_t)(v >> 32) == xtag;
                        st[p][f] = __uint_as_float((uint32_t)v);
                    }
                }
                lw[p] = 0.0f;
                lwc[p] = 0.0f;
            }
            if (!fresh) {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    if (!valid[p]) continue;
                    const int anc = s_anc[threadIdx.x * P + p];
                    if (kOwnX && (uint64_t)(anc - tile0) < (uint64_t)tlen) continue;
#pragma unroll
                    for (int f = 0; f < M::NF; ++f)
                        st[p][f] = read_x(a.xtag + (size_t)f * N + anc, xtag, abort_flag, bad);
                }
            }
        } else {
            // resample-move: the gathered particles go through memory one at a
            // time, so only the moving particle's state occupies registers
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (!valid[p]) continue;
                const int anc = s_anc[threadIdx.x * P + p];
#pragma unroll
                for (int f = 0; f < M::NF; ++f)
                    a.xbuf2[(size_t)f * N + jb + p] = read_x(a.xtag + (size_t)f * N + anc, xtag, abort_flag, bad);
                lw[p] = 0.0f;
                lwc[p] = 0.0f;
            }
            double *arow = (a.alpha_out && nres - 1 < a.max_events)
                               ? a.alpha_out + (size_t)(nres - 1) * a.move_steps * N : nullptr;
#pragma unroll 1
            for (int p = 0; p < P; ++p) {
                const int j = jb + p;
                if (j >= N) break;
                MoveOf<M>::run(a, s, (uint32_t)j, a.xbuf2 + j, (size_t)N, arow, N);
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
#pragma unroll
                for (int f = 0; f < M::NF; ++f) st[p][f] = valid[p] ? a.xbuf2[(size_t)f * N + jb + p] : 0.0f;
            }
        }
        if (__syncthreads_or(bad ? 1 : 0)) { alive = false; break; }   // a tagged read gave up
    }

    // ---- stop: the run's state into the checkpoint
    const bool stopped = a.t1 < a.T;
    if (stopped && alive) {
        float *cs = (float *)(a.ckpt + kCkptHeader);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (!valid[p]) continue;
#pragma unroll
            for (int f = 0; f < M::NF; ++f) cs[(size_t)f * N + base + p] = st[p][f];
            cs[(size_t)M::NF * N + base + p] = lw[p];
            cs[(size_t)(M::NF + 1) * N + base + p] = lwc[p];
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            SmcCkpt *h = (SmcCkpt *)a.ckpt;
            h->t = a.t1;
            h->N = N;
            h->nres = nres;
            h->nf = M::NF;
            h->status = status;
            h->logz = logz;
            h->mlast = Mlast;
        }
    }
    // ---- final normaliser (FP64) over the last epoch
    double ess_final = stopped ? 0.0 : (double)N;
    if (alive && status == 0 && a.T > 0 && !stopped) {
        double e1 = 0.0, e2 = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (valid[p]) {
                const double e = exp_f64((double)lw[p] - (double)Mlast);
                e1 += e;
                e2 += e * e;
            }
        }
        block_sum2_f64(e1, e2, ldsd);
        uint32_t rt[4];
        if (!tagged_barrier<4>(a.rec, a.bar, ++epoch, nb, {hi32(e1), lo32(e1), hi32(e2), lo32(e2)}, rt)) {
            alive = false;
        } else {
            double t1 = threadIdx.x < nb ? from32(rt[0], rt[1]) : 0.0;
            double t2 = threadIdx.x < nb ? from32(rt[2], rt[3]) : 0.0;
            block_sum2_f64(t1, t2, ldsd);
            const double inc = (double)Mlast + log_f64(t1) - logN;
            logz += inc;
            if (a.logz_tr && blockIdx.x == 0 && threadIdx.x == 0) a.logz_tr[a.T - 1] = inc;
            ess_final = t1 * t1 / t2;
        }
    }
    if (!alive) status = PPL_E_HIP;

#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (!valid[p]) continue;
        const int64_t j = base + p;
        if (a.lw_out) a.lw_out[j] = lw[p];
        if (a.lat_out) {
#pragma unroll
            for (int f = 0; f < M::NF; ++f) a.lat_out[(size_t)f * N + j] = st[p][f];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.scalars[0] = status ? (status == PPL_E_ZERO_WEIGHT ? -INFINITY : NAN) : logz;
        a.scalars[1] = status ? 0.0 : ess_final;
        a.scalars[2] = (double)nres;
        a.scalars[3] = (double)status;
        a.scalars[4] = (double)Mlast;
        a.scalars[5] = 0.0;
        a.scalars[6] = 0.0;
        a.scalars[7] = (double)N;
    }
}

// Clears the abort flag and the record lines' epochs (a fill kernel, so the
// launch sequence stays capturable).
__global__ void smc_reset_kernel(unsigned *bar, uint64_t *rec, int n_lines, uint64_t *tagged, int64_t n_tagged) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = i0; i < kBarWords; i += stride) bar[i] = 0u;
    for (int64_t i = i0; i < (int64_t)n_lines * kRecWords; i += stride) rec[i] = 0u;
    for (int64_t i = i0; i < n_tagged; i += stride) tagged[i] = 0u;
}

// ------------------------------------------------------------------ host --
static int pick_p(int64_t N) {
    // particles per thread so that one block per CU covers N (up to 8)
    const int64_t per_cu = (N + 255) / 256;
    int P = 1;
    while (P < 8 && (int64_t)kSmcThreads * P < per_cu) P <<= 1;
    return P;
}

static int64_t smc_blocks(int64_t N, int P) { return (N + (int64_t)kSmcThreads * P - 1) / ((int64_t)kSmcThreads * P); }

struct SmcLayout {
    double *scal;
    unsigned *bar;
    uint64_t *rec, *qtag, *xtag;     // qtag and xtag adjacent: [N] then [NF][N]
    float *xbuf2;
    size_t bytes;
};

static SmcLayout smc_layout(void *ws, int NF, int64_t N, int64_t nb) {
    SmcLayout L;
    char *p = (char *)ws;
    size_t o = 0;
    auto take = [&](size_t n) { char *r = p + o; o += align_up(n, 256); return r; };
    L.scal = (double *)take(8 * sizeof(double));
    L.bar = (unsigned *)take(kBarWords * sizeof(unsigned));
    L.rec = (uint64_t *)take((size_t)2 * nb * kRecWords * sizeof(uint64_t));
    L.qtag = (uint64_t *)take((size_t)(NF + 1) * N * sizeof(uint64_t));
    L.xtag = L.qtag + N;
    L.xbuf2 = NF > 1 ? (float *)take((size_t)NF * N * sizeof(float)) : nullptr;   // mixture models only
    L.bytes = o;
    return L;
}

size_t smc_checkpoint_bytes(int model, int K, int64_t N) {
    const int NF = model == PPL_MODEL_LGSSM ? 1 : 2 * K;
    return kCkptHeader + align_up((size_t)(NF + 2) * N * sizeof(float), 256);
}

size_t smc_ws_bytes(int model, int K, int64_t N) {
    const int NF = model == PPL_MODEL_LGSSM ? 1 : 2 * K;
    const int P = pick_p(N);
    return smc_layout(nullptr, NF, N, smc_blocks(N, P)).bytes;
}

double *smc_scalars_ptr(const SmcArgs &a) { return a.out.d_scalars ? a.out.d_scalars : (double *)a.ws; }

template <class M, int P>
static int launch(SmcDev &d, int64_t nb, hipStream_t st) {
    auto kern = d.move_steps > 0 ? smc_persistent_kernel<M, P, true> : smc_persistent_kernel<M, P, false>;
    int dev = 0, ncu = 0, occ = 0;
    PPL_HIP(hipGetDevice(&dev));
    PPL_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    // stage as many prefix sums as the per-block LDS limit leaves room for (<= kStage)
    int max_lds = 0;
    PPL_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int64_t tile = (int64_t)kSmcThreads * P;
    const int64_t own_x = M::NF == 1 ? tile * (int64_t)sizeof(float) : 0;
    const int64_t fixed = (int64_t)(2 * nb + tile) * sizeof(uint64_t) + tile * (int64_t)sizeof(int32_t) + own_x +
                          (int64_t)kYChunk * sizeof(float) + 1024;      // + static LDS of the kernel
    d.stage_cap = (int)std::max<int64_t>(0, std::min<int64_t>(kStage, (max_lds - fixed) / 8));
    const size_t lds = (size_t)(2 * nb + d.stage_cap + tile) * sizeof(uint64_t) + (size_t)tile * sizeof(int32_t) +
                       (size_t)own_x;
    PPL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kSmcThreads, lds));
    if ((int64_t)occ * ncu < nb)
        return fail(PPL_E_UNSUPPORTED, "SMC needs %lld co-resident blocks, device holds %d", (long long)nb, occ * ncu);
    // clears the barrier words, the record lines and the tagged resampling data
    // (so no word of an earlier call carries a tag this call looks for)
    const int64_t n_tagged = (int64_t)(d.xtag - d.qtag) + (int64_t)M::NF * d.N;
    const int reset_blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n_tagged + 255) / 256));
    hipLaunchKernelGGL(smc_reset_kernel, dim3(reset_blocks), dim3(256), 0, st, d.bar, d.rec, (int)(2 * nb), d.qtag,
                       n_tagged);
    PPL_LAUNCH_CHECK("smc_reset_kernel");
    void *args[] = {&d};
    KernelTimer timer("smc_persistent_kernel", st);
    PPL_HIP(hipLaunchCooperativeKernel((const void *)kern, dim3((unsigned)nb), dim3(kSmcThreads), args, lds, st));
    timer.stop();
    return PPL_OK;
}

template <class M>
static int launch_p(SmcDev &d, int P, int64_t nb, hipStream_t st) {
    switch (P) {
        case 1: return launch<M, 1>(d, nb, st);
        case 2: return launch<M, 2>(d, nb, st);
        case 4: return launch<M, 4>(d, nb, st);
        case 8: return launch<M, 8>(d, nb, st);
    }
    return fail(PPL_E_UNSUPPORTED, "particles per thread %d", P);
}

int run_smc(const SmcArgs &a, hipStream_t st) {
    const int NF = a.model == PPL_MODEL_LGSSM ? 1 : 2 * a.K;
    const int P = pick_p(a.N);
    const int64_t nb = smc_blocks(a.N, P);
    // every block merges the per-block partials one per thread
    if (nb > kSmcMaxBlocks || nb > kSmcThreads)
        return fail(PPL_E_UNSUPPORTED, "SMC supports at most %lld particles",
                    (long long)std::min(kSmcMaxBlocks, kSmcThreads) * kSmcThreads * 8);
    if (a.T > 0x7fffffffLL) return fail(PPL_E_ARG, "too many factors");
    // a run passes at most 2 T + 1 barriers, each with its own epoch
    if (2 * a.T + 2 >= 0xffffffffLL) return fail(PPL_E_UNSUPPORTED, "barrier epoch would overflow");
    SmcLayout L = smc_layout(a.ws, NF, a.N, nb);
    SmcDev d{};
    d.y = a.y;
    d.T = a.T;
    d.N = a.N;
    d.K = a.K;
    d.key = make_key(a.seed);
    d.inst = a.inst;
    d.ess_frac = (float)a.ess_frac;
    for (int i = 0; i < 5; ++i) d.hyp[i] = (float)a.hyper[i];
    if (a.model == PPL_MODEL_LGSSM) d.lconst = -0.5 * log(2.0 * M_PI * a.hyper[2] * a.hyper[2]);
    else d.lconst = -0.5 * log(2.0 * M_PI) - log(a.hyper[1]);
    int c = 0;
    while (((int64_t)1 << c) < a.N) ++c;
    d.kbits = 62 - c;
    d.scalars = a.out.d_scalars ? a.out.d_scalars : L.scal;
    d.lw_out = (float *)a.out.d_log_weights;
    d.lat_out = (float *)a.out.d_latents;
    d.ess_trace = a.out.d_ess_trace;
    d.resampled = a.out.d_resampled;
    d.anc_out = a.out.d_ancestors;
    d.elw_out = a.out.d_event_lw;
    d.logz_tr = a.out.d_logz_trace;
    d.alpha_out = a.out.d_move_log_alpha;
    d.max_events = a.out.max_events;
    d.t0 = a.t_begin;
    d.t1 = a.t_end;
    d.ckpt = (char *)a.ckpt;
    d.move_steps = a.move_steps;
    // PPL_SMC_POLL_ALL=1 sends every tagged read through the polling path
    // (checking aid: the results must not change)
    {
        const char *e = getenv("PPL_SMC_POLL_ALL");
        d.poll_all = (e && e[0] == '1') ? 1 : 0;
    }
    d.move_lam = a.move_scale > 0.0 ? a.move_scale : 2.38 / sqrt(2.0 * a.K - 1.0);
    d.hyp64[0] = a.hyper[0];
    d.hyp64[1] = a.hyper[1];
    d.bar = L.bar;
    d.rec = L.rec;
    d.qtag = L.qtag;
    d.xtag = L.xtag;
    d.xbuf2 = L.xbuf2;
    if (a.model == PPL_MODEL_LGSSM) return launch_p<Lgssm>(d, P, nb, st);
    switch (a.K) {
        case 1: return launch_p<Gmm<1>>(d, P, nb, st);
        case 2: return launch_p<Gmm<2>>(d, P, nb, st);
        case 3: return launch_p<Gmm<3>>(d, P, nb, st);
        case 4: return launch_p<Gmm<4>>(d, P, nb, st);
        case 5: return launch_p<Gmm<5>>(d, P, nb, st);
        case 6: return launch_p<Gmm<6>>(d, P, nb, st);
        case 7: return launch_p<Gmm<7>>(d, P, nb, st);
        case 8: return launch_p<Gmm<8>>(d, P, nb, st);
    }
    return fail(PPL_E_ARG, "GMM K must be in 1..8");
}

}  // namespace ppl
