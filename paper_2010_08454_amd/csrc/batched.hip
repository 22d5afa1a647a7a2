// batched.hip -- many SMC instances in one persistent cooperative launch.
//
// Each instance is a mixture model with its own data and particle count; the
// per-instance algorithm is the SMC of smc.hip (the particle method the paper
// names as future work, Sec. 6, over the sample/factor semantics of Sec. 3.4).
//
// Mapping.  The grid (one 512-thread workgroup per CU: each wave then has 256
// registers, so with up to four particles per lane the particle state and the
// speculative-block bookkeeping stay out of scratch memory; eight per lane
// spill some of it) is split into teams of W workgroups; a team holds one
// instance at a time (slots j = w * 512 P + thread * P + p, P particles per
// thread, state in registers) and walks a list
// of instances assigned on the host by longest-processing-time-first, so the
// makespan is balanced.  Teams never wait on each other.
//
// Speculative blocks.  A team advances its particles through up to B factors
// before synchronising: after each factor every wave records {max, sum e,
// sum e^2} of its particles in LDS; at the end of the block the workgroups
// publish per-factor partials, meet at a team barrier, and every workgroup
// merges them in the same order.  The first factor t* whose ESS falls below
// ess_frac N decides: if there is none the block is committed (B doubles up to
// the tuned maximum); otherwise the log-weights are rolled back to the block
// start, the factors up to t* are recomputed (the same FP32 operations in the
// same order, so the result is bit-identical to a factor-by-factor run), the
// particles are resampled at t* with the integer rule of ppl_resample, and the
// next block starts at t* + 1 with B = 1.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "device.h"
#include "host.h"
#include "timing.h"
#include "batched.h"

namespace ppl {

constexpr int kBtThreads = 512;
constexpr int kBtWaves = kBtThreads / 64;
constexpr int kBtMaxInst = 1024;
constexpr int kBtMaxTeams = 256;
constexpr int kBtMaxB = 256;                  // largest speculative block
constexpr int kBtMaxW = 64;                   // largest team
constexpr int kBtStage = 8192;                // prefix sums staged for the ancestor search
constexpr int kBtNF = 16;                     // state floats per particle (2 K, K <= 8)
constexpr uint32_t kBtSpinLimit = 1u << 24;
constexpr int kBtBarLine = 32;

struct BtDev {
    const ppl_instance *inst;
    int n_inst;
    int any_moves;           // some instance has move_steps > 0 (selects the resample-move kernel)
    Key key;
    float ess_frac;
    int W;                   // workgroups per team
    int Bmax;                // speculative block limit
    int stage_cap;
    int64_t cap;             // slots per team (W * kBtThreads * P)
    double *out;             // [n_inst][4]
    float *lw_out, *lat_out;
    double *ess_tr;
    uint8_t *res_tr;
    int32_t *anc_out;        // [max_events * sum' N]: recorded instance i at max_events * R_i as [max_events][N_i]
    float *elw_out;          // same layout: the log-weights each event resampled from
    double *logz_tr;         // [sum D]: normaliser increment added after each factor
    double *alpha_out;       // resample-move log acceptance ratios, [max_events][M_i][N_i] per recorded instance
    int64_t max_events;
    unsigned long long *counters;   // [4] or null: work counters summed over instances (see ppl_batch_result)
    unsigned *bar;          // [1 + teams] lines: line 0 word 1 = abort flag; line 1 + t = team t counter
    double *part;            // [teams][2][W][Bmax][3]: two copies, picked by barrier-epoch parity
    uint64_t *tot;           // [teams][W]
    double *esum;            // [teams][W]: sum of the fraction words r of the event's weights (exact)
    uint64_t *fin;           // [teams][W][4]: 128-bit fixed-point sums of e and e^2 at the end
    uint64_t *qloc;          // [teams][cap]
    float *xbuf;             // [teams][NF][cap]
    float *xbuf2;            // [teams][NF][cap]: gathered particles while they move (resample-move)
    uint16_t order[kBtMaxInst];           // instances in scheduling order
    uint16_t team_off[kBtMaxTeams + 1];   // team t runs order[team_off[t] .. team_off[t+1])
};

// ------------------------------------------------------------ barrier ----
__device__ __forceinline__ bool team_barrier(unsigned *bar, int team, unsigned target) {
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned *ctr = &bar[kBtBarLine * (1 + team)];
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        int ok = 1;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if ((++spins & 63) == 0) {
                if (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
                if (spins > kBtSpinLimit) {
                    __hip_atomic_store(&bar[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (ok && __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

__device__ __noinline__ double bt_log(double v) { return log(v); }
__device__ __noinline__ double bt_exp(double v) { return exp(v); }

// ------------------------------------------------ exact normaliser sums ----
// The normaliser sums the FP64 weights e = exp(lw - max), in [0, 1], as
// integers, whose sums do not depend on the order of the additions: log Z-hat
// and the final ESS are then the same bits for every launch configuration
// (particles per lane, workgroups per instance).  With k the quantisation
// exponent of the resampling weights (x = e 2^k is exact):
//   - at a resampling event the sum is (S + 2^-32 R) 2^-k, where S = sum
//     floor(x) is the resampling total and R = sum floor(frac(x) 2^32); R's
//     partial sums are integers below 2^50, exact in FP64 in any grouping, so
//     the cheap FP64 wave reductions serve;
//   - at the end of a run the sums of e and e^2 are floor(x 2^64) in 128-bit
//     integers.
// What the floors drop is at most N 2^-(k+32) <= 2^-32 (events) or N 2^-(k+64)
// (end) of a sum that is at least 1 (the largest weight is 1).
typedef unsigned __int128 u128;

// Adds floor(e 2^(k + 64)) to the 128-bit sum (hi, lo) for e in [0, 1]:
// x = e 2^k is exact, its integer part goes to hi and its fraction, exact in
// FP64 (x - floor(x) keeps a subset of x's bits), is scaled by 2^64 and
// truncated into lo.  A NaN e adds nothing (the NaN status is raised elsewhere).
__device__ __forceinline__ void bt_fix_add(uint64_t &hi, uint64_t &lo, double e, int k) {
    if (!(e >= 0.0)) return;
    const double x = ldexp(e, k), xi = floor(x);
    const uint64_t l = (uint64_t)ldexp(x - xi, 64);
    lo += l;
    hi += (uint64_t)xi + (lo < l ? 1u : 0u);
}

__device__ __forceinline__ double bt_unfix(u128 v, int F) {
    const double hi = (double)(uint64_t)(v >> 64), lo = (double)(uint64_t)v;
    return ldexp(fma(hi, 18446744073709551616.0, lo), -F);
}

__device__ __forceinline__ u128 bt_wave_sum_u128(u128 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t lo = __shfl_xor((uint64_t)v, o, 64), hi = __shfl_xor((uint64_t)(v >> 64), o, 64);
        v += ((u128)hi << 64) | lo;
    }
    return v;
}

// Sum over the workgroup of two 128-bit values (lds: 4 * kBtWaves words).
__device__ __forceinline__ void bt_block_sum_u128x2(u128 &u, u128 &v, uint64_t *lds) {
    u = bt_wave_sum_u128(u);
    v = bt_wave_sum_u128(v);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        lds[4 * wv] = (uint64_t)u;
        lds[4 * wv + 1] = (uint64_t)(u >> 64);
        lds[4 * wv + 2] = (uint64_t)v;
        lds[4 * wv + 3] = (uint64_t)(v >> 64);
    }
    __syncthreads();
    u128 a = 0, b = 0;
#pragma unroll
    for (int w = 0; w < kBtWaves; ++w) {
        a += ((u128)lds[4 * w + 1] << 64) | lds[4 * w];
        b += ((u128)lds[4 * w + 3] << 64) | lds[4 * w + 2];
    }
    __syncthreads();
    u = a;
    v = b;
}

// --------------------------------------------------------------- model ----
// Mixture with KK <= 8 known components.  State (registers and the staging
// buffers): log pi_k at [k], mu_k at [KK + k].  Prior draws as in the
// single-instance SMC.
template <int KK>
__device__ __forceinline__ void bt_init(uint32_t j, uint32_t c3, Key key, float mu_sd, float st[2 * KK]) {
    const uint4 w0 = philox(j, 0, 0, c3, key), w1 = philox(j, 1, 0, c3, key);
    const uint32_t w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
    float E[KK], tot = 0.0f;
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        E[k] = -logf(unit_f32(w[k]));
        tot += E[k];
    }
    float z[8];
    normals4(philox(j, 2, 0, c3, key), z);
    normals4(philox(j, 3, 0, c3, key), z + 4);
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        st[k] = logf(E[k] / tot);
        st[KK + k] = mu_sd * z[k];
    }
}

// log sum_k pi_k N(y; mu_k, sd) for a compile-time component count KK (fully
// unrolled: no per-component branch and no padding of the term array).  The
// exponentials and the logarithm are the hardware's (v_exp_f32 / v_log_f32,
// about 1 ulp); their error is far below the FP32 rounding of the log-weight
// sum over the data.
// Every term t_k = log pi_k - r_k^2 / 2 is <= 0, so the plain sum of exp(t_k)
// cannot overflow; it is used when it exceeds kBtTiny (then no term has lost
// more than a few bits to underflow).  A datum far from every mean gives a
// smaller sum, and the factor is then the sum shifted by its largest term.
// Which form a particle takes depends on its own terms only.
constexpr float kBtTiny = 1e-30f;

template <int KK>
__device__ __forceinline__ void bt_terms(const float *st, float inv_sd, float ys, float (&t)[KK]) {
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        const float r = (ys - st[KK + k]) * inv_sd;
        t[k] = fmaf(-0.5f * r, r, st[k]);
    }
}

template <int KK>
__device__ __forceinline__ float bt_plain_sum(const float *st, float inv_sd, float ys) {
    float t[KK];
    bt_terms<KK>(st, inv_sd, ys, t);
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < KK; ++k) s += __expf(t[k]);
    return s;
}

template <int KK>
__device__ __forceinline__ float bt_shifted(const float *st, float inv_sd, float lconst, float ys) {
    float t[KK];
    bt_terms<KK>(st, inv_sd, ys, t);
    float mx = t[0];
#pragma unroll
    for (int k = 1; k < KK; ++k) mx = fmaxf(mx, t[k]);
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < KK; ++k) s += __expf(t[k] - mx);
    return lconst + mx + __logf(s);
}

template <int KK>
__device__ __forceinline__ float bt_factor(const float *st, float inv_sd, float lconst, float ys) {
    const float s = bt_plain_sum<KK>(st, inv_sd, ys);
    return s > kBtTiny ? lconst + __logf(s) : bt_shifted<KK>(st, inv_sd, lconst, ys);
}

// The factors of a thread's P particles for one datum: the plain sums first
// (no branch between the particles, so their arithmetic interleaves), then,
// only if some lane of the wave has a small sum, the shifted form for the
// particles that need it.  Each particle's value is bt_factor's.
template <int P, int KK>
__device__ __forceinline__ void bt_factors(const float (&st)[P][2 * KK], float inv_sd, float lconst, float ys,
                                           float (&f)[P]) {
    float s[P];
    bool small = false;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        s[p] = bt_plain_sum<KK>(st[p], inv_sd, ys);
        small = small || !(s[p] > kBtTiny);
    }
#pragma unroll
    for (int p = 0; p < P; ++p) f[p] = lconst + __logf(s[p]);
    if (__ballot(small)) {
#pragma unroll
        for (int p = 0; p < P; ++p)
            if (!(s[p] > kBtTiny)) f[p] = bt_shifted<KK>(st[p], inv_sd, lconst, ys);
    }
}

// ------------------------------------------------------- resample-move --
// The move step of ppl_smc_ex (see there and smc.hip) for a team's particles:
// after the resampling at factor s each particle takes M Metropolis-Hastings
// steps whose target is the posterior given y_0..y_s, with the mixture factor
// of this engine (FP32, summed in FP32 within blocks of 16 data and in FP64
// across them).  State: log pi_k at [k], mu_k at [KK + k].
template <int KK>
__device__ double bt_loglik_upto(const float *st, const float *__restrict__ y, int64_t s, float inv_sd,
                                 float lconst) {
    double tot = 0.0;
    float blk = 0.0f;
    int c = 0;
    for (int64_t d = 0; d <= s; ++d) {
        blk += bt_factor<KK>(st, inv_sd, lconst, y[d]);
        if (++c == 16) {
            tot += (double)blk;
            blk = 0.0f;
            c = 0;
        }
    }
    return tot + (double)blk;
}

template <int KK>
__device__ __forceinline__ double bt_log_prior(const float *st, float inv_mu_sd) {
    double l = 0.0;
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        const float r = st[KK + k] * inv_mu_sd;
        l += (double)st[k] - 0.5 * (double)(r * r);
    }
    return l;
}

struct BtMove {
    int M;
    float h_b, h_mu, inv_mu_sd, inv_sd, lconst;
    uint32_t c3;
    Key key;
    const float *y;
};

// One particle's moves; its state is read from and written back to g[f * stride].
template <int KK>
__device__ void bt_move(float *g, size_t stride, int64_t s, uint32_t j, BtMove mv, double *alpha_row,
                                     int64_t N) {
    float st[2 * KK];
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        st[k] = g[k * stride];
        st[KK + k] = g[(KK + k) * stride];
    }
    double ll = bt_loglik_upto<KK>(st, mv.y, s, mv.inv_sd, mv.lconst);
    double lp = bt_log_prior<KK>(st, mv.inv_mu_sd);
    for (int m = 0; m < mv.M; ++m) {
        float z[16];
#pragma unroll
        for (int b = 0; b < 4; ++b) normals4(philox(j, (uint32_t)(8 * m + b), (uint32_t)s, mv.c3, mv.key), z + 4 * b);
        const float v = unit_f32(philox(j, (uint32_t)(8 * m + 4), (uint32_t)s, mv.c3, mv.key).x);
        float st2[2 * KK];
        float mx = 0.0f;
#pragma unroll
        for (int k = 0; k < KK - 1; ++k) {
            st2[k] = fmaf(mv.h_b, z[k], st[k] - st[KK - 1]);
            mx = fmaxf(mx, st2[k]);
        }
        float se = expf(-mx);
#pragma unroll
        for (int k = 0; k < KK - 1; ++k) se += expf(st2[k] - mx);
        const float lse = mx + logf(se);
#pragma unroll
        for (int k = 0; k < KK - 1; ++k) st2[k] -= lse;
        st2[KK - 1] = -lse;
#pragma unroll
        for (int k = 0; k < KK; ++k) st2[KK + k] = fmaf(mv.h_mu, z[KK - 1 + k], st[KK + k]);
        const double ll2 = bt_loglik_upto<KK>(st2, mv.y, s, mv.inv_sd, mv.lconst);
        const double lp2 = bt_log_prior<KK>(st2, mv.inv_mu_sd);
        const double la = (ll2 + lp2) - (ll + lp);
        if (alpha_row) alpha_row[(size_t)m * N + j] = la;
        if (log((double)v) < la) {
#pragma unroll
            for (int k = 0; k < KK; ++k) {
                st[k] = st2[k];
                st[KK + k] = st2[KK + k];
            }
            ll = ll2;
            lp = lp2;
        }
    }
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        g[k * stride] = st[k];
        g[(KK + k) * stride] = st[KK + k];
    }
}

// One speculative block: advance every particle's log-weight over the tb
// data in ybuf and record, per factor, the wave's {max, s1, s2} of the
// log-weights in wpart (a NaN log-weight poisons s1).
template <int P, int KK>
__device__ __forceinline__ void bt_block_factors(const float (&st)[P][2 * KK], const bool (&valid)[P], float (&lw)[P],
                                                 float (&lwc)[P],
                                                 const float *ybuf, int tb, float inv_sd, float lconst,
                                                 float (*wpart)[kBtWaves][3], int wave, int lane) {
    for (int t = 0; t < tb; ++t) {
        const float ys = ybuf[t];
        float ml = -INFINITY;
        int nan_seen = 0;
        float f[P];
        bt_factors<P, KK>(st, inv_sd, lconst, ys, f);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (valid[p]) kahan_add(lw[p], lwc[p], f[p]);
            ml = fmaxf(ml, lw[p]);
            nan_seen |= isnan(lw[p]) ? 1 : 0;
        }
        const float mw = wave_max_dpp(ml);
        float s1 = 0.0f, s2 = 0.0f;
        if (mw > -INFINITY) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const float e = __expf(lw[p] - mw);
                s1 += e;
                s2 = fmaf(e, e, s2);
            }
        }
        s1 = wave_sum_dpp(s1);
        s2 = wave_sum_dpp(s2);
        if (__ballot(nan_seen != 0)) s1 = NAN;
        if (lane == 0) {
            wpart[t][wave][0] = mw;
            wpart[t][wave][1] = s1;
            wpart[t][wave][2] = s2;
        }
    }
}

// Recompute the log-weights over the block's first nt data (after a rollback).
template <int P, int KK>
__device__ __forceinline__ void bt_block_redo(const float (&st)[P][2 * KK], const bool (&valid)[P], float (&lw)[P],
                                              float (&lwc)[P],
                                              const float *ybuf, int nt, float inv_sd, float lconst) {
    for (int t = 0; t < nt; ++t) {
        const float ys = ybuf[t];
        float f[P];
        bt_factors<P, KK>(st, inv_sd, lconst, ys, f);
#pragma unroll
        for (int p = 0; p < P; ++p)
            if (valid[p]) kahan_add(lw[p], lwc[p], f[p]);
    }
}

// --------------------------------------------------------- LDS helpers ----
__device__ __forceinline__ float bt_block_max(float v, float *lds) {
    v = wave_max_dpp(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    float m = lds[0];
#pragma unroll
    for (int w = 1; w < kBtWaves; ++w) m = fmaxf(m, lds[w]);
    __syncthreads();
    return m;
}

// Sum over the workgroup (waves in a fixed order; lds: kBtWaves doubles).
__device__ __forceinline__ double bt_block_sum_f64(double v, double *lds) {
    v = wave_sum_dpp(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBtWaves; ++w) t += lds[w];
    __syncthreads();
    return t;
}

__device__ __forceinline__ uint64_t bt_block_exscan(uint64_t v, uint64_t *lds, uint64_t &total) {
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
    for (int w = 0; w < kBtWaves; ++w) {
        const uint64_t x = lds[w];
        if (w < wv) off += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return off + incl - v;
}

// Context a workgroup carries from one instance to the next: its place in
// the grid, the team's slices of the workspace and the kernel's LDS arrays.
struct BtCtx {
    int W, team, wg, lane, wave;
    unsigned epoch;
    bool alive;
    double *tpart2;
    uint64_t *ttot, *tfin, *tq;
    double *tesum;
    float *tx, *tx2;
    uint64_t *ldsu, *lds4;
    double *ldsd;
    float *ybuf;
    float (*wpart)[kBtWaves][3];
    float *sM;
    unsigned char *sBad;
    int *s_first, *s_rng;
    uint64_t *tile_end, *tile_pre, *stage;
    int32_t *s_anc;
    float *s_c0;
};

// One instance from its prior draw to its outputs, with the component count
// KK fixed at compile time: a particle's state takes 2 KK registers, so teams
// holding small-K instances keep eight particles per lane in registers.
template <int P, int KK, bool MOVES>
__device__ __forceinline__ void bt_instance(const BtDev &a, BtCtx &cx, int i) {
    const int W = cx.W, team = cx.team, wg = cx.wg, lane = cx.lane, wave = cx.wave;
    unsigned &epoch = cx.epoch;
    bool &alive = cx.alive;
    double *tpart2 = cx.tpart2;
    uint64_t *ttot = cx.ttot, *tfin = cx.tfin, *tq = cx.tq;
    double *tesum = cx.tesum;
    float *tx = cx.tx, *tx2 = cx.tx2;
    uint64_t *ldsu = cx.ldsu, *lds4 = cx.lds4;
    double *ldsd = cx.ldsd;
    float *ybuf = cx.ybuf;
    float (*wpart)[kBtWaves][3] = cx.wpart;
    float *sM = cx.sM;
    unsigned char *sBad = cx.sBad;
    int &s_first = *cx.s_first;
    int *s_rng = cx.s_rng;
    uint64_t *tile_end = cx.tile_end, *tile_pre = cx.tile_pre, *stage = cx.stage;
    int32_t *s_anc = cx.s_anc;
    float *s_c0 = cx.s_c0;
    constexpr int kTile = kBtThreads * P;
    const ppl_instance I = a.inst[i];
    const int64_t N = I.n_particles, D = I.n_data;
    const int K = I.dim;
    const float mu_sd = I.hyper[0] > 0 ? (float)I.hyper[0] : 5.0f;
    const double comp_sd = I.hyper[1] > 0 ? I.hyper[1] : 1.0;
    const float inv_sd = (float)(1.0 / comp_sd);
    const float lconst = (float)(-0.5 * log(2.0 * M_PI) - log(comp_sd));
    const uint32_t c3 = ((uint32_t)i << 8) | kTagPrior;
    // particle, data and event-record offsets of this instance in the concatenated outputs
    int64_t poff = 0, doff = 0, roff = 0, aoff = 0;
    for (int k = 0; k < i; ++k) {
        poff += a.inst[k].n_particles;
        doff += a.inst[k].n_data;
        if (!(a.inst[k].flags & PPL_INST_NO_RECORD)) {
            roff += a.inst[k].n_particles;
            aoff += (int64_t)a.inst[k].move_steps * a.inst[k].n_particles;
        }
    }
    const bool record = !(I.flags & PPL_INST_NO_RECORD);
    int c = 0;
    while (((int64_t)1 << c) < N) ++c;
    const int kbits = 62 - c;
    const int F = 64 + kbits;                    // fixed-point scale of the normaliser sums
    const double logN = bt_log((double)N);

    const int jb0 = wg * kTile + threadIdx.x * P;
    float st[P][2 * KK];
    float lw[P], lwc[P];     // log-weight and its compensation term
    bool valid[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        valid[p] = jb0 + p < N;
        bt_init<KK>((uint32_t)(jb0 + p), c3, a.key, mu_sd, st[p]);
        lw[p] = valid[p] ? 0.0f : -INFINITY;
        lwc[p] = 0.0f;
    }

    double logz = 0.0;
    int64_t nres = 0;
    int status = 0;
    float Mlast = 0.0f;
    int64_t t0 = 0;
    int B = 1;
    int64_t n_first = 0, n_redo = 0, n_blocks = 0;     // factors advanced, recomputed; speculative blocks
    while (t0 < D) {
        const int tb = (int)std::min<int64_t>(B, D - t0);
        n_first += tb;
        ++n_blocks;
        __syncthreads();
        for (int t = threadIdx.x; t < tb; t += kBtThreads) ybuf[t] = I.y[t0 + t];
        __syncthreads();
        // block-start log-weights, kept in LDS for a rollback (the ancestor
        // area is free until resampling, which only starts after the rollback)
        float *s_lw0 = (float *)s_anc;
        float *s_lwc0 = s_c0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            s_lw0[threadIdx.x * P + p] = lw[p];
            s_lwc0[threadIdx.x * P + p] = lwc[p];
        }
        bt_block_factors<P, KK>(st, valid, lw, lwc, ybuf, tb, inv_sd, lconst, wpart, wave, lane);
        __syncthreads();
        // workgroup partial per factor: merge the waves in order
        double *tpart = tpart2 + (size_t)((epoch + 1) & 1) * W * a.Bmax * 3;
        for (int t = threadIdx.x; t < tb; t += kBtThreads) {
            float m = -INFINITY;
            for (int w = 0; w < kBtWaves; ++w) m = fmaxf(m, wpart[t][w][0]);
            double s1 = 0.0, s2 = 0.0;
            if (m > -INFINITY) {
                for (int w = 0; w < kBtWaves; ++w) {
                    const float cw = expf(wpart[t][w][0] - m);
                    s1 += (double)wpart[t][w][1] * cw;
                    s2 += (double)wpart[t][w][2] * (double)(cw * cw);
                }
            }
            double *dst = tpart + ((size_t)wg * a.Bmax + t) * 3;
            dst[0] = (double)m;
            dst[1] = s1;
            dst[2] = s2;
        }
        if (!team_barrier(a.bar, team, ++epoch * (unsigned)W)) { alive = false; break; }
        // team merge per factor (same order in every workgroup) and the trigger
        if (threadIdx.x == 0) s_first = tb;
        __syncthreads();
        for (int t = threadIdx.x; t < tb; t += kBtThreads) {
            float m = -INFINITY;
            for (int w = 0; w < W; ++w) m = fmaxf(m, (float)tpart[((size_t)w * a.Bmax + t) * 3]);
            double s1 = 0.0, s2 = 0.0;
            if (m > -INFINITY) {
                for (int w = 0; w < W; ++w) {
                    const double *src = tpart + ((size_t)w * a.Bmax + t) * 3;
                    const float cw = expf((float)src[0] - m);
                    s1 += src[1] * cw;
                    s2 += src[2] * (double)(cw * cw);
                }
            }
            sM[t] = m;
            const double ess = s1 * s1 / s2;
            const bool bad = !(m > -INFINITY) || !(s1 > 0.0) || isnan(s1) || isnan(s2);
            sBad[t] = bad ? (m > -INFINITY ? 2 : 1) : 0;
            const bool trig = bad || ((t0 + t < D - 1) && ess < (double)a.ess_frac * (double)N);
            if (wg == 0 && a.ess_tr) a.ess_tr[doff + t0 + t] = bad ? 0.0 : ess;
            if (trig) atomicMin(&s_first, t);
        }
        __syncthreads();
        const int tf = s_first;
        if (tf == tb) {                    // no trigger: commit the block
            if (wg == 0 && a.res_tr)
                for (int t = threadIdx.x; t < tb; t += kBtThreads) a.res_tr[doff + t0 + t] = 0;
            if (wg == 0 && a.logz_tr)
                for (int t = threadIdx.x; t < tb; t += kBtThreads) a.logz_tr[doff + t0 + t] = 0.0;
            Mlast = sM[tb - 1];
            t0 += tb;
            B = std::min(2 * B, a.Bmax);
            continue;
        }
        const float Mg = sM[tf];
        if (sBad[tf]) {                    // the same verdict in every workgroup of the team
            status = sBad[tf] == 1 ? PPL_E_ZERO_WEIGHT : PPL_E_NONFINITE;
            break;
        }
        if (wg == 0 && a.res_tr)
            for (int t = threadIdx.x; t <= tf; t += kBtThreads) a.res_tr[doff + t0 + t] = t == tf ? 1 : 0;
        if (wg == 0 && a.logz_tr)
            for (int t = threadIdx.x; t < tf; t += kBtThreads) a.logz_tr[doff + t0 + t] = 0.0;
        // roll back to the block start and recompute up to factor tf
        if (tf < tb - 1) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                lw[p] = s_lw0[threadIdx.x * P + p];
                lwc[p] = s_lwc0[threadIdx.x * P + p];
            }
            bt_block_redo<P, KK>(st, valid, lw, lwc, ybuf, tf + 1, inv_sd, lconst);
            n_redo += tf + 1;
        }
        // ---- resampling at factor s = t0 + tf
        const int64_t s = t0 + tf;
        // The state goes to the staging buffer first: it is dead in registers
        // until the gather refills it, which keeps the scan below out of scratch.
        int jb = jb0;
        asm volatile("" : "+v"(jb));
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (valid[p]) {
#pragma unroll
                for (int f = 0; f < 2 * KK; ++f) tx[(size_t)f * a.cap + jb + p] = st[p][f];
                if (a.elw_out && record && nres < a.max_events)
                    a.elw_out[(size_t)a.max_events * roff + (size_t)nres * N + jb + p] = lw[p];
            }
        }
        // integer weights q = floor(e 2^k) and the next 32 bits of each, r =
        // floor(frac(e 2^k) 2^32): the normaliser is (sum q + 2^-32 sum r) 2^-k,
        // where sum q is the resampling total S and sum r is exact in FP64
        // (integers below 2^50 in any grouping), so it does not depend on the
        // launch shape
        uint64_t q[P];
        uint64_t run = 0;
        double rsum = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const double e = valid[p] ? bt_exp((double)lw[p] - (double)Mg) : 0.0;
            if (e >= 0.0) {
                const double x = ldexp(e, kbits), xi = floor(x);
                run += (uint64_t)xi;
                rsum += floor(ldexp(x - xi, 32));
            }
            q[p] = run;
        }
        uint64_t btot;
        const uint64_t off = bt_block_exscan(run, ldsu, btot);
#pragma unroll
        for (int p = 0; p < P; ++p)
            if (valid[p]) tq[jb + p] = off + q[p];
        rsum = bt_block_sum_f64(rsum, ldsd);
        if (threadIdx.x == 0) {
            ttot[wg] = btot;
            tesum[wg] = rsum;
        }
        if (!team_barrier(a.bar, team, ++epoch * (unsigned)W)) { alive = false; break; }
        {
            const uint64_t v = threadIdx.x < W ? ttot[threadIdx.x] : 0;
            const double rv = threadIdx.x < W ? tesum[threadIdx.x] : 0.0;
            uint64_t S;
            const uint64_t ex = bt_block_exscan(v, ldsu, S);
            if (threadIdx.x < W) {
                tile_pre[threadIdx.x] = ex;
                tile_end[threadIdx.x] = ex + v;
            }
            const double R = bt_block_sum_f64(rv, ldsd);
            const uint4 rw = philox(0, 0, (uint32_t)s, ((uint32_t)i << 8) | kTagResample, a.key);
            const uint64_t U = __umul64hi(((uint64_t)rw.y << 32) | rw.x, S);
            const double ev = ldexp((double)S, -kbits) + ldexp(R, -(kbits + 32));
            const double inc = (double)Mg + bt_log(ev) - logN;
            logz += inc;
            if (a.logz_tr && wg == 0 && threadIdx.x == 0) a.logz_tr[doff + s] = inc;
            ++nres;
            const uint64_t NN = (uint64_t)N;
            const uint64_t Sq = S / NN, Sr = S - Sq * NN;
            // ancestors: min{a : Q_a > tau_j}, tau_j = j Sq + floor((j Sr + U) / N)
            const int js0 = wg * kTile;
            const int js1 = (int)std::min<int64_t>((int64_t)js0 + kTile, N) - 1;
            if (js0 < N) {
                for (int e = 0; e < 2; ++e) {
                    if (threadIdx.x == 64 * e) {
                        const int jj = e ? js1 : js0;
                        const uint64_t num = (uint64_t)jj * Sr + U;
                        const uint64_t tau = (uint64_t)jj * Sq + num / NN;
                        int lo = 0, hi = W - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (tile_end[mid] > tau) hi = mid; else lo = mid + 1;
                        }
                        int a0 = lo * kTile, a1 = (int)std::min<int64_t>((int64_t)a0 + kTile, N) - 1;
                        while (a0 < a1) {
                            const int mid = (a0 + a1) >> 1;
                            if (tile_pre[lo] + tq[mid] > tau) a1 = mid; else a0 = mid + 1;
                        }
                        s_rng[e] = a0;
                    }
                }
            }
            __syncthreads();
            if (js0 < N) {
                const int a_lo = s_rng[0], a_hi = s_rng[1];
                const int span = a_hi - a_lo + 1;
                const bool staged = span <= a.stage_cap;
                int32_t *anc_row = (a.anc_out && record && nres - 1 < a.max_events)
                                       ? a.anc_out + (size_t)a.max_events * roff + (size_t)(nres - 1) * N
                                       : nullptr;
                if (staged)
                    for (int k = threadIdx.x; k < span; k += kBtThreads) {
                        const int aa = a_lo + k;
                        stage[k] = tile_pre[aa / kTile] + tq[aa];
                    }
                __syncthreads();
                int prev = a_lo;
                uint64_t num = (uint64_t)jb * Sr + U;
                uint64_t quo = num / NN, rem = num - quo * NN;
#pragma unroll 1
                for (int p = 0; p < P; ++p) {
                    const int j = jb + p;
                    if (j >= N) break;
                    if (p) {
                        rem += Sr;
                        if (rem >= NN) { rem -= NN; ++quo; }
                    }
                    const uint64_t tau = (uint64_t)j * Sq + quo;
                    int anc;
                    if (staged) {
                        int lo = prev - a_lo, hi = span - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (stage[mid] > tau) hi = mid; else lo = mid + 1;
                        }
                        anc = a_lo + lo;
                    } else {
                        int lo = prev / kTile, hi = W - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (tile_end[mid] > tau) hi = mid; else lo = mid + 1;
                        }
                        int a0 = std::max(lo * kTile, prev), a1 = (int)std::min<int64_t>((int64_t)lo * kTile + kTile, N) - 1;
                        while (a0 < a1) {
                            const int mid = (a0 + a1) >> 1;
                            if (tile_pre[lo] + tq[mid] > tau) a1 = mid; else a0 = mid + 1;
                        }
                        anc = a0;
                    }
                    s_anc[threadIdx.x * P + p] = anc;
                    if (anc_row) anc_row[j] = anc;
                    prev = anc;
                }
            } else {
                __syncthreads();
            }
        }
        if (!MOVES || I.move_steps == 0) {
            // gather (slots past N take zeros: their state is never used)
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int anc = valid[p] ? s_anc[threadIdx.x * P + p] : 0;
#pragma unroll
                for (int f = 0; f < 2 * KK; ++f) st[p][f] = valid[p] ? tx[(size_t)f * a.cap + anc] : 0.0f;
                if (valid[p]) lw[p] = 0.0f;
                lwc[p] = 0.0f;
            }
        } else if constexpr (MOVES) {
            // resample-move: the gathered particles go through memory one at a
            // time, so only the moving particle's state occupies registers
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (!valid[p]) continue;
                const int anc = s_anc[threadIdx.x * P + p];
#pragma unroll
                for (int f = 0; f < 2 * KK; ++f) tx2[(size_t)f * a.cap + jb + p] = tx[(size_t)f * a.cap + anc];
                lw[p] = 0.0f;
                lwc[p] = 0.0f;
            }
            const double nd = (double)(s + 1);
            const double lam = I.move_scale > 0.0 ? I.move_scale : 2.38 / sqrt(2.0 * K - 1.0);
            BtMove mv;
            mv.M = I.move_steps;
            mv.h_mu = (float)(lam / sqrt(1.0 / ((double)mu_sd * (double)mu_sd) + nd / ((double)K * comp_sd * comp_sd)));
            mv.h_b = (float)(lam / sqrt(3.0 / (M_PI * M_PI) + nd / (2.0 * K)));
            mv.inv_mu_sd = 1.0f / mu_sd;
            mv.inv_sd = inv_sd;
            mv.lconst = lconst;
            mv.c3 = ((uint32_t)i << 8) | kTagMove;
            mv.key = a.key;
            mv.y = I.y;
            double *arow = (a.alpha_out && record && nres - 1 < a.max_events)
                               ? a.alpha_out + (size_t)a.max_events * aoff + (size_t)(nres - 1) * I.move_steps * N
                               : nullptr;
#pragma unroll 1
            for (int p = 0; p < P; ++p) {
                const int j = jb + p;
                if (j >= N) break;
                float *g = tx2 + j;
                bt_move<KK>(g, (size_t)a.cap, s, (uint32_t)j, mv, arow, N);
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
#pragma unroll
                for (int f = 0; f < 2 * KK; ++f) st[p][f] = valid[p] ? tx2[(size_t)f * a.cap + jb + p] : 0.0f;
            }
        }
        t0 = s + 1;
        B = 1;
    }

    // ---- final normaliser over the last epoch
    double ess_final = (double)N;
    if (alive && status == 0 && D > 0) {
        uint64_t h1 = 0, l1 = 0, h2 = 0, l2 = 0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (valid[p]) {
                const double e = bt_exp((double)lw[p] - (double)Mlast);
                bt_fix_add(h1, l1, e, kbits);
                bt_fix_add(h2, l2, e * e, kbits);
            }
        }
        u128 e1 = ((u128)h1 << 64) | l1, e2 = ((u128)h2 << 64) | l2;
        bt_block_sum_u128x2(e1, e2, lds4);
        if (threadIdx.x == 0) {
            tfin[4 * wg] = (uint64_t)e1;
            tfin[4 * wg + 1] = (uint64_t)(e1 >> 64);
            tfin[4 * wg + 2] = (uint64_t)e2;
            tfin[4 * wg + 3] = (uint64_t)(e2 >> 64);
        }
        if (!team_barrier(a.bar, team, ++epoch * (unsigned)W)) {
            alive = false;
        } else {
            const int w = threadIdx.x;
            u128 t1 = w < W ? (((u128)tfin[4 * w + 1] << 64) | tfin[4 * w]) : 0;
            u128 t2 = w < W ? (((u128)tfin[4 * w + 3] << 64) | tfin[4 * w + 2]) : 0;
            bt_block_sum_u128x2(t1, t2, lds4);
            const double s1 = bt_unfix(t1, F), s2 = bt_unfix(t2, F);
            const double inc = (double)Mlast + bt_log(s1) - logN;
            logz += inc;
            if (a.logz_tr && wg == 0 && threadIdx.x == 0) a.logz_tr[doff + D - 1] = inc;
            ess_final = s1 * s1 / s2;
        }
    }
    if (!alive) status = PPL_E_HIP;
    // outputs
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (!valid[p]) continue;
        const int64_t j = jb0 + p;
        if (a.lw_out) a.lw_out[poff + j] = lw[p];
        if (a.lat_out) {
#pragma unroll
            for (int f = 0; f < 2 * KK; ++f) a.lat_out[(size_t)kBtNF * poff + (size_t)f * N + j] = st[p][f];
        }
    }
    if (a.counters && wg == 0 && threadIdx.x == 0) {
        atomicAdd(&a.counters[0], (unsigned long long)(n_first * N));
        atomicAdd(&a.counters[1], (unsigned long long)(n_redo * N));
        atomicAdd(&a.counters[2], (unsigned long long)n_blocks);
        atomicAdd(&a.counters[3], (unsigned long long)nres);
    }
    if (wg == 0 && threadIdx.x == 0) {
        double *o = a.out + 4 * (size_t)i;
        o[0] = status ? (status == PPL_E_ZERO_WEIGHT ? -INFINITY : NAN) : logz;
        o[1] = status ? 0.0 : ess_final;
        o[2] = (double)nres;
        o[3] = (double)status;
    }
    // all workgroups of the team leave the instance together before its buffers are reused
    if (alive && !team_barrier(a.bar, team, ++epoch * (unsigned)W)) alive = false;
}

// ---------------------------------------------------------------- kernel --
// MOVES: the resample-move instantiation (a separate kernel, so the moves'
// registers never add to the plain engine's).
template <int P, bool MOVES>
__global__ __launch_bounds__(kBtThreads) void smc_batched_kernel(BtDev a) {
    __shared__ uint64_t ldsu[kBtWaves];
    __shared__ uint64_t lds4[4 * kBtWaves];
    __shared__ double ldsd[kBtWaves];
    __shared__ float ybuf[kBtMaxB];
    __shared__ float wpart[kBtMaxB][kBtWaves][3];     // per-factor wave partials {max, s1, s2}
    __shared__ float sM[kBtMaxB];                      // merged max per factor
    __shared__ unsigned char sBad[kBtMaxB];            // 1: all weights zero, 2: NaN
    __shared__ int s_first;                            // first triggering factor in the block
    __shared__ int s_rng[2];
    __shared__ uint64_t tile_end[kBtMaxW], tile_pre[kBtMaxW];
    extern __shared__ uint64_t dyn[];                  // stage[stage_cap] | s_anc[kBtThreads P] | s_c0[kBtThreads P]
    uint64_t *stage = dyn;
    int32_t *s_anc = (int32_t *)(dyn + a.stage_cap);
    float *s_c0 = (float *)(s_anc + kBtThreads * P);

    const int W = a.W;
    const int team = blockIdx.x / W, wg = blockIdx.x % W;

    // Per-factor partials have two copies, used alternately by consecutive block
    // barriers (copy = parity of the barrier epoch the writes precede).  After a
    // committed block a workgroup writes the next block's partials while a
    // slower one may still be merging this block's; the copies keep them apart.
    // Reuse of a copy is two barriers later, which every workgroup has passed
    // only after all merges of the earlier block are done.
    BtCtx cx;
    cx.W = W;
    cx.team = team;
    cx.wg = wg;
    cx.lane = threadIdx.x & 63;
    cx.wave = threadIdx.x >> 6;
    cx.epoch = 0;
    cx.alive = true;
    cx.tpart2 = a.part + (size_t)team * 2 * W * a.Bmax * 3;
    cx.ttot = a.tot + (size_t)team * W;
    cx.tesum = a.esum + (size_t)team * W;
    cx.tfin = a.fin + (size_t)team * W * 4;
    cx.tq = a.qloc + (size_t)team * a.cap;
    cx.tx = a.xbuf + (size_t)team * kBtNF * a.cap;
    cx.tx2 = a.xbuf2 + (size_t)team * kBtNF * a.cap;
    cx.ldsu = ldsu;
    cx.lds4 = lds4;
    cx.ldsd = ldsd;
    cx.ybuf = ybuf;
    cx.wpart = wpart;
    cx.sM = sM;
    cx.sBad = sBad;
    cx.s_first = &s_first;
    cx.s_rng = s_rng;
    cx.tile_end = tile_end;
    cx.tile_pre = tile_pre;
    cx.stage = stage;
    cx.s_anc = s_anc;
    cx.s_c0 = s_c0;

    for (int idx = a.team_off[team]; idx < a.team_off[team + 1] && cx.alive; ++idx) {
        const int i = a.order[idx];
        switch (a.inst[i].dim) {   // the same for every thread of the team
            case 1: bt_instance<P, 1, MOVES>(a, cx, i); break;
            case 2: bt_instance<P, 2, MOVES>(a, cx, i); break;
            case 3: bt_instance<P, 3, MOVES>(a, cx, i); break;
            case 4: bt_instance<P, 4, MOVES>(a, cx, i); break;
            case 5: bt_instance<P, 5, MOVES>(a, cx, i); break;
            case 6: bt_instance<P, 6, MOVES>(a, cx, i); break;
            case 7: bt_instance<P, 7, MOVES>(a, cx, i); break;
            case 8: bt_instance<P, 8, MOVES>(a, cx, i); break;
        }
    }
}


__global__ void smc_batched_reset_kernel(unsigned *bar, int words, unsigned long long *counters) {
    for (int i = threadIdx.x; i < words; i += blockDim.x) bar[i] = 0u;
    if (counters && threadIdx.x < 4) counters[threadIdx.x] = 0ull;
}

// ------------------------------------------------------------------ host --
struct BtLayout {
    unsigned *bar;
    double *part;
    double *esum;
    uint64_t *fin;
    uint64_t *tot, *qloc;
    float *xbuf, *xbuf2;
    size_t bytes;
};

static BtLayout bt_layout(void *ws, int teams, int W, int Bmax, int64_t cap) {
    BtLayout L;
    char *p = (char *)ws;
    size_t o = 0;
    auto take = [&](size_t n) { char *r = p + o; o += align_up(n, 256); return r; };
    L.bar = (unsigned *)take((size_t)kBtBarLine * (1 + teams) * sizeof(unsigned));
    L.part = (double *)take((size_t)teams * 2 * W * Bmax * 3 * sizeof(double));
    L.esum = (double *)take((size_t)teams * W * sizeof(double));
    L.fin = (uint64_t *)take((size_t)teams * W * 4 * sizeof(uint64_t));
    L.tot = (uint64_t *)take((size_t)teams * W * sizeof(uint64_t));
    L.qloc = (uint64_t *)take((size_t)teams * cap * sizeof(uint64_t));
    L.xbuf = (float *)take((size_t)teams * kBtNF * cap * sizeof(float));
    L.xbuf2 = (float *)take((size_t)teams * kBtNF * cap * sizeof(float));
    L.bytes = o;
    return L;
}

static int device_cus(int &ncu) {
    int dev = 0;
    PPL_HIP(hipGetDevice(&dev));
    PPL_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    return PPL_OK;
}

// Resolved configuration: P and W chosen so that a team covers the largest instance.
static int bt_resolve(const ppl_instance *h, int n, const ppl_tune *tune, int ncu, ppl_tune &cfg, int &teams,
                      int64_t &cap) {
    int64_t nmax = 1;
    for (int i = 0; i < n; ++i) nmax = std::max<int64_t>(nmax, h[i].n_particles);
    cfg.particles_per_lane = tune && tune->particles_per_lane ? tune->particles_per_lane : 4;
    cfg.spec_block = tune && tune->spec_block ? tune->spec_block : 64;
    const int P = cfg.particles_per_lane;
    if (P != 1 && P != 2 && P != 4 && P != 8) return fail(PPL_E_ARG, "particles_per_lane must be 1, 2, 4 or 8");
    if (cfg.spec_block < 1 || cfg.spec_block > kBtMaxB) return fail(PPL_E_ARG, "spec_block must be in 1..%d", kBtMaxB);
    const int64_t need = (nmax + (int64_t)kBtThreads * P - 1) / ((int64_t)kBtThreads * P);
    int W = tune && tune->wgs_per_instance ? tune->wgs_per_instance : (int)need;
    if (W < need) return fail(PPL_E_ARG, "wgs_per_instance %d cannot hold %lld particles at %d per lane", W,
                              (long long)nmax, P);
    if (W > kBtMaxW || W > ncu) return fail(PPL_E_UNSUPPORTED, "an instance of %lld particles needs %d workgroups",
                                            (long long)nmax, W);
    cfg.wgs_per_instance = W;
    teams = std::min(ncu / W, kBtMaxTeams);
    teams = std::max(1, std::min(teams, n));
    cap = (int64_t)W * kBtThreads * P;
    return PPL_OK;
}

size_t bt_ws_bytes_for(const ppl_instance *h, int n, const ppl_tune *tune) {
    int ncu = 256;
    if (device_cus(ncu) != PPL_OK) ncu = 256;
    ppl_tune cfg;
    int teams;
    int64_t cap;
    if (bt_resolve(h, n, tune, ncu, cfg, teams, cap) != PPL_OK) return 0;
    return bt_layout(nullptr, teams, cfg.wgs_per_instance, cfg.spec_block, cap).bytes;
}

int bt_check(int model, int n, const ppl_instance *h) {
    if (model != PPL_MODEL_GMM) return fail(PPL_E_MODEL, "batched SMC supports the mixture model (got %d)", model);
    if (n < 1 || n > kBtMaxInst) return fail(PPL_E_ARG, "n_inst must be in 1..%d", kBtMaxInst);
    if (!h) return fail(PPL_E_ARG, "host instance table is NULL");
    for (int i = 0; i < n; ++i) {
        const ppl_instance &I = h[i];
        if (I.n_particles < 1 || I.n_particles > (1LL << 30)) return fail(PPL_E_ARG, "instance %d: bad particle count", i);
        if (I.n_data < 0 || I.n_data > 0x7fffffffLL) return fail(PPL_E_ARG, "instance %d: bad data length", i);
        if (I.n_data > 0 && !I.y) return fail(PPL_E_ARG, "instance %d: y is NULL", i);
        if (I.dim < 1 || I.dim > 8) return fail(PPL_E_ARG, "instance %d: K must be in 1..8", i);
        if (I.move_steps < 0 || I.move_steps > 64) return fail(PPL_E_ARG, "instance %d: move_steps must be in 0..64", i);
        if (!(I.move_scale >= 0.0) || !isfinite(I.move_scale))
            return fail(PPL_E_ARG, "instance %d: move_scale must be finite and >= 0", i);
        if (!(I.hyper[0] >= 0) || !(I.hyper[1] >= 0) || !isfinite(I.hyper[0]) || !isfinite(I.hyper[1]))
            return fail(PPL_E_ARG, "instance %d: hyper-parameters must be finite and non-negative (0 = default)", i);
    }
    return PPL_OK;
}

template <int P>
static int bt_launch(BtDev &d, int nblocks, hipStream_t st) {
    auto kern = d.any_moves ? smc_batched_kernel<P, true> : smc_batched_kernel<P, false>;
    int dev = 0, ncu = 0, occ = 0, max_lds = 0;
    PPL_HIP(hipGetDevice(&dev));
    PPL_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    PPL_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    hipFuncAttributes fa;
    PPL_HIP(hipFuncGetAttributes(&fa, (const void *)kern));
    const int64_t fixed = (int64_t)fa.sharedSizeBytes + (int64_t)kBtThreads * P * 2 * sizeof(int32_t);
    d.stage_cap = (int)std::max<int64_t>(0, std::min<int64_t>(kBtStage, (max_lds - fixed) / 8));
    const size_t lds = (size_t)d.stage_cap * sizeof(uint64_t) + (size_t)kBtThreads * P * 2 * sizeof(int32_t);
    PPL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kBtThreads, lds));
    if ((int64_t)occ * ncu < nblocks)
        return fail(PPL_E_UNSUPPORTED, "batched SMC needs %d co-resident workgroups, device holds %d", nblocks, occ * ncu);
    void *args[] = {&d};
    KernelTimer timer("smc_batched_kernel", st);
    PPL_HIP(hipLaunchCooperativeKernel((const void *)kern, dim3((unsigned)nblocks), dim3(kBtThreads), args, lds, st));
    timer.stop();
    return PPL_OK;
}

int run_smc_batched(int n, const ppl_instance *h, const ppl_instance *d_inst, uint64_t seed, double ess_frac,
                    const ppl_tune *tune, void *ws, size_t ws_bytes, hipStream_t st, const ppl_batch_result &out,
                    ppl_tune *used) {
    int ncu = 0;
    if (int rc = device_cus(ncu)) return rc;
    ppl_tune cfg;
    int teams;
    int64_t cap;
    if (int rc = bt_resolve(h, n, tune, ncu, cfg, teams, cap)) return rc;
    const int W = cfg.wgs_per_instance;
    BtLayout L = bt_layout(ws, teams, W, cfg.spec_block, cap);
    if (ws_bytes < L.bytes) return fail(PPL_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, L.bytes);
    // longest-processing-time-first assignment of instances to teams
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    auto work = [&](int i) { return (double)h[i].n_particles * (double)h[i].n_data * (h[i].dim + 2); };
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return work(x) > work(y); });
    std::vector<std::vector<int>> lists(teams);
    std::vector<double> load(teams, 0.0);
    for (int i : ord) {
        const int t = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        lists[t].push_back(i);
        load[t] += work(i) + 1.0;
    }
    static_assert(sizeof(BtDev) <= 4096, "kernel argument block too large");
    BtDev d{};
    int pos = 0;
    for (int t = 0; t < teams; ++t) {
        d.team_off[t] = (uint16_t)pos;
        for (int i : lists[t]) d.order[pos++] = (uint16_t)i;
    }
    d.team_off[teams] = (uint16_t)pos;
    d.inst = d_inst;
    d.n_inst = n;
    for (int i = 0; i < n; ++i) d.any_moves |= h[i].move_steps > 0 ? 1 : 0;
    d.key = make_key(seed);
    d.ess_frac = (float)ess_frac;
    d.W = W;
    d.Bmax = cfg.spec_block;
    d.cap = cap;
    d.out = out.d_out;
    d.lw_out = out.d_log_weights;
    d.lat_out = out.d_latents;
    d.ess_tr = out.d_ess_trace;
    d.res_tr = out.d_resampled;
    d.anc_out = out.d_ancestors;
    d.elw_out = out.d_event_lw;
    d.logz_tr = out.d_logz_trace;
    d.alpha_out = out.d_move_log_alpha;
    d.max_events = (out.d_ancestors || out.d_event_lw || out.d_move_log_alpha) ? out.max_events : 0;
    d.counters = (unsigned long long *)out.d_counters;
    d.bar = L.bar;
    d.part = L.part;
    d.tot = L.tot;
    d.esum = L.esum;
    d.fin = L.fin;
    d.qloc = L.qloc;
    d.xbuf = L.xbuf;
    d.xbuf2 = L.xbuf2;
    hipLaunchKernelGGL(smc_batched_reset_kernel, dim3(1), dim3(256), 0, st, L.bar, kBtBarLine * (1 + teams),
                       (unsigned long long *)out.d_counters);
    PPL_LAUNCH_CHECK("smc_batched_reset_kernel");
    if (used) *used = cfg;
    const int nblocks = teams * W;
    switch (cfg.particles_per_lane) {
        case 1: return bt_launch<1>(d, nblocks, st);
        case 2: return bt_launch<2>(d, nblocks, st);
        case 4: return bt_launch<4>(d, nblocks, st);
        case 8: return bt_launch<8>(d, nblocks, st);
    }
    return fail(PPL_E_ARG, "particles_per_lane must be 1, 2, 4 or 8");
}

}  // namespace ppl
