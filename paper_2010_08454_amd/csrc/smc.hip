// smc.hip -- sequential Monte Carlo in one persistent cooperative launch.
//
// The paper suspends a model at each factor with a delimited continuation
// (Sec. 3.4, 4.3) and names particle-based inference on the GPU as future work
// (Sec. 6).  Here a suspended particle is its resume point (the factor index s,
// shared by all particles) plus fixed-size state held in registers across the
// whole run; only resampling moves state through HBM.
//
// One workgroup of 1024 threads per CU, P particles per thread (slots
// j = block * 1024 P + thread * P + p).  Per factor s:
//   1. every particle advances to factor s and adds its log-factor (FP32);
//   2. block partial {max lw, sum e, sum e^2}, e = exp(lw - max) -> HBM;
//      grid barrier; every block merges the partials in the same order, so
//      all blocks take the same ESS decision;
//   3. if ESS < ess_frac N (and s is not the last factor): FP64 weights
//      e = exp(lw - max) give the epoch normaliser and the quantised integer
//      weights q; each block scans its q, publishes tile totals, its state
//      and its local scan; grid barrier; each slot finds its ancestor
//      (binary search over tile ends, then inside the tile) and gathers the
//      ancestor's state; lw = 0.
// The grid barrier is a monotone counter with a bounded spin: if a wait ever
// exceeds the limit, the block raises the abort flag and every block leaves
// its loop at its next barrier, so the grid always drains.
#include <math.h>
#include <string.h>

#include "device.h"
#include "host.h"
#include "smc.h"
#include "timing.h"

namespace ppl {

constexpr int kSmcThreads = 1024;
constexpr int kSmcWaves = kSmcThreads / 64;
constexpr uint32_t kSpinLimit = 1u << 24;     // ~1 s of s_sleep(2) per barrier wait

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
    // outputs (may be null)
    double *scalars;
    float *lw_out, *lat_out;
    double *ess_trace;
    uint8_t *resampled;
    int32_t *anc_out;
    int64_t max_events;
    // workspace
    unsigned *bar;           // [0] barrier counter, [1] abort flag
    double *part;            // [2][nb][3]
    uint64_t *tot;           // [nb]
    double *esum;            // [nb]
    double *fin;             // [nb][2]
    uint64_t *qloc;          // [N]
    float *xbuf;             // [NF][N]
};

// ------------------------------------------------------------- barrier --
// Returns false (uniformly in the block) once any block has aborted.
__device__ __forceinline__ bool grid_barrier(unsigned *bar, unsigned target) {
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        int ok = 1;
        while (__hip_atomic_load(&bar[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
            __builtin_amdgcn_s_sleep(2);
            if (++spins > kSpinLimit) {
                __hip_atomic_store(&bar[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
        if (ok && __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
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
    // Noise of slot j at factor s is normal (s mod 4) of block (j, 0, s div 4).
    __device__ static float step(const SmcDev &a, int64_t s, uint32_t j, float st[NF], float zc[4], float ys) {
        if ((s & 3) == 0) normals4(philox(j, 0, (uint32_t)(s >> 2), (a.inst << 8) | kTagPrior, a.key), zc);
        const float x = fmaf(a.hyp[0], st[0], a.hyp[1] * zc[s & 3]);
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
    __device__ static float step(const SmcDev &a, int64_t, uint32_t, float st[NF], float *, float ys) {
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

// ------------------------------------------------------ block helpers --
__device__ __forceinline__ float block_max_f32(float v, float *lds) {
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    float m = lds[0];
#pragma unroll
    for (int w = 1; w < kSmcWaves; ++w) m = fmaxf(m, lds[w]);
    __syncthreads();
    return m;
}

__device__ __forceinline__ double block_sum_f64(double v, double *lds) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kSmcWaves; ++w) s += lds[w];
    __syncthreads();
    return s;
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
__device__ __forceinline__ void merge_partials(const double *part, int nb, float *ldsf, double *ldsd,
                                               float &M, double &S1, double &S2) {
    float m = -INFINITY;
    for (int b = threadIdx.x; b < nb; b += kSmcThreads) m = fmaxf(m, (float)part[3 * b]);
    M = block_max_f32(m, ldsf);
    double s1 = 0.0, s2 = 0.0;
    if (M > -INFINITY) {
        for (int b = threadIdx.x; b < nb; b += kSmcThreads) {
            const float mb = (float)part[3 * b];
            const float c = expf(mb - M);
            s1 += part[3 * b + 1] * (double)c;
            s2 += part[3 * b + 2] * (double)(c * c);
        }
    }
    S1 = block_sum_f64(s1, ldsd);
    S2 = block_sum_f64(s2, ldsd);
}

// (ahi:alo) > (bhi:blo) for 128-bit values split in 64-bit halves.
__device__ __forceinline__ bool gt128(uint64_t ahi, uint64_t alo, uint64_t bhi, uint64_t blo) {
    return ahi > bhi || (ahi == bhi && alo > blo);
}

// Ancestor of slot j: min{a : N Q_a > j S + U}, with Q_a = (tile_end[b] - tot[b]) + qloc[a]
// for a in tile b.  `prev` (the previous slot's ancestor, or -1) bounds the search
// from below, since ancestors are non-decreasing in j.
__device__ __forceinline__ int find_ancestor(uint32_t j, uint64_t S, uint64_t U, uint64_t N, int nb, int tile,
                                             const uint64_t *tile_end, const uint64_t *__restrict__ tot,
                                             const uint64_t *__restrict__ qloc, int prev) {
    const uint64_t tl0 = (uint64_t)j * S;
    const uint64_t tlo = tl0 + U;
    const uint64_t thi = __umul64hi((uint64_t)j, S) + (tlo < tl0 ? 1 : 0);
    if (prev >= 0) {
        const uint64_t q = tile_end[prev / tile] - tot[prev / tile] + qloc[prev];
        if (gt128(__umul64hi(N, q), N * q, thi, tlo)) return prev;
    }
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const uint64_t q = tile_end[mid];
        if (gt128(__umul64hi(N, q), N * q, thi, tlo)) hi = mid; else lo = mid + 1;
    }
    const uint64_t pre = tile_end[lo] - tot[lo];
    int a0 = lo * tile, a1 = a0 + tile - 1;
    if (a1 > (int)N - 1) a1 = (int)N - 1;
    if (prev >= a0) a0 = prev + 1;
    while (a0 < a1) {
        const int mid = (a0 + a1) >> 1;
        const uint64_t q = pre + qloc[mid];
        if (gt128(__umul64hi(N, q), N * q, thi, tlo)) a1 = mid; else a0 = mid + 1;
    }
    return a0;
}

// ---------------------------------------------------------------- kernel --
template <class M, int P>
__global__ __launch_bounds__(kSmcThreads) void smc_persistent_kernel(SmcDev a) {
    __shared__ float ldsf[kSmcWaves];
    __shared__ double ldsd[kSmcWaves];
    __shared__ uint64_t ldsu[kSmcWaves];
    extern __shared__ uint64_t tile_end[];          // [nb] inclusive tile ends (resampling)

    const int nb = gridDim.x;
    const int64_t N = a.N;
    const int64_t base = (int64_t)blockIdx.x * kSmcThreads * P + (int64_t)threadIdx.x * P;

    float st[P][M::NF];
    float lw[P];
    float zc[P][4];
    bool valid[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        valid[p] = base + p < N;
        M::init(a, (uint32_t)(base + p), st[p]);
        lw[p] = valid[p] ? 0.0f : -INFINITY;
    }

    unsigned epoch = 0;
    double logz = 0.0;
    int64_t nres = 0;
    int status = 0;
    float Mlast = 0.0f;
    bool alive = true;
    const double logN = log((double)N);

    for (int64_t s = 0; s < a.T; ++s) {
        const float ys = a.y[s];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const float f = M::step(a, s, (uint32_t)(base + p), st[p], zc[p], ys);
            if (valid[p]) lw[p] += f;
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
        const double s1b = block_sum_f64((double)s1l, ldsd);
        const double s2b = block_sum_f64((double)s2l, ldsd);
        double *pp = a.part + (size_t)(s & 1) * nb * 3;
        if (threadIdx.x == 0) {
            pp[3 * blockIdx.x] = (double)mb;
            pp[3 * blockIdx.x + 1] = s1b;
            pp[3 * blockIdx.x + 2] = s2b;
        }
        if (!grid_barrier(a.bar, ++epoch * (unsigned)nb)) { alive = false; status = PPL_E_HIP; break; }

        float Mg;
        double S1, S2;
        merge_partials(pp, nb, ldsf, ldsd, Mg, S1, S2);
        Mlast = Mg;
        if (!(Mg > -INFINITY)) { status = PPL_E_ZERO_WEIGHT; break; }
        if (!(S1 > 0.0) || isnan(S1) || isnan(S2)) { status = PPL_E_NONFINITE; break; }
        const double ess = S1 * S1 / S2;
        const bool res = (s < a.T - 1) && (ess < (double)a.ess_frac * (double)N);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (a.ess_trace) a.ess_trace[s] = ess;
            if (a.resampled) a.resampled[s] = res ? 1 : 0;
        }
        if (!res) continue;

        // ---- resampling: FP64 weights, normaliser, integer quantisation, scan
        uint64_t q[P];
        uint64_t run = 0;
        double esl = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const double e = valid[p] ? exp((double)lw[p] - (double)Mg) : 0.0;
            esl += e;
            run += (uint64_t)floor(ldexp(e, a.kbits));
            q[p] = run;
        }
        uint64_t btot;
        const uint64_t off = block_exclusive_scan_u64(run, ldsu, btot);
        const double eb = block_sum_f64(esl, ldsd);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (valid[p]) {
                a.qloc[base + p] = off + q[p];
#pragma unroll
                for (int f = 0; f < M::NF; ++f) a.xbuf[(size_t)f * N + base + p] = st[p][f];
            }
        }
        if (threadIdx.x == 0) {
            a.tot[blockIdx.x] = btot;
            a.esum[blockIdx.x] = eb;
        }
        if (!grid_barrier(a.bar, ++epoch * (unsigned)nb)) { alive = false; status = PPL_E_HIP; break; }

        // tile ends (inclusive prefix of tile totals) and the normaliser sum, same order everywhere
        uint64_t tv = 0;
        double ev = 0.0;
        for (int b0 = 0; b0 < nb; b0 += kSmcThreads) {
            const int b = b0 + threadIdx.x;
            const uint64_t v = b < nb ? a.tot[b] : 0;
            uint64_t chunk;
            const uint64_t ex = block_exclusive_scan_u64(v, ldsu, chunk);
            if (b < nb) tile_end[b] = tv + ex + v;
            tv += chunk;
            ev += block_sum_f64(b < nb ? a.esum[b] : 0.0, ldsd);
        }
        __syncthreads();
        const uint64_t S = tv;
        const uint4 rw = philox(0, 0, (uint32_t)s, (a.inst << 8) | kTagResample, a.key);
        const uint64_t U = __umul64hi(((uint64_t)rw.y << 32) | rw.x, S);
        logz += (double)Mg + log(ev) - logN;
        ++nres;

        // phase A (one loop body, not unrolled): ancestors of this thread's slots -> LDS
        int32_t *s_anc = (int32_t *)(tile_end + nb);
        int32_t *anc_row = (a.anc_out && nres - 1 < a.max_events) ? a.anc_out + (size_t)(nres - 1) * N : nullptr;
        int prev = -1;
#pragma unroll 1
        for (int p = 0; p < P; ++p) {
            const int j = (int)base + p;
            if (j >= N) break;
            const int anc = find_ancestor((uint32_t)j, S, U, (uint64_t)N, nb, kSmcThreads * P, tile_end, a.tot,
                                          a.qloc, prev);
            s_anc[threadIdx.x * P + p] = anc;
            if (anc_row) anc_row[j] = anc;
            prev = anc;
        }
        // phase B: gather the ancestors' state
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (!valid[p]) continue;
            const int anc = s_anc[threadIdx.x * P + p];
#pragma unroll
            for (int f = 0; f < M::NF; ++f) st[p][f] = a.xbuf[(size_t)f * N + anc];
            lw[p] = 0.0f;
        }
    }

    // ---- final normaliser (FP64) over the last epoch
    double ess_final = (double)N;
    if (alive && status == 0 && a.T > 0) {
        double e1 = 0.0, e2 = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (valid[p]) {
                const double e = exp((double)lw[p] - (double)Mlast);
                e1 += e;
                e2 += e * e;
            }
        }
        e1 = block_sum_f64(e1, ldsd);
        e2 = block_sum_f64(e2, ldsd);
        if (threadIdx.x == 0) {
            a.fin[2 * blockIdx.x] = e1;
            a.fin[2 * blockIdx.x + 1] = e2;
        }
        if (!grid_barrier(a.bar, ++epoch * (unsigned)nb)) {
            alive = false;
            status = PPL_E_HIP;
        } else {
            double t1 = 0.0, t2 = 0.0;
            for (int b0 = 0; b0 < nb; b0 += kSmcThreads) {
                const int b = b0 + threadIdx.x;
                t1 += block_sum_f64(b < nb ? a.fin[2 * b] : 0.0, ldsd);
                t2 += block_sum_f64(b < nb ? a.fin[2 * b + 1] : 0.0, ldsd);
            }
            logz += (double)Mlast + log(t1) - logN;
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

__global__ void smc_reset_kernel(unsigned *bar) {
    if (threadIdx.x < 2) bar[threadIdx.x] = 0u;
}

// ------------------------------------------------------------------ host --
static int pick_p(int64_t N) {
    // particles per thread so that one 1024-thread block per CU covers N (up to 8)
    const int64_t per_cu = (N + 255) / 256;
    int P = 1;
    while (P < 8 && (int64_t)kSmcThreads * P < per_cu) P <<= 1;
    return P;
}

static int64_t smc_blocks(int64_t N, int P) { return (N + (int64_t)kSmcThreads * P - 1) / ((int64_t)kSmcThreads * P); }

struct SmcLayout {
    double *scal;
    unsigned *bar;
    double *part, *esum, *fin;
    uint64_t *tot, *qloc;
    float *xbuf;
    size_t bytes;
};

static SmcLayout smc_layout(void *ws, int NF, int64_t N, int64_t nb) {
    SmcLayout L;
    char *p = (char *)ws;
    size_t o = 0;
    auto take = [&](size_t n) { char *r = p + o; o += align_up(n, 256); return r; };
    L.scal = (double *)take(8 * sizeof(double));
    L.bar = (unsigned *)take(2 * sizeof(unsigned));
    L.part = (double *)take(2 * nb * 3 * sizeof(double));
    L.esum = (double *)take(nb * sizeof(double));
    L.fin = (double *)take(2 * nb * sizeof(double));
    L.tot = (uint64_t *)take(nb * sizeof(uint64_t));
    L.qloc = (uint64_t *)take(N * sizeof(uint64_t));
    L.xbuf = (float *)take((size_t)NF * N * sizeof(float));
    L.bytes = o;
    return L;
}

size_t smc_ws_bytes(int model, int K, int64_t N) {
    const int NF = model == PPL_MODEL_LGSSM ? 1 : 2 * K;
    const int P = pick_p(N);
    return smc_layout(nullptr, NF, N, smc_blocks(N, P)).bytes;
}

double *smc_scalars_ptr(const SmcArgs &a) { return a.out.d_scalars ? a.out.d_scalars : (double *)a.ws; }

template <class M, int P>
static int launch(SmcDev &d, int64_t nb, hipStream_t st) {
    auto kern = smc_persistent_kernel<M, P>;
    int dev = 0, ncu = 0, occ = 0;
    PPL_HIP(hipGetDevice(&dev));
    PPL_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const size_t lds = (size_t)nb * sizeof(uint64_t) + (size_t)kSmcThreads * P * sizeof(int32_t);
    PPL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kSmcThreads, lds));
    if ((int64_t)occ * ncu < nb)
        return fail(PPL_E_UNSUPPORTED, "SMC needs %lld co-resident blocks, device holds %d", (long long)nb, occ * ncu);
    hipLaunchKernelGGL(smc_reset_kernel, dim3(1), dim3(64), 0, st, d.bar);
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
    if (nb > 4096) return fail(PPL_E_UNSUPPORTED, "SMC supports at most %lld particles", (long long)4096 * kSmcThreads * 8);
    if (a.T > 0x7fffffffLL) return fail(PPL_E_ARG, "too many factors");
    if ((a.T + 2) * 2 * nb >= 0xffffffffLL) return fail(PPL_E_UNSUPPORTED, "barrier counter would overflow");
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
    d.max_events = a.out.max_events;
    d.bar = L.bar;
    d.part = L.part;
    d.tot = L.tot;
    d.esum = L.esum;
    d.fin = L.fin;
    d.qloc = L.qloc;
    d.xbuf = L.xbuf;
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
