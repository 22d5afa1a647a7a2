// device.h -- device primitives shared by the libppl kernels (gfx950 only).
//
// Random stream: Philox4x32-10 as described by Salmon, Moraes, Dror and Shaw,
// "Parallel Random Numbers: As Easy as 1, 2, 3" (SC'11).  Counter words are
// (particle or slot index, block index, step, instance << 8 | tag); the key is
// the 64-bit seed split into two 32-bit words.  Sampling and scoring of the
// built-in distributions is what the paper's runtime library provides on each
// target (Sec. 4.2.3); here it is a set of inline device functions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ppl.h"

namespace ppl {

// Philox S-box multipliers and Weyl key increments (SC'11).
constexpr uint32_t kPhiloxMulA = 0xD2511F53u;
constexpr uint32_t kPhiloxMulB = 0xCD9E8D57u;
constexpr uint32_t kPhiloxWeylA = 0x9E3779B9u;
constexpr uint32_t kPhiloxWeylB = 0xBB67AE85u;

enum : uint32_t { kTagPrior = 0, kTagProposal = 1, kTagResample = 2, kTagMove = 7 };

// Compensated (Kahan) FP32 accumulation: sum += v with the running rounding
// error kept in c.  The error of the sum stays near 2 ulp of sum |v| however
// many terms are added, where a plain FP32 running sum loses up to a
// relative L 2^-24 over L terms (the SMC log-weights add one term per factor
// for as long as an epoch lasts).
__device__ __forceinline__ void kahan_add(float &sum, float &c, float v) {
    const float y = v - c;
    const float t = sum + y;
    c = (t - sum) - y;
    sum = t;
}

struct Key {
    uint32_t k0, k1;
};

__host__ __device__ inline Key make_key(uint64_t seed) { return Key{(uint32_t)seed, (uint32_t)(seed >> 32)}; }

// Ten Philox rounds on one 128-bit counter block.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, Key key) {
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kPhiloxWeylA;
            k1 += kPhiloxWeylB;
        }
        const uint32_t hi_a = __umulhi(kPhiloxMulA, c0), lo_a = kPhiloxMulA * c0;
        const uint32_t hi_b = __umulhi(kPhiloxMulB, c2), lo_b = kPhiloxMulB * c2;
        const uint32_t n0 = hi_b ^ c1 ^ k0;
        const uint32_t n2 = hi_a ^ c3 ^ k1;
        c0 = n0;
        c1 = lo_b;
        c2 = n2;
        c3 = lo_a;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Uniform on (0,1) from one word: the 23 high bits plus one half, times 2^-23.
// Every step is exact in FP32, so both precisions see the same value.
__device__ __forceinline__ float unit_f32(uint32_t w) { return ((float)(w >> 9) + 0.5f) * 0x1p-23f; }

// Uniform on (0,1) from two words (lo first): 52 bits plus one half, times 2^-52.
__device__ __forceinline__ double unit_f64(uint32_t lo, uint32_t hi) {
    const uint64_t v = ((uint64_t)hi << 32) | lo;
    return ((double)(v >> 12) + 0.5) * 0x1p-52;
}

// Box-Muller pair: radius sqrt(-2 ln u1), angle 2 pi u2 (sincospi avoids rounding 2 pi).
__device__ __forceinline__ void box_muller(float u1, float u2, float &z0, float &z1) {
    const float r = sqrtf(-2.0f * logf(u1));
    float s, c;
    sincospif(2.0f * u2, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

__device__ __forceinline__ void box_muller(double u1, double u2, double &z0, double &z1) {
    const double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// Four standard normals from one Philox block (two single-precision pairs).
__device__ __forceinline__ void normals4(uint4 w, float z[4]) {
    box_muller(unit_f32(w.x), unit_f32(w.y), z[0], z[1]);
    box_muller(unit_f32(w.z), unit_f32(w.w), z[2], z[3]);
}

// Uniform-discrete on {lo .. lo + range - 1}: lo + floor(w * range / 2^32).
__device__ __forceinline__ int uniform_discrete(uint32_t w, int lo, uint32_t range) {
    return lo + (int)__umulhi(w, range);
}

// ------------------------------------------------------- wave reductions --
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
// Wave-wide FP32 reductions through DPP row operations (full-rate VALU
// moves, no LDS permute): two quad permutations, the half-row and row
// mirrors, then the row-15 and row-31 broadcasts (rows left out of a
// broadcast keep the identity), which leave the total in lane 63; one
// v_readlane returns it to every lane.  All 64 lanes must be active.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f32(float v, float identity) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, identity),
                                                                 __builtin_bit_cast(int, v), CTRL, ROWS, 0xF, false));
}
__device__ __forceinline__ float wave_max_dpp(float v) {
    const float id = -INFINITY;
    v = fmaxf(v, dpp_f32<0xB1, 0xF>(v, id));    // quad_perm [1,0,3,2]
    v = fmaxf(v, dpp_f32<0x4E, 0xF>(v, id));    // quad_perm [2,3,0,1]
    v = fmaxf(v, dpp_f32<0x141, 0xF>(v, id));   // row_half_mirror
    v = fmaxf(v, dpp_f32<0x140, 0xF>(v, id));   // row_mirror
    v = fmaxf(v, dpp_f32<0x142, 0xA>(v, id));   // row_bcast15 into rows 1, 3
    v = fmaxf(v, dpp_f32<0x143, 0xC>(v, id));   // row_bcast31 into rows 2, 3
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ float wave_sum_dpp(float v) {
    v += dpp_f32<0xB1, 0xF>(v, 0.0f);
    v += dpp_f32<0x4E, 0xF>(v, 0.0f);
    v += dpp_f32<0x141, 0xF>(v, 0.0f);
    v += dpp_f32<0x140, 0xF>(v, 0.0f);
    v += dpp_f32<0x142, 0xA>(v, 0.0f);
    v += dpp_f32<0x143, 0xC>(v, 0.0f);
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
// FP64 sum with the same DPP steps: both 32-bit halves move with the same
// pattern and the add is FP64.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWS, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_f64<0xB1, 0xF>(v);
    v += dpp_f64<0x4E, 0xF>(v);
    v += dpp_f64<0x141, 0xF>(v);
    v += dpp_f64<0x140, 0xF>(v);
    v += dpp_f64<0x142, 0xA>(v);
    v += dpp_f64<0x143, 0xC>(v);
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

// ------------------------------------------- weighted-sum partial records --
// A partial over a set of particles: {m = max lw, s1 = sum e, s2 = sum e^2,
// nan = number of NaN log-weights, f[k] = sum e * f_k}, with e = exp(lw - m).
// Partials merge by rescaling their sums to the largest maximum.
template <int NF>
struct Partial {
    double m, s1, s2, nan;
    double f[NF];
};

template <int NF>
__device__ __forceinline__ Partial<NF> partial_load(const double *src) {
    Partial<NF> p;
    p.m = src[0];
    p.s1 = src[1];
    p.s2 = src[2];
    p.nan = src[3];
#pragma unroll
    for (int k = 0; k < NF; ++k) p.f[k] = src[4 + k];
    return p;
}

template <int NF>
__device__ __forceinline__ Partial<NF> partial_empty() {
    Partial<NF> p;
    p.m = -INFINITY;
    p.s1 = 0.0;
    p.s2 = 0.0;
    p.nan = 0.0;
#pragma unroll
    for (int k = 0; k < NF; ++k) p.f[k] = 0.0;
    return p;
}

// Reduce-scatter of F doubles across the 64 lanes of a wave by recursive
// halving.  At each level a lane and its partner (lane ^ O) hold the same N
// slots; the lane with bit O clear keeps the first ceil(N/2) slots, the other
// the last ceil(N/2) (for odd N both keep the middle one), and each adds the
// partner's copy of what it keeps.  Every add is a + b on one side and b + a on
// the other, so a slot held by several lanes holds bitwise the same total.
// A level costs ceil(N/2) shuffles instead of N, about 2F shuffles in all
// instead of 6F for a butterfly.  On return slot j of the lane holds the
// wave total of field lo + j (j < the final slot count).
template <int F, int N, int O>
struct WaveReduceScatter {
    static constexpr int kFinal = WaveReduceScatter<F, N - N / 2, O / 2>::kFinal;
    __device__ __forceinline__ static void run(double (&v)[F], int lane, int &lo) {
        constexpr int H = N / 2, C = N - H;
        const bool up = (lane & O) != 0;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const double keep = up ? v[H + j] : v[j];
            const double send = up ? v[j] : v[H + j];
            v[j] = keep + __shfl_xor(send, O, 64);
        }
        if (up) lo += H;
        WaveReduceScatter<F, C, O / 2>::run(v, lane, lo);
    }
};
template <int F, int N>
struct WaveReduceScatter<F, N, 0> {
    static constexpr int kFinal = N;
    __device__ __forceinline__ static void run(double (&)[F], int, int &) {}
};

// Block-wide maximum of one double per thread; every thread receives it.
template <int NWAVES>
__device__ __forceinline__ double block_max_f64(double v) {
    __shared__ double lds_m[NWAVES];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) lds_m[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = lds_m[0];
#pragma unroll
    for (int w = 1; w < NWAVES; ++w) m = fmax(m, lds_m[w]);
    return m;
}

// Sum of F doubles per thread across the block (blockDim = 64 * NWAVES):
// a reduce-scatter within each wave, then a fixed-order sum over the waves;
// dst[t] receives the total of field t.  Called at most once per kernel.
template <int F, int NWAVES>
__device__ __forceinline__ void block_sum_store(double (&v)[F], double *dst) {
    __shared__ double lds[NWAVES][F];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int lo = 0;
    WaveReduceScatter<F, F, 32>::run(v, lane, lo);
#pragma unroll
    for (int j = 0; j < WaveReduceScatter<F, F, 32>::kFinal; ++j)
        if (lo + j < F) lds[wv][lo + j] = v[j];
    __syncthreads();
    for (int t = threadIdx.x; t < F; t += 64 * NWAVES) {
        double s = lds[0][t];
#pragma unroll
        for (int w = 1; w < NWAVES; ++w) s += lds[w][t];
        dst[t] = s;
    }
}

// Block-level reduction of per-thread partials (blockDim = 64 * nwaves) into
// one record at dst.  The block maximum M comes first; each thread rescales
// its sums to M (one exp), and the sums then reduce with plain adds: a
// reduce-scatter within each wave and a fixed-order sum over the waves.  The
// result does not depend on timing.
template <int NF, int NWAVES>
__device__ __forceinline__ void partial_block_reduce_store(Partial<NF> &p, double *dst) {
    constexpr int F = 3 + NF;  // s1, s2, nan, f[NF]
    const double M = block_max_f64<NWAVES>(p.m);
    const double c = (p.m > -INFINITY) ? exp(p.m - M) : 0.0;
    double v[F];
    v[0] = p.s1 * c;
    v[1] = p.s2 * (c * c);
    v[2] = p.nan;
#pragma unroll
    for (int k = 0; k < NF; ++k) v[3 + k] = p.f[k] * c;
    block_sum_store<F, NWAVES>(v, dst + 1);
    if (threadIdx.x == 0) dst[0] = M;
}

// Block-level merge of the records in[r], r in [lo, hi), each {m, s1, s2, nan,
// f[NF]}, into one record at dst.  A first pass takes the maximum M of the
// record maxima; a second scales each record to M (one exp per record) and
// sums with plain adds.  Called at most once per kernel.
template <int NF, int NWAVES>
__device__ __forceinline__ void records_block_reduce_store(const double *__restrict__ in, int64_t lo, int64_t hi,
                                                           double *dst) {
    constexpr int F = 3 + NF;
    constexpr int R = 4 + NF;
    double m = -INFINITY;
    for (int64_t r = lo + threadIdx.x; r < hi; r += 64 * NWAVES) m = fmax(m, in[(size_t)r * R]);
    const double M = block_max_f64<NWAVES>(m);
    double v[F];
#pragma unroll
    for (int k = 0; k < F; ++k) v[k] = 0.0;
    for (int64_t r = lo + threadIdx.x; r < hi; r += 64 * NWAVES) {
        const double *rec = in + (size_t)r * R;
        const double mr = rec[0];
        v[2] += rec[3];
        if (mr > -INFINITY) {
            const double c = exp(mr - M);
            v[0] += rec[1] * c;
            v[1] += rec[2] * (c * c);
#pragma unroll
            for (int k = 0; k < NF; ++k) v[3 + k] += rec[4 + k] * c;
        }
    }
    block_sum_store<F, NWAVES>(v, dst + 1);
    if (threadIdx.x == 0) dst[0] = M;
}

// ------------------------------------------------ two-level partial merge --
// Up to kMergeDirect block partials are merged by the one workgroup of the
// finalize kernel; beyond that a first pass of at most kMergeGroups workgroups
// merges fixed contiguous ranges (a fixed order, so the result does not depend
// on timing) and the finalize workgroup merges those records.
constexpr int kMergeGroups = 512;
constexpr int64_t kMergeDirect = 2048;
constexpr int kFinalizeThreads = 256;

template <int NF>
__global__ __launch_bounds__(256) void partial_merge_kernel(const double *__restrict__ in, int64_t n, int64_t per,
                                                            double *__restrict__ out) {
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    records_block_reduce_store<NF, 4>(in, lo, hi, out + (size_t)blockIdx.x * (4 + NF));
}

// Bytes of second-level records a merge of NF-field partials may need.
inline size_t merge_scratch_bytes(int nf) { return (size_t)kMergeGroups * (4 + nf) * sizeof(double); }

// Runs the first pass when nblocks is large; returns the records the final
// wave merges and their count in *nrec.  scratch holds merge_scratch_bytes(NF).
template <int NF>
inline const double *merge_partials_first(const double *part, int64_t nblocks, double *scratch, int *nrec,
                                          hipStream_t st) {
    if (nblocks <= kMergeDirect) {
        *nrec = (int)nblocks;
        return part;
    }
    const int64_t per = (nblocks + kMergeGroups - 1) / kMergeGroups;
    const int groups = (int)((nblocks + per - 1) / per);
    hipLaunchKernelGGL(partial_merge_kernel<NF>, dim3(groups), dim3(256), 0, st, part, nblocks, per, scratch);
    *nrec = groups;
    return scratch;
}


// ------------------------------------------------ importance finalize --
// One workgroup merges the block partials and writes scalars[8] = {log Z-hat,
// ESS, 0, status, M, s1, s2, N} and the model summaries: for the polynomial
// model P(n | y) for n = 2..5, coefficient means per degree and overall
// (29 fields); for the others the weighted mean of each field.
template <int NF>
__global__ __launch_bounds__(kFinalizeThreads) void weights_finalize_kernel(const double *__restrict__ part,
                                                                          int nrec, int64_t N, int model,
                                                                          double *__restrict__ scalars,
                                                                          double *__restrict__ summaries) {
    __shared__ double rec[4 + NF];
    records_block_reduce_store<NF, kFinalizeThreads / 64>(part, 0, nrec, rec);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const Partial<NF> a = partial_load<NF>(rec);
    int status = 0;
    if (a.nan > 0) status = PPL_E_NONFINITE;
    else if (!(a.m > -INFINITY)) status = PPL_E_ZERO_WEIGHT;
    scalars[0] = status ? (a.nan > 0 ? NAN : -INFINITY) : a.m + log(a.s1) - log((double)N);
    scalars[1] = status ? 0.0 : a.s1 * a.s1 / a.s2;
    scalars[2] = 0.0;
    scalars[3] = (double)status;
    scalars[4] = a.m;
    scalars[5] = a.s1;
    scalars[6] = a.s2;
    scalars[7] = (double)N;
    if (!summaries) return;
    if constexpr (NF == 29) {
        if (model == PPL_MODEL_POLY) {
            for (int s = 0; s < 4; ++s) {
                const double mass = a.f[s];
                summaries[s] = status ? 0.0 : mass / a.s1;
                for (int j = 0; j < 5; ++j)
                    summaries[4 + 5 * s + j] = (!status && mass > 0) ? a.f[4 + 5 * s + j] / mass : 0.0;
            }
            for (int j = 0; j < 5; ++j) summaries[24 + j] = status ? 0.0 : a.f[24 + j] / a.s1;
            return;
        }
    }
    for (int k = 0; k < NF; ++k) summaries[k] = status ? 0.0 : a.f[k] / a.s1;
}

}  // namespace ppl
