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

namespace ppl {

// Philox S-box multipliers and Weyl key increments (SC'11).
constexpr uint32_t kPhiloxMulA = 0xD2511F53u;
constexpr uint32_t kPhiloxMulB = 0xCD9E8D57u;
constexpr uint32_t kPhiloxWeylA = 0x9E3779B9u;
constexpr uint32_t kPhiloxWeylB = 0xBB67AE85u;

enum : uint32_t { kTagPrior = 0, kTagProposal = 1, kTagResample = 2 };

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
__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

// ------------------------------------------- weighted-sum partial records --
// A partial over a set of particles: {m = max lw, s1 = sum e, s2 = sum e^2,
// nan = number of NaN log-weights, f[k] = sum e * f_k}, with e = exp(lw - m).
// Two partials merge by rescaling to the larger maximum.
template <int NF>
struct Partial {
    double m, s1, s2, nan;
    double f[NF];
};

template <int NF>
__device__ __forceinline__ void partial_merge(Partial<NF> &a, const Partial<NF> &b) {
    a.nan += b.nan;
    if (!(b.m > -INFINITY)) return;
    if (!(a.m > -INFINITY)) {
        a.m = b.m;
        a.s1 = b.s1;
        a.s2 = b.s2;
#pragma unroll
        for (int k = 0; k < NF; ++k) a.f[k] = b.f[k];
        return;
    }
    const double M = fmax(a.m, b.m);
    const double ca = exp(a.m - M), cb = exp(b.m - M);
    a.s1 = a.s1 * ca + b.s1 * cb;
    a.s2 = a.s2 * (ca * ca) + b.s2 * (cb * cb);
#pragma unroll
    for (int k = 0; k < NF; ++k) a.f[k] = a.f[k] * ca + b.f[k] * cb;
    a.m = M;
}

template <int NF>
__device__ __forceinline__ Partial<NF> partial_shfl_xor(const Partial<NF> &p, int o) {
    Partial<NF> q;
    q.m = __shfl_xor(p.m, o, 64);
    q.s1 = __shfl_xor(p.s1, o, 64);
    q.s2 = __shfl_xor(p.s2, o, 64);
    q.nan = __shfl_xor(p.nan, o, 64);
#pragma unroll
    for (int k = 0; k < NF; ++k) q.f[k] = __shfl_xor(p.f[k], o, 64);
    return q;
}

// Reduce a partial across the 64 lanes of a wave (fixed butterfly order).
template <int NF>
__device__ __forceinline__ void partial_wave_reduce(Partial<NF> &p) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        Partial<NF> q = partial_shfl_xor(p, o);
        partial_merge(p, q);
    }
}

template <int NF>
__device__ __forceinline__ void partial_store(double *dst, const Partial<NF> &p) {
    dst[0] = p.m;
    dst[1] = p.s1;
    dst[2] = p.s2;
    dst[3] = p.nan;
#pragma unroll
    for (int k = 0; k < NF; ++k) dst[4 + k] = p.f[k];
}

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

// Block-level reduction of per-thread partials (blockDim = 64 * nwaves) into
// one record written to dst by thread 0.  LDS scratch: nwaves records.
template <int NF, int NWAVES>
__device__ __forceinline__ void partial_block_reduce_store(Partial<NF> &p, double *dst) {
    __shared__ double lds[NWAVES][4 + NF];
    partial_wave_reduce(p);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) partial_store(lds[wv], p);
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial<NF> a = partial_load<NF>(lds[0]);
#pragma unroll
        for (int w = 1; w < NWAVES; ++w) {
            Partial<NF> b = partial_load<NF>(lds[w]);
            partial_merge(a, b);
        }
        partial_store(dst, a);
    }
}

// ------------------------------------------------ two-level partial merge --
// Up to kMergeDirect block partials are merged by one wave; beyond that a first
// pass of at most kMergeGroups workgroups merges fixed contiguous ranges (a
// fixed order, so the result does not depend on timing) and the wave merges
// those records.
constexpr int kMergeGroups = 512;
constexpr int64_t kMergeDirect = 8192;

template <int NF>
__global__ __launch_bounds__(256) void partial_merge_kernel(const double *__restrict__ in, int64_t n, int64_t per,
                                                            double *__restrict__ out) {
    Partial<NF> a = partial_empty<NF>();
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    for (int64_t r = lo + threadIdx.x; r < hi; r += 256) {
        Partial<NF> q = partial_load<NF>(in + (size_t)r * (4 + NF));
        partial_merge(a, q);
    }
    partial_block_reduce_store<NF, 4>(a, out + (size_t)blockIdx.x * (4 + NF));
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

}  // namespace ppl
